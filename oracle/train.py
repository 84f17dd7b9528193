"""Adam ascent of the FP64 oracle energy over a batch of starting angles.

TEST INFRASTRUCTURE ONLY (see the package header).  The same update rule as the
library's trainer, written out in numpy with the oracle's forward-mode gradient, so that
GPU and oracle trajectories can be compared step by step.
"""
import numpy as np

from .energy import energy, energy_grad


def adam_ascent(pl, gamma0, beta0, steps=100, lr=0.02, b1=0.9, b2=0.999, eps=1e-8):
    """pl: oracle.plan(...).  Returns (gamma, beta, E_final, history [steps, P])."""
    g = np.array(gamma0, dtype=np.float64, copy=True)
    b = np.array(beta0, dtype=np.float64, copy=True)
    mg, vg = np.zeros_like(g), np.zeros_like(g)
    mb, vb = np.zeros_like(b), np.zeros_like(b)
    hist = np.empty((steps, g.shape[0]))
    for t in range(1, steps + 1):
        E, dg, db, _ = energy_grad(pl, g, b)
        hist[t - 1] = E
        c1, c2 = 1.0 - b1 ** t, 1.0 - b2 ** t
        for x, d, m, v in ((g, dg, mg, vg), (b, db, mb, vb)):
            m *= b1
            m += (1.0 - b1) * d
            v *= b2
            v += (1.0 - b2) * d * d
            x += lr * (m / c1) / (np.sqrt(v / c2) + eps)
    Ef, _ = energy(pl, g, b)
    return g, b, Ef, hist
