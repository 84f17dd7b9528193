"""Multi-start training of QAOA angles: Adam ascent of E(gamma, beta) over a batch of
starting points, one batched energy + gradient call of the library per step.

The paper motivates the symmetry reduction by training: the same reduced light cones are
evaluated at many angle points (Sec. 1, Sec. 5 discussion of repeated evaluation), so the
plan is built once and reused for every step.  The update itself is a few element-wise
operations on [P, p] tensors; every energy and gradient comes from the HIP kernels.
"""
from __future__ import annotations


def adam_ascent(plan, gamma0, beta0, steps: int = 100, lr: float = 0.02, b1: float = 0.9, b2: float = 0.999,
                eps: float = 1e-8):
    """Maximise E over P independent starts.

    gamma0, beta0: [P, p] tensors on the GPU.  Returns (gamma, beta, E, history) with the
    final angles [P, p], their energies [P] and the energy before every step
    [steps, P].  Angles are updated in place in fixed buffers, so a plan built with
    graph=True replays one captured call per step.
    """
    import torch

    g = gamma0.detach().to(torch.float64).contiguous().clone()
    b = beta0.detach().to(torch.float64).contiguous().clone()
    if g.shape != b.shape or g.dim() != 2 or g.shape[1] != plan.p:
        raise ValueError("gamma0 and beta0 must both be [P, p]")
    P = g.shape[0]
    E = torch.empty(P, dtype=torch.float64, device=g.device)
    dg = torch.empty_like(g)
    db = torch.empty_like(b)
    mg, vg = torch.zeros_like(g), torch.zeros_like(g)
    mb, vb = torch.zeros_like(b), torch.zeros_like(b)
    hist = torch.empty((steps, P), dtype=torch.float64, device=g.device)
    for t in range(1, steps + 1):
        plan.energy_grad(g, b, out=(E, dg, db))
        hist[t - 1].copy_(E)
        c1, c2 = 1.0 - b1 ** t, 1.0 - b2 ** t
        for x, d, m, v in ((g, dg, mg, vg), (b, db, mb, vb)):
            m.mul_(b1).add_(d, alpha=1.0 - b1)
            v.mul_(b2).addcmul_(d, d, value=1.0 - b2)
            x.add_(lr * (m / c1) / ((v / c2).sqrt() + eps))
    Ef = plan.energy(g, b)
    return g, b, Ef, hist
