"""Recursive QAOA on MaxCut, written out plainly from its definition, with correlations
from the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

One step: compute <Z_u Z_v> for every edge of the current weighted graph (every edge its
own light cone, no symmetry), choose the edge with the largest |<Z_u Z_v>| (values within
1e-6 of the largest are ties: first in sorted edge order), impose z_v = s z_u with s the sign of that correlation, and
rewrite the cut sum_{xy} w_xy (1 - z_x z_y) / 2 with z_v replaced: terms (v, y) turn into
(u, y) with weight s w, equal pairs are added, zero weights vanish, and the term (u, v)
becomes a constant.  Below the stopping size the remaining variables are enumerated.
"""
import itertools

import numpy as np

from .energy import energy, plan


def oracle_correlations(n, edges, weights, p, gamma, beta):
    unit = all(w == 1 for w in weights)
    pl = plan(n, np.asarray(edges), None if unit else np.asarray(weights, dtype=float), None, p,
              reduce=False, max_k=24)
    _, zz = energy(pl, np.reshape(gamma, (1, p)), np.reshape(beta, (1, p)))
    return [float(x) for x in zz[0]]


def _cut(terms, z):
    return sum(w * (1 - z[a] * z[b]) / 2 for (a, b), w in terms.items())


def rqaoa(n, edges, weights, p, angles, n_stop=8):
    """Returns (z as a list of +-1, cut of the input graph, [(u, v, s), ...])."""
    if weights is None:
        weights = [1.0] * len(edges)
    original = {(min(int(a), int(b)), max(int(a), int(b))): float(w) for (a, b), w in zip(edges, weights)}
    terms = dict(original)
    live = list(range(n))
    steps = []
    k = 0
    while len(live) > n_stop and terms:
        index = {x: i for i, x in enumerate(live)}
        keys = sorted(terms)
        local = [(index[a], index[b]) for a, b in keys]
        ga, be = angles(k, len(live))
        zz = oracle_correlations(len(live), local, [terms[e] for e in keys], p, ga, be)
        top = max(abs(x) for x in zz)
        best = min(i for i in range(len(keys)) if abs(zz[i]) >= top - 1e-6)
        u, v = keys[best]
        s = 1 if zz[best] >= 0 else -1
        steps.append((u, v, s))
        new = {}
        for (a, b), w in terms.items():
            if (a, b) == (u, v):
                continue
            a2, b2, w2 = a, b, w
            if a == v:
                a2, w2 = u, s * w
            if b == v:
                b2, w2 = u, s * w
            e = (min(a2, b2), max(a2, b2))
            new[e] = new.get(e, 0.0) + w2
        terms = {e: w for e, w in new.items() if w != 0}
        live.remove(v)
        k += 1
    # enumerate the rest: the last live node fixed to +1, first best assignment wins
    z = {}
    best_val, best_z = None, None
    free = live[:-1]
    for bits in itertools.product((1, -1), repeat=len(free)):
        zz_ = dict(zip(free, bits))
        if live:
            zz_[live[-1]] = 1
        val = _cut(terms, zz_)
        if best_val is None or val > best_val:
            best_val, best_z = val, zz_
    z.update(best_z or {})
    for u, v, s in reversed(steps):
        z[v] = s * z[u]
    zl = [z.get(i, 1) for i in range(n)]
    return zl, _cut(original, zl), steps
