"""Recursive QAOA on MaxCut: repeatedly fix the pair with the strongest correlation.

One step: evaluate <Z_u Z_v> of every edge (one light cone per orbit, broadcast to the
orbit's edges through the plan's edge -> orbit map), take the edge with the largest
|<Z_u Z_v>| (values within TIE of the largest count as ties, broken by the smallest edge
index, so that symmetric edges evaluated in different qubit orders cannot decide the
choice by rounding), impose z_v = s z_u with s its sign, and substitute:
every edge (v, x) of weight w becomes (u, x) of weight s w, merged with an existing (u, x)
(a zero sum drops the edge); the edge (u, v) itself becomes the constant w (1 - s) / 2 of
the cut.  When at most `n_stop` variables remain they are solved by enumeration.  The
cut of the weighted graph is C(z) = sum w_uv (1 - z_u z_v) / 2 (Sec. 2.4, weights as in
Sec. 4); the correlations come from the QAOA state of the current graph (Sec. 2.2, 2.3).

Symmetry after a step: a generator is kept if it still maps the live nodes onto themselves
and the weighted edge set onto itself (a subgroup of the stabiliser of the fixed pair).
"""
from __future__ import annotations

import numpy as np

TIE = 1e-6


def eliminate(edges: np.ndarray, weights: np.ndarray, zz: np.ndarray):
    """One elimination.  edges [m, 2] (u < v), weights [m], zz [m].  Returns
    (u, v, s, edges', weights', constant); node v has no edge left."""
    a = np.abs(zz)
    e = int(np.flatnonzero(a >= a.max() - TIE)[0])
    u, v = int(edges[e, 0]), int(edges[e, 1])
    s = 1 if zz[e] >= 0 else -1
    const = float(weights[e]) * (1 - s) / 2
    acc = {}
    for (x, y), w in zip(edges.tolist(), weights.tolist()):
        if (x, y) == (u, v):
            continue
        if x == v:
            x, w = u, s * w
        elif y == v:
            y, w = u, s * w
        key = (min(x, y), max(x, y))
        acc[key] = acc.get(key, 0.0) + w
    keys = sorted(k for k, w in acc.items() if w != 0)
    ne = np.array(keys, dtype=np.int64).reshape(-1, 2)
    nw = np.array([acc[k] for k in keys], dtype=np.float64)
    return u, v, s, ne, nw, const


def cut_value(edges, weights, z) -> float:
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if len(edges) == 0:
        return 0.0
    return float(np.sum(np.asarray(weights) * (1 - z[edges[:, 0]] * z[edges[:, 1]]) / 2))


def brute_force(n: int, edges, weights):
    """Best z in {-1, +1}^n for the weighted cut (node n-1 fixed to +1; first best wins)."""
    best, arg = -np.inf, np.ones(n, np.int64)
    for x in range(1 << max(n - 1, 0)):
        z = 1 - 2 * ((x >> np.arange(n)) & 1)
        if n:
            z[n - 1] = 1
        c = cut_value(edges, weights, z)
        if c > best:
            best, arg = c, z.copy()
    return arg


def _is_automorphism(perm, edges, weights) -> bool:
    table = {(int(a), int(b)): w for (a, b), w in zip(edges.tolist(), weights.tolist())}
    for (a, b), w in table.items():
        x, y = int(perm[a]), int(perm[b])
        if table.get((min(x, y), max(x, y))) != w:
            return False
    return True


def run(n: int, edges, weights, p: int, angles, correlations, n_stop: int = 8, generators=None):
    """Recursive QAOA with a pluggable correlation source.

    angles(step, n_live) -> (gamma [p], beta [p]);
    correlations(n_live, edges, weights, generators, p, gamma, beta) -> <Z_u Z_v> per edge.
    Returns (z [n] in {-1, +1}, cut of the input graph, [(u, v, s), ...] in input ids)."""
    e0 = np.sort(np.asarray(edges, dtype=np.int64).reshape(-1, 2), axis=1)
    w0 = np.ones(len(e0)) if weights is None else np.asarray(weights, dtype=np.float64)
    edges_c, w_c = e0.copy(), w0.copy()
    gens = [] if generators is None else [np.asarray(g, np.int64) for g in np.asarray(generators).reshape(-1, n)]
    alive = np.ones(n, bool)
    steps, k = [], 0
    while alive.sum() > n_stop and len(edges_c):
        ids = np.flatnonzero(alive)
        remap = -np.ones(n, np.int64)
        remap[ids] = np.arange(len(ids))
        loc = remap[edges_c]
        keep = [remap[g[ids]] for g in gens if np.all(alive[g[ids]])]
        keep = [g for g in keep if _is_automorphism(g, loc, w_c)]
        ga, be = angles(k, len(ids))
        zz = correlations(len(ids), loc, w_c, np.array(keep) if keep else None, p, ga, be)
        u, v, s, ne, nw, _ = eliminate(loc, w_c, zz)
        U, V = int(ids[u]), int(ids[v])
        steps.append((U, V, s))
        alive[V] = False
        edges_c, w_c = (ids[ne] if len(ne) else ne), nw
        k += 1
    ids = np.flatnonzero(alive)
    remap = -np.ones(n, np.int64)
    remap[ids] = np.arange(len(ids))
    z = np.zeros(n, np.int64)
    z[ids] = brute_force(len(ids), remap[edges_c] if len(edges_c) else edges_c, w_c)
    for U, V, s in reversed(steps):
        z[V] = s * z[U]
    return z, cut_value(e0, w0, z), steps


def gpu_correlations(n, edges, weights, generators, p, gamma, beta):
    """<Z_u Z_v> of every edge from the library (one cone per orbit, broadcast by orbit)."""
    import torch

    from . import Plan
    unit = bool(np.all(weights == 1))
    pl = Plan(n, edges, p=p, weights=None if unit else weights, generators=generators)
    gt = torch.tensor(np.reshape(gamma, (1, p)), dtype=torch.float64, device="cuda")
    bt = torch.tensor(np.reshape(beta, (1, p)), dtype=torch.float64, device="cuda")
    _, zz = pl.energy(gt, bt, term_zz=True)
    out = zz[0].cpu().numpy()[pl.orbits()[0]]
    pl.close()
    return out


def rqaoa(n: int, edges, weights, p: int, angles, n_stop: int = 8, generators=None):
    """Recursive QAOA with correlations from the GPU (see run)."""
    return run(n, edges, weights, p, angles, gpu_correlations, n_stop, generators)
