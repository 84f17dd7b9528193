"""Orbit-weighted QAOA MaxCut energy, its gradient, and plain references (O3-O9).

Sec. 2.3, Eq. 4: by linearity E_p = sum_S f(S) <prod_{j in S} Z_j>, each term
evaluated separately on its reverse causal cone.  For MaxCut (Sec. 2.4)
    E = <H_MaxCut> = sum_(u,v) w_uv (1 - <Z_u Z_v>) / 2.
Sec. 3 (reduced-energy display, after Theorem 1): terms related by a symmetry have
equal expectation, so with classes S~_m and representatives s_m
    E = sum_m W_m (1 - <Z Z>_{s_m}) / 2,     W_m = sum_{e in S~_m} w_e.
(The paper's display drops the constant and the 1/2 of H_MaxCut; the energy returned
here is <H_MaxCut> itself, the quantity maximised in Sec. 2.2-2.3.)

``reduce=False`` evaluates every edge's cone (the plain light-cone sum).
``bruteforce_full`` simulates the whole n-qubit graph and returns
E = sum_x |psi_x|^2 C(x), the plain definition with no light cones at all.
"""
from __future__ import annotations

import numpy as np

from .cones import light_cone
from .orbits import edge_orbits
from .problem import ProblemError, adjacency, canonical_edges
from .statevector import cut_values, qaoa_state, zz_and_grad, zz_expectation


class ConeTooLarge(ProblemError):
    pass


def plan(n, edges, weights, generators, p, reduce=True, max_k=24):
    """Orbits and cones.  Returns a dict with edge_orbit, rep, size, W, cones."""
    if p < 1:
        raise ProblemError("p must be >= 1")
    u, v, w = canonical_edges(n, edges, weights)
    gens = generators if (reduce and generators is not None and np.size(generators)) else np.zeros((0, n))
    orbit, rep, size = edge_orbits(n, u, v, w, gens)
    W = np.zeros(len(rep))
    for e in range(len(u)):                       # W_m = sum of weights in the class
        W[orbit[e]] += w[e]
    adj = adjacency(n, u, v)
    cones = []
    for r in rep:
        nodes, ledges, ids = light_cone(adj, int(u[r]), int(v[r]), p)
        if len(nodes) > max_k:
            raise ConeTooLarge(f"cone of edge {r} has {len(nodes)} qubits")
        cones.append(dict(nodes=nodes, edges=ledges, weights=w[ids], k=len(nodes)))
    return dict(u=u, v=v, w=w, edge_orbit=orbit, rep=rep, size=size, W=W, cones=cones, p=p)


def _cone_cut(cone):
    return cut_values(cone["k"], cone["edges"], cone["weights"])


def energy(pl, gammas, betas):
    """Return (E [P], zz [P, M]) for angle batches of shape [P, p]."""
    gammas = np.atleast_2d(np.asarray(gammas, np.float64))
    betas = np.atleast_2d(np.asarray(betas, np.float64))
    P = gammas.shape[0]
    zz = np.zeros((P, len(pl["rep"])))
    for m, cone in enumerate(pl["cones"]):
        cut = _cone_cut(cone)
        for i in range(P):
            psi = qaoa_state(cone["k"], cut, gammas[i], betas[i])
            zz[i, m] = zz_expectation(psi, cone["k"])
    E = (pl["W"][None, :] * (1.0 - zz) / 2.0).sum(axis=1)
    return E, zz


def energy_grad(pl, gammas, betas):
    """Return (E [P], dE/dgamma [P, p], dE/dbeta [P, p], zz [P, M])."""
    gammas = np.atleast_2d(np.asarray(gammas, np.float64))
    betas = np.atleast_2d(np.asarray(betas, np.float64))
    P, p = gammas.shape
    M = len(pl["rep"])
    zz = np.zeros((P, M))
    dzz_g = np.zeros((P, M, p))
    dzz_b = np.zeros((P, M, p))
    for m, cone in enumerate(pl["cones"]):
        cut = _cone_cut(cone)
        for i in range(P):
            zz[i, m], dzz_g[i, m], dzz_b[i, m] = zz_and_grad(cone["k"], cut, gammas[i], betas[i])
    W = pl["W"]
    E = (W[None, :] * (1.0 - zz) / 2.0).sum(axis=1)
    dg = -0.5 * (W[None, :, None] * dzz_g).sum(axis=1)
    db = -0.5 * (W[None, :, None] * dzz_b).sum(axis=1)
    return E, dg, db, zz


def energy_fd(pl, gammas, betas, h=1e-6):
    """Central finite differences of ``energy`` (FP64), shape [P, p] each."""
    gammas = np.atleast_2d(np.asarray(gammas, np.float64))
    betas = np.atleast_2d(np.asarray(betas, np.float64))
    P, p = gammas.shape
    dg = np.zeros((P, p))
    db = np.zeros((P, p))
    for l in range(p):
        gp, gm = gammas.copy(), gammas.copy()
        gp[:, l] += h
        gm[:, l] -= h
        dg[:, l] = (energy(pl, gp, betas)[0] - energy(pl, gm, betas)[0]) / (2 * h)
        bp, bm = betas.copy(), betas.copy()
        bp[:, l] += h
        bm[:, l] -= h
        db[:, l] = (energy(pl, gammas, bp)[0] - energy(pl, gammas, bm)[0]) / (2 * h)
    return dg, db


def bruteforce_full(n, edges, weights, gammas, betas):
    """Whole-graph statevector (n <= 20).  Returns (E, zz per edge [m])."""
    if n > 20:
        raise ProblemError("brute force limited to n <= 20")
    u, v, w = canonical_edges(n, edges, weights)
    pairs = list(zip(u.tolist(), v.tolist()))
    cut = cut_values(n, pairs, w)
    psi = qaoa_state(n, cut, gammas, betas)
    prob = np.abs(psi) ** 2
    E = float(np.sum(prob * cut))
    zz = np.array([zz_expectation(psi, n, a, b) for a, b in pairs])
    return E, zz
