"""MaxCut problem input (oracle step O1).

The problem is a simple graph G=(V,E) (Sec. 2.4) with optional real edge weights
J_ij (Sec. 4, Eq. 6).  Edges are canonicalised to u < v; the input order is kept
as the edge index.  Self-loops, duplicate edges and out-of-range ids are rejected:
the MaxCut Hamiltonian of Sec. 2.4 is a sum over the edges of a simple graph.
"""
from __future__ import annotations

import numpy as np


class ProblemError(ValueError):
    pass


def canonical_edges(n: int, edges, weights=None):
    """Return (u, v, w): int64 [m], int64 [m], float64 [m] with u < v.

    ``weights=None`` means unit weights.
    """
    if int(n) < 1:
        raise ProblemError("n_nodes must be >= 1")
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    m = e.shape[0]
    if m and (e.min() < 0 or e.max() >= n):
        raise ProblemError("edge endpoint out of range")
    u = np.minimum(e[:, 0], e[:, 1])
    v = np.maximum(e[:, 0], e[:, 1])
    if np.any(u == v):
        raise ProblemError("self-loop")
    seen = set()
    for a, b in zip(u.tolist(), v.tolist()):
        if (a, b) in seen:
            raise ProblemError("duplicate edge")
        seen.add((a, b))
    if weights is None:
        w = np.ones(m, dtype=np.float64)
    else:
        w = np.asarray(weights, dtype=np.float64).reshape(-1)
        if w.shape[0] != m:
            raise ProblemError("weights length mismatch")
        if not np.all(np.isfinite(w)):
            raise ProblemError("non-finite weight")
    return u, v, w


def adjacency(n: int, u, v):
    """Neighbour lists with the edge index of each incidence."""
    adj = [[] for _ in range(n)]
    for i, (a, b) in enumerate(zip(u.tolist(), v.tolist())):
        adj[a].append((b, i))
        adj[b].append((a, i))
    return adj
