"""Edge orbits under a supplied group of automorphisms (oracle step O2).

Sec. 2.6 defines an automorphism as a node permutation sigma with
(sigma(u), sigma(v)) in E exactly when (u, v) in E.  For weighted problems (Sec. 4,
Eq. 6) symmetries must also keep J: a generator must map every edge to an edge of the
same weight (compared bit for bit here).

Sec. 3 (Theorem 1 and the reduced-energy display) needs the equivalence classes of
Hamiltonian terms under the group, with one representative per class ("arbitrarily
chosen" in the paper).  The reading taken: the representative is the smallest edge
index of its class and classes are numbered by ascending representative.

The classes are computed by explicit closure: starting from the smallest unassigned
edge, apply every generator to every newly reached edge until nothing new appears.
In a finite group the inverse of a generator is one of its powers, so the closure
under the generators alone is the orbit under the generated group.
"""
from __future__ import annotations

import numpy as np

from .problem import ProblemError


class NotAutomorphism(ProblemError):
    pass


def edge_orbits(n: int, u, v, w, generators):
    """Return (edge_orbit int64 [m], rep int64 [M], size int64 [M])."""
    m = len(u)
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(u, v))}
    wbits = np.asarray(w, np.float64).view(np.uint64)
    gens = [np.asarray(g, np.int64) for g in np.asarray(generators).reshape(-1, n)] if np.size(generators) else []
    for g in gens:
        if g.shape[0] != n or not np.array_equal(np.sort(g), np.arange(n)):
            raise NotAutomorphism("generator is not a permutation of the nodes")
        for i in range(m):
            a, b = int(g[u[i]]), int(g[v[i]])
            j = index.get((min(a, b), max(a, b)))
            if j is None:
                raise NotAutomorphism("generator maps an edge to a non-edge")
            if wbits[j] != wbits[i]:
                raise NotAutomorphism("generator does not preserve edge weights")
    orbit = np.full(m, -1, dtype=np.int64)
    reps = []
    for e in range(m):
        if orbit[e] >= 0:
            continue
        oid = len(reps)
        reps.append(e)
        orbit[e] = oid
        frontier = [e]
        while frontier:
            reached = []
            for f in frontier:
                for g in gens:
                    a, b = int(g[u[f]]), int(g[v[f]])
                    j = index[(min(a, b), max(a, b))]
                    if orbit[j] < 0:
                        orbit[j] = oid
                        reached.append(j)
            frontier = reached
    size = np.bincount(orbit, minlength=len(reps)).astype(np.int64) if m else np.zeros(0, np.int64)
    return orbit, np.asarray(reps, np.int64), size
