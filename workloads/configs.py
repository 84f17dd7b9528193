"""The synthetic workloads: graph families, depths, angle batches and seeds.

Each entry stands in for a part of the paper's benchmark (Sec. 5, Tables 1-2), whose
graph files are not available: random 3-regular graphs stand in for rnd-3-reg-*,
the torus for grid-w-2-100, hypercubes and circulants for the edge-transitive and
highly symmetric instances.

``workload(name)`` returns a list of ``(Graph, p)`` pairs and the angle batch.
"""
from __future__ import annotations

from .angles import draw_angles
from .graphs import circulant, hypercube, random_regular, torus2d

_C4_SIZES = [100, 150, 200, 300, 500, 700, 1000, 1500, 2000, 3000, 4000, 5000, 6000, 8000, 10000]
_C4_CIRC = [100, 150, 200, 300, 500, 700, 1000, 1500, 2000, 3000, 5000, 7000, 10000]


def _c4_graphs():
    out, s = [], 400
    for L in (32, 64, 100):
        out.append((torus2d(L), 2))
    out.append((hypercube(8), 1))
    out.append((hypercube(10), 1))
    for n in _C4_CIRC:
        out.append((circulant(n, (1, 2, 5)), 2))
    for i, n in enumerate(_C4_SIZES):
        out.append((random_regular(n, 3, s + i), 1 if i % 2 == 0 else 2))
    for i, n in enumerate(_C4_SIZES):
        out.append((random_regular(n, 4, s + 20 + i), 1))
    return out


def workload(name: str):
    """Return (list of (graph, p), gamma[P, p_max], beta[P, p_max])."""
    if name == "c1":   # n=16 random 3-regular, p=1, one angle point
        g, (ga, be) = random_regular(16, 3, 0), draw_angles(1, 1, 100)
        return [(g, 1)], ga, be
    if name == "c2i":  # C_10000(1,2), p=2, 256 points
        ga, be = draw_angles(256, 2, 201)
        return [(circulant(10000, (1, 2)), 2)], ga, be
    if name == "c2ii":  # random 3-regular n=10000, p=2, 256 points
        ga, be = draw_angles(256, 2, 201)
        return [(random_regular(10000, 3, 202), 2)], ga, be
    if name == "c3":   # random 3-regular n=1000, p=2, 64 points
        ga, be = draw_angles(64, 2, 300)
        return [(random_regular(1000, 3, 3), 2)], ga, be
    if name == "c4":   # 48 mixed graphs, 32 points (p<=2)
        ga, be = draw_angles(32, 2, 499)
        return _c4_graphs(), ga, be
    if name == "c5i":  # Q_12, p=1, 8 points
        ga, be = draw_angles(8, 1, 501)
        return [(hypercube(12), 1)], ga, be
    if name == "c5ii":  # random 3-regular n=200, p=3, 8 points
        ga, be = draw_angles(8, 3, 503)
        return [(random_regular(200, 3, 502), 3)], ga, be
    raise KeyError(name)
