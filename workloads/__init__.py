"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and bench.py.

This package holds no part of the method's arithmetic: it only draws graphs, their
automorphism generators (known by construction for each family) and QAOA angles.
Both the oracle and the HIP path receive exactly the arrays produced here.
"""
from .graphs import (  # noqa: F401
    Graph,
    random_regular,
    circulant,
    torus2d,
    torus3d,
    hypercube,
    complete,
    rook,
    paley,
    triangle,
    single_edge,
    star,
    spider_pair,
    relabel,
    degree_root_weights,
)
from .angles import draw_angles  # noqa: F401
from .configs import workload  # noqa: F401
