"""Seeded QAOA angle batches.

``draw_angles(P, p, seed)`` draws gamma ~ U[0, pi] and then beta ~ U[0, pi/2], each of
shape [P, p], from one ``numpy.random.default_rng(seed)`` stream (gamma first).
"""
from __future__ import annotations

import numpy as np


def draw_angles(P: int, p: int, seed: int):
    rng = np.random.default_rng(seed)
    gamma = rng.uniform(0.0, np.pi, size=(P, p))
    beta = rng.uniform(0.0, np.pi / 2, size=(P, p))
    return gamma, beta
