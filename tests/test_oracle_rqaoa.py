"""Pins of the oracle's recursive QAOA (CPU).

* the substitution rule on a hand-checked example;
* bipartite graphs (even rings, K_{3,3}) end at their maximum cut (every edge cut) with
  p = 1 angles gamma = pi/4, beta = pi/8 (the ring's p = 1 optimum, where every edge has
  <Z_u Z_v> = -1/2), and every fixed pair respects the bipartition;
* on small random graphs the assignment is valid and its cut never exceeds the
  brute-force maximum.
"""
import itertools

import numpy as np

import oracle
import workloads as W

GA, BE = [np.pi / 4], [np.pi / 8]


def fixed(k, n):
    return GA, BE


def brute(n, edges):
    best = 0
    for z in itertools.product((1, -1), repeat=n):
        best = max(best, sum((1 - z[a] * z[b]) // 2 for a, b in edges))
    return best


def test_substitution_rule_by_hand():
    # path 0-1-2 plus edge 0-2 (a triangle) with zz strongest and negative on (1, 2):
    # z_2 = -z_1, so (0, 2) becomes (0, 1) with weight -1 and merges with (0, 1) -> 0:
    # nothing is left; the triangle's cut is 2 for any z with z_2 = -z_1.
    zl, cut, steps = oracle.rqaoa.rqaoa(3, [(0, 1), (0, 2), (1, 2)], None, 1, fixed, n_stop=2)
    assert steps[0][:2] in ((0, 1), (0, 2), (1, 2))
    assert cut == 2
    assert zl[steps[0][1]] == steps[0][2] * zl[steps[0][0]]


def test_bipartite_reach_max_cut():
    for g in (W.circulant(10, (1,)), W.circulant(14, (1,))):
        zl, cut, steps = oracle.rqaoa.rqaoa(g.n, g.edges.tolist(), None, 1, fixed, n_stop=4)
        assert cut == g.m, (g.name, cut)
        # even ring: z_v = s z_u must hold for the alternating colouring
        assert all(s == (-1) ** ((v - u) % 2) for u, v, s in steps)
    k33 = [(a, b) for a in range(3) for b in range(3, 6)]
    zl, cut, steps = oracle.rqaoa.rqaoa(6, k33, None, 1, fixed, n_stop=2)
    assert cut == 9


def test_random_graphs_valid_and_bounded():
    for seed in range(4):
        g = W.random_regular(12, 3, 40 + seed)
        zl, cut, steps = oracle.rqaoa.rqaoa(g.n, g.edges.tolist(), None, 1, fixed, n_stop=6)
        assert set(zl) <= {1, -1}
        direct = sum((1 - zl[a] * zl[b]) / 2 for a, b in g.edges.tolist())
        assert cut == direct
        assert cut <= brute(g.n, g.edges.tolist())
        assert len(steps) == g.n - 6
