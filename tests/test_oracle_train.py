"""Pins of the oracle trainer: Adam ascent reaches known optima (p = 1, 2, 3).

* a single edge: <C> = (1 + sin 4beta sin gamma) / 2 (the closed form at p = 1), maximal
  value 1 at gamma = pi/2, beta = pi/8;
* the ring C_n (every vertex of degree 2, no triangles): the p = 1 optimum of the cut
  fraction is 3/4 (Farhi, Goldstone and Gutmann's ring result, which the closed form gives
  for d = 1, lambda = 0: max over (gamma, beta) of 1/2 + sin 4beta sin gamma cos gamma / 2).
"""
import numpy as np

import oracle
import workloads as W


def test_single_edge_reaches_one():
    g = W.single_edge()
    pl = oracle.plan(g.n, g.edges, None, None, 1, reduce=False)
    ga, be, E, hist = oracle.adam_ascent(pl, [[1.0], [2.5]], [[0.3], [1.2]], steps=400, lr=0.02)
    assert np.all(E > 1 - 1e-6), E
    assert np.all(hist[-1] > hist[0])
    # the maximiser: sin 4beta sin gamma = 1
    assert np.allclose(np.sin(4 * be[:, 0]) * np.sin(ga[:, 0]), 1.0, atol=1e-5)


def test_ring_reaches_three_quarters():
    g = W.circulant(12, (1,))
    pl = oracle.plan(g.n, g.edges, None, g.gens(), 1, reduce=True)
    ga, be, E, hist = oracle.adam_ascent(pl, [[0.5]], [[0.2]], steps=600, lr=0.01)
    assert abs(E[0] / g.m - 0.75) < 1e-6, E[0] / g.m
    # the closed form at that point agrees
    zz = oracle.zz_p1(g.n, g.edges, None, 0, 1, ga[0, 0], be[0, 0])
    assert abs((1 - zz) / 2 - 0.75) < 1e-6


def test_ring_p2_reaches_five_sixths():
    # The ring at depth 2: every edge's cone is a path of six vertices, and the optimum cut
    # fraction is 5/6 (Farhi, Goldstone and Gutmann's ring values (2p + 1) / (2p + 2)).  The
    # value is fixed independently of this code; reaching it exercises the layer loop of
    # both the forward-mode gradient (the trajectory) and the plain statevector (the
    # returned energy), at p >= 2 where the closed form does not apply.
    g = W.circulant(12, (1,))
    pl = oracle.plan(g.n, g.edges, None, g.gens(), 2, reduce=True)
    assert [c["k"] for c in pl["cones"]] == [6]
    ga, be, E, hist = oracle.adam_ascent(pl, [[0.5, 0.8], [0.3, 0.6]], [[0.4, 0.2], [0.5, 0.3]], steps=800,
                                         lr=0.01)
    assert np.abs(E / g.m - 5 / 6).max() < 1e-7, E / g.m
    # and on the full ring state, without light cones
    Eb, _ = oracle.bruteforce_full(g.n, g.edges, None, ga[0], be[0])
    assert abs(Eb / g.m - 5 / 6) < 1e-7


def test_ring_p3_reaches_seven_eighths():
    g = W.circulant(16, (1,))
    pl = oracle.plan(g.n, g.edges, None, g.gens(), 3, reduce=True)
    assert [c["k"] for c in pl["cones"]] == [8]
    _, _, E, _ = oracle.adam_ascent(pl, [[0.4, 0.8, 1.1]], [[0.5, 0.4, 0.2]], steps=1500, lr=0.01)
    assert abs(E[0] / g.m - 7 / 8) < 1e-6, E / g.m
