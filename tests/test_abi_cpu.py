"""C ABI and host planner (CPU only): exports, orbits and cones against the oracle.

The planner (union-find orbits, BFS cones) must agree with the oracle (closure orbits,
its own cone extraction) bit for bit: orbit ids, representatives, sizes, cone node order
and induced-edge counts.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2101_10296_amd as Q
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "qaoa.h")).read()
    names = set(re.findall(r"^\s*(?:qaoa_status|void|const char\*)\s+(qaoa_\w+)\s*\(", hdr, re.M))
    assert {"qaoa_plan_lightcones", "qaoa_energy", "qaoa_energy_grad", "qaoa_plan_query", "qaoa_plan_orbits",
            "qaoa_plan_destroy", "qaoa_last_error", "qaoa_plan_cone", "qaoa_plan_opts_default"} <= names
    lib = ctypes.CDLL(Q.library_path())
    for n in names:
        assert hasattr(lib, n), n


def _oracle_plan(g, p, reduce=True, w=None):
    return oracle.plan(g.n, g.edges, w, g.gens() if reduce else None, p, reduce=reduce, max_k=40)


PLANNER_CASES = [
    ("C40(1,2)", lambda: W.circulant(40, (1, 2)), 2),
    ("C60(1,2,5)", lambda: W.circulant(60, (1, 2, 5)), 1),
    ("torus7", lambda: W.torus2d(7), 2),
    ("Q5", lambda: W.hypercube(5), 1),
    ("rand3-100", lambda: W.random_regular(100, 3, 5), 2),
    ("rand4-60", lambda: W.random_regular(60, 4, 6), 1),
    ("K6", lambda: W.complete(6), 1),
    ("paley13", lambda: W.paley(13), 1),
    ("torus3d-4", lambda: W.torus3d(4), 1),
    ("rook5", lambda: W.rook(5), 1),
    # 4500 orbits: enough for the planner to split the cones over threads
    ("rand3-3000", lambda: W.random_regular(3000, 3, 7), 2),
]


@pytest.mark.parametrize("name,make,p", PLANNER_CASES, ids=[c[0] for c in PLANNER_CASES])
@pytest.mark.parametrize("reduce", [True, False])
def test_planner_matches_oracle_bit_exactly(name, make, p, reduce):
    g = make()
    pl = Q.Plan(g.n, g.edges, p=p, generators=g.gens(), reduce=reduce)
    ref = _oracle_plan(g, p, reduce)
    eo, rep, size = pl.orbits()
    assert np.array_equal(eo, ref["edge_orbit"])
    assert np.array_equal(rep, ref["rep"])
    assert np.array_equal(size, ref["size"])
    info = pl.info()
    assert info["n_orbits"] == len(ref["rep"])
    hist = np.bincount([c["k"] for c in ref["cones"]], minlength=31)
    assert list(hist[:31]) == info["k_hist"]
    for m, cone in enumerate(ref["cones"]):
        k, nodes, ne = pl.cone(m)
        assert k == cone["k"] and list(nodes) == list(cone["nodes"]) and ne == len(cone["edges"])
    assert abs(info["total_weight"] - g.m) < 1e-12


def test_planner_orbits_on_paper_table_graphs():
    # N_orb printed in the paper's Table 2 for grid-w-2-100 and paley-461 (both 1)
    for g in (W.torus2d(100), W.paley(461)):
        pl = Q.Plan(g.n, g.edges, p=1, generators=g.gens(), max_cone_qubits=30) if g.name != "paley461" else None
        if pl is None:
            # the Paley graph's p=1 cone exceeds 30 qubits: orbits are still checked through
            # the error path below, which happens after the orbits are formed
            with pytest.raises(Q.QaoaError) as ei:
                Q.Plan(g.n, g.edges, p=1, generators=g.gens())
            assert ei.value.status == Q.QAOA_ECONE
            continue
        assert pl.info()["n_orbits"] == 1


def test_weighted_planner_and_weight_preservation():
    g = W.circulant(12, (1, 2))
    w = np.array([1.0 if abs(int(b) - int(a)) in (1, 11) else 2.0 for a, b in g.edges])
    pl = Q.Plan(g.n, g.edges, p=1, weights=w, generators=g.gens())
    ref = oracle.plan(g.n, g.edges, w, g.gens(), 1)
    eo, rep, size = pl.orbits()
    assert np.array_equal(eo, ref["edge_orbit"]) and len(rep) == 2
    info = pl.info()
    assert info["cut_max"] == int(max(sum(c["weights"]) for c in ref["cones"]))
    w2 = w.copy()
    w2[0] = 3.0
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan(g.n, g.edges, p=1, weights=w2, generators=g.gens())
    assert ei.value.status == Q.QAOA_ENOTAUT


@pytest.mark.parametrize("bad,status", [
    (dict(edges=[[0, 0]], n=3), Q.QAOA_EINVAL),
    (dict(edges=[[0, 1], [1, 0]], n=3), Q.QAOA_EINVAL),
    (dict(edges=[[0, 5]], n=3), Q.QAOA_EINVAL),
    (dict(edges=[[0, 1]], n=3, p=0), Q.QAOA_EINVAL),
    (dict(edges=[[0, 1], [1, 2]], n=3, weights=[1.0, float("inf")]), Q.QAOA_EINVAL),
    (dict(edges=[[0, 1], [1, 2]], n=3, weights=[1.0, float("nan")]), Q.QAOA_EINVAL),
    (dict(edges=[[0, 1], [1, 2]], n=3, generators=[[1, 0, 2]]), Q.QAOA_ENOTAUT),
    (dict(edges=[[0, 1], [1, 2]], n=3, generators=[[0, 0, 2]]), Q.QAOA_ENOTAUT),
    (dict(edges=W.complete(40).edges, n=40), Q.QAOA_ECONE),
])
def test_error_codes(bad, status):
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan(bad["n"], bad["edges"], p=bad.get("p", 1), weights=bad.get("weights"),
               generators=bad.get("generators"))
    assert ei.value.status == status
    assert len(str(ei.value)) > len("QAOA_EINVAL: ")


@pytest.mark.parametrize("opts", [dict(checkpoint_mode=3), dict(checkpoint_mode=-1), dict(k_lds_max=12), dict(k_lds_max=15),
                                  dict(max_cone_qubits=31), dict(mem_budget_bytes=-1),
                                  dict(graph=True, profile=True), dict(graph=True, one_cone_at_a_time=True)])
def test_option_errors(opts):
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan(3, [[0, 1], [1, 2]], p=1, **opts)
    assert ei.value.status == Q.QAOA_EINVAL


@pytest.mark.parametrize("w,unit", [([1.0, 2.0, 3.0], 1.0), ([0.5, 1.5, 1.0], 0.5), ([0.1, 0.3, 0.2], 0.1),
                                    ([0.25, -0.75, 1.0], 0.25), ([1 / 3, 2 / 3, 1.0], 1 / 3), ([2.0, 4.0, 6.0], 1.0)])
def test_weight_unit(w, unit):
    # weights are counted in their common unit: the largest delta with every w / delta an
    # integer (integer weights keep delta = 1)
    pl = Q.Plan(4, [[0, 1], [1, 2], [2, 3]], p=1, weights=w)
    info = pl.info()
    assert abs(info["weight_unit"] - unit) <= 1e-15 * max(1.0, unit)
    assert info["total_weight"] == pytest.approx(sum(w), rel=1e-15, abs=1e-15)


def test_real_weights():
    # weights without a common unit, or integer cut values spanning more than 255 units,
    # plan as real weights (phases from each amplitude's own cut value) for cones of at most
    # 14 qubits; a larger cone is refused
    g = W.rook(3)   # 3 x 3 rook graph, weight 30 per edge: cut values span more than 255
    for w in (np.full(g.m, 30.0), np.random.default_rng(1).normal(size=g.m)):
        info = Q.Plan(g.n, g.edges, p=1, weights=w).info()
        assert info["real_weights"] == 1 and info["weight_unit"] == 0.0
    c = W.circulant(40, (1, 2))
    d = (c.edges[:, 1] - c.edges[:, 0]) % c.n
    w = np.where(np.minimum(d, c.n - d) == 1, 1.0, 2 ** 0.5)
    pl = Q.Plan(c.n, c.edges, p=2, weights=w, generators=c.gens())
    assert pl.info()["real_weights"] == 1 and pl.info()["n_orbits"] == 2
    assert Q.Plan(c.n, c.edges, p=2, weights=np.where(w == 1.0, 1.0, 2.0)).info()["real_weights"] == 0
    s = W.star(15)   # one 16-qubit cone, held in device memory: real weights there too
    info = Q.Plan(s.n, s.edges, p=1, weights=np.full(s.m, 30.0)).info()
    assert info["real_weights"] == 1 and info["n_hbm_cones"] == s.m


def test_empty_and_isolated():
    pl = Q.Plan(5, np.zeros((0, 2), np.int64), p=2)
    assert pl.info()["n_orbits"] == 0
    pl = Q.Plan(6, [[0, 1], [3, 4]], p=3)
    assert pl.info()["k_hist"][2] == 2


def test_first_failing_cone_is_reported():
    # cones are extracted on several threads for large plans; the error must still name
    # the lowest failing orbit.  Random 3-regular, p = 2: every cone has more than 6 qubits
    # except those closed off by short cycles, so orbit 0 is the first to fail.
    g = W.random_regular(6000, 3, 11)
    ref = oracle.plan(g.n, g.edges, None, None, 2, reduce=True, max_k=40)
    first = next(m for m, c in enumerate(ref["cones"]) if c["k"] > 6)
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan(g.n, g.edges, p=2, max_cone_qubits=6)
    assert ei.value.status == Q.QAOA_ECONE
    assert f"light cone of orbit {first} " in str(ei.value)
    # weight 300 on one late edge makes the weights real (its cones' cut values span more
    # than 255 units); that is no error any more
    w = np.ones(g.m)
    w[g.m - 5] = 300.0
    assert Q.Plan(g.n, g.edges, p=1, weights=w).info()["real_weights"] == 1


def test_batch_plan_concatenates_instances():
    # a plan over three graphs: each instance's orbits, representatives and cones are those
    # of its own plan, numbered after the instances before it
    graphs = [(W.circulant(40, (1, 2)), True, None), (W.random_regular(30, 3, 4), False, None),
              (W.torus2d(5), True, np.full(50, 0.5))]
    inst = [(g.n, g.edges, w, g.gens() if red else None) for g, red, w in graphs]
    bp = Q.Plan.batch(inst, 2)
    info = bp.info()
    assert info["n_instances"] == 3 and bp.n_instances == 3
    assert info["weight_unit"] == 0.0   # units 1 and 1/2
    eo, rep, size = bp.orbits()
    n0 = e0 = o0 = 0
    for (g, red, w) in graphs:
        single = Q.Plan(g.n, g.edges, p=2, weights=w, generators=g.gens() if red else None)
        seo, srep, ssize = single.orbits()
        M = len(srep)
        np.testing.assert_array_equal(eo[e0:e0 + g.m], seo + o0)
        np.testing.assert_array_equal(rep[o0:o0 + M], srep + e0)
        np.testing.assert_array_equal(size[o0:o0 + M], ssize)
        for m in range(M):
            k, nodes, ne = bp.cone(o0 + m)
            ks, snodes, sne = single.cone(m)
            assert (k, ne) == (ks, sne) and np.array_equal(nodes, snodes + n0)
        n0, e0, o0 = n0 + g.n, e0 + g.m, o0 + M
    assert (info["n_nodes"], info["n_edges"], info["n_orbits"]) == (n0, e0, o0)


def test_batch_plan_errors_name_the_instance():
    g = W.circulant(12, (1,))
    bad = np.arange(g.n)[::-1].copy()
    bad[0], bad[1] = bad[1], bad[0]
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan.batch([(g.n, g.edges), (g.n, g.edges, None, bad[None, :])], 1)
    assert ei.value.status == Q.QAOA_ENOTAUT and "instance 1" in str(ei.value)
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan.batch([], 1)
    assert ei.value.status == Q.QAOA_EINVAL


def test_tune_range():
    # tune: 0 (off), 1 (timed choices), 2..5 (a fixed layout variant); anything else is refused
    import paper_2101_10296_amd as Q
    g = W.circulant(12, (1,))
    for t in (0, 1, 2, 5):
        Q.Plan(g.n, g.edges, p=2, tune=t).close()
    for t in (-1, 6):
        with pytest.raises(Exception, match="tune"):
            Q.Plan(g.n, g.edges, p=2, tune=t)
