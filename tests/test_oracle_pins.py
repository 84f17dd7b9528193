"""Pins that fix the FP64 oracle against the paper and the mathematics (CPU only).

Each pin is something other than the oracle's own formula: a closed form, the whole
graph simulated with no light cones, the paper's Theorem 1, invariances of the ansatz,
finite differences, brute-force automorphism groups, and the orbit counts printed in
the paper's Tables 1-2.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.automorphisms import automorphism_group, group_closure, orbits_under
from oracle.orbits import NotAutomorphism
from oracle.problem import ProblemError
from oracle.statevector import cut_values, qaoa_state
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _erdos(n, prob, seed, weighted=None):
    rng = np.random.default_rng(seed)
    a, b = np.triu_indices(n, 1)
    keep = rng.random(a.size) < prob
    e = np.stack([a[keep], b[keep]], 1)
    w = None
    if weighted == "int":
        w = rng.integers(1, 4, size=e.shape[0]).astype(float)
    elif weighted == "real":
        w = rng.uniform(-1.5, 1.5, size=e.shape[0])
    return e, w


# ---------------------------------------------------------------- p = 1 closed form
@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("weighted", [None, "int", "real"])
def test_closed_form_p1(seed, weighted):
    n = 9
    e, w = _erdos(n, 0.45, seed, weighted)
    rng = np.random.default_rng(1000 + seed)
    gamma, beta = rng.uniform(0, np.pi), rng.uniform(0, np.pi / 2)
    pl = oracle.plan(n, e, w, None, 1, reduce=False)
    _, zz = oracle.energy(pl, [[gamma]], [[beta]])
    ref = [oracle.zz_p1(n, e, w, int(a), int(b), gamma, beta) for a, b in e]
    np.testing.assert_allclose(zz[0], ref, atol=1e-12)


def test_single_edge_closed_form_and_optimum():
    # K_2: the cone is the edge itself; <ZZ> = -sin(4 beta) sin(gamma) (closed form with
    # no other neighbours), so E = (1 - <ZZ>)/2 reaches its maximum 1 at gamma = pi/2,
    # beta = pi/8.
    g = W.single_edge()
    pl = oracle.plan(g.n, g.edges, None, g.gens(), 1)
    rng = np.random.default_rng(7)
    for _ in range(5):
        ga, be = rng.uniform(-3, 3), rng.uniform(-3, 3)
        E, zz = oracle.energy(pl, [[ga]], [[be]])
        assert abs(zz[0, 0] + np.sin(4 * be) * np.sin(ga)) < 1e-14
    E, _ = oracle.energy(pl, [[np.pi / 2]], [[np.pi / 8]])
    assert abs(E[0] - 1.0) < 1e-14


# ------------------------------------------------- light cones vs whole-graph brute force
BRUTE_CASES = [
    ("rand3-n12", lambda: (W.random_regular(12, 3, 11), None), (1, 2, 3)),
    ("torus3", lambda: (W.torus2d(3), None), (1, 2)),
    ("C10(1,2)", lambda: (W.circulant(10, (1, 2)), None), (1, 2)),
    ("Q3", lambda: (W.hypercube(3), None), (1, 2, 3)),
    ("er-int", lambda: (lambda e, w: (W.Graph("er", 10, e.astype(np.int32)), w))(*_erdos(10, 0.35, 3, "int")), (1, 2)),
    ("er-real", lambda: (lambda e, w: (W.Graph("er", 10, e.astype(np.int32)), w))(*_erdos(10, 0.3, 4, "real")), (1, 2, 3)),
]


@pytest.mark.parametrize("name,make,ps", BRUTE_CASES, ids=[c[0] for c in BRUTE_CASES])
def test_lightcone_sum_equals_bruteforce(name, make, ps):
    g, w = make()
    for p in ps:
        ga, be = W.draw_angles(2, p, 40 + p)
        pl = oracle.plan(g.n, g.edges, w, None, p, reduce=False, max_k=g.n)
        E, zz = oracle.energy(pl, ga, be)
        for i in range(2):
            Eb, zzb = oracle.bruteforce_full(g.n, g.edges, w, ga[i], be[i])
            assert abs(E[i] - Eb) < 1e-11 * max(1.0, abs(Eb))
            np.testing.assert_allclose(zz[i], zzb, atol=1e-12)


# ------------------------------------------------------ Theorem 1 and the reduced energy
@pytest.mark.parametrize("make,p", [(lambda: W.circulant(13, (1, 2)), 2), (lambda: W.torus2d(4), 2),
                                    (lambda: W.hypercube(4), 2), (lambda: W.circulant(11, (1, 3)), 3)])
def test_theorem1_and_reduced_equals_unreduced(make, p):
    g = make()
    ga, be = W.draw_angles(3, p, 77)
    full = oracle.plan(g.n, g.edges, None, None, p, reduce=False)
    red = oracle.plan(g.n, g.edges, None, g.gens(), p, reduce=True)
    Ef, zzf = oracle.energy(full, ga, be)
    Er, zzr = oracle.energy(red, ga, be)
    for m in range(len(red["rep"])):
        members = np.nonzero(red["edge_orbit"] == m)[0]
        # Theorem 1: every term of a class has the same expectation
        np.testing.assert_allclose(zzf[:, members], zzf[:, [red["rep"][m]] * len(members)], atol=1e-12)
        np.testing.assert_allclose(zzr[:, m], zzf[:, red["rep"][m]], atol=1e-13)
    np.testing.assert_allclose(Er, Ef, rtol=1e-12)
    assert len(red["rep"]) < len(full["rep"])


# ---------------------------------------------------------------- angle-space invariants
def test_angle_invariants():
    g = W.random_regular(10, 3, 5)
    rng = np.random.default_rng(3)
    p = 2
    ga, be = rng.uniform(0, np.pi, (3, p)), rng.uniform(0, np.pi / 2, (3, p))
    pl = oracle.plan(g.n, g.edges, None, None, p, reduce=False)
    E0, _ = oracle.energy(pl, ga, be)
    for l in range(p):
        b2 = be.copy()
        b2[:, l] += np.pi / 2         # U_B(beta + pi/2) = (-i)^n X^n U_B(beta)
        np.testing.assert_allclose(oracle.energy(pl, ga, b2)[0], E0, atol=1e-12)
        g2 = ga.copy()
        g2[:, l] += 2 * np.pi         # integer cut values
        np.testing.assert_allclose(oracle.energy(pl, g2, be)[0], E0, atol=1e-11)
    np.testing.assert_allclose(oracle.energy(pl, -ga, -be)[0], E0, atol=1e-12)  # complex conjugation
    W_total = g.m
    z = np.zeros_like(ga)
    np.testing.assert_allclose(oracle.energy(pl, z, be)[0], W_total / 2, atol=1e-12)
    np.testing.assert_allclose(oracle.energy(pl, ga, z)[0], W_total / 2, atol=1e-12)


def test_state_norm_and_global_flip_symmetry():
    g = W.random_regular(12, 3, 9)
    pl = oracle.plan(g.n, g.edges, None, None, 3, reduce=False)
    ga, be = W.draw_angles(1, 3, 1)
    for cone in pl["cones"][:4]:
        k = cone["k"]
        psi = qaoa_state(k, cut_values(k, cone["edges"]), ga[0], be[0])
        assert abs(np.vdot(psi, psi).real - 1) < 1e-12
        flip = np.arange(1 << k) ^ ((1 << k) - 1)
        np.testing.assert_allclose(psi, psi[flip], atol=1e-14)


def test_qubit_order_invariance():
    g = W.random_regular(14, 3, 21)
    perm = np.random.default_rng(2).permutation(g.n)
    h = W.relabel(g, perm)
    ga, be = W.draw_angles(2, 2, 8)
    Eg, zg = oracle.energy(oracle.plan(g.n, g.edges, None, None, 2, reduce=False), ga, be)
    Eh, zh = oracle.energy(oracle.plan(h.n, h.edges, None, None, 2, reduce=False), ga, be)
    np.testing.assert_allclose(Eg, Eh, rtol=1e-12)
    np.testing.assert_allclose(zg, zh[:, h.edge_map], atol=1e-12)


# ---------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("weighted", [None, "real"])
def test_forward_mode_gradient_vs_central_differences(weighted):
    e, w = _erdos(9, 0.4, 12, weighted)
    p = 3
    pl = oracle.plan(9, e, w, None, p, reduce=False, max_k=9)
    ga, be = W.draw_angles(2, p, 19)
    E, dg, db, _ = oracle.energy_grad(pl, ga, be)
    fg, fb = oracle.energy_fd(pl, ga, be, h=1e-6)
    np.testing.assert_allclose(E, oracle.energy(pl, ga, be)[0], rtol=1e-13)
    scale = max(1.0, np.abs(dg).max(), np.abs(db).max())
    assert np.abs(dg - fg).max() < 1e-7 * scale
    assert np.abs(db - fb).max() < 1e-7 * scale


# ---------------------------------------------------------------------- orbits
TINY_SYM = [
    ("C6(1,2)", lambda: W.circulant(6, (1, 2))),
    ("C8(1,3)", lambda: W.circulant(8, (1, 3))),
    ("C9(1,2)", lambda: W.circulant(9, (1, 2))),
    ("Q3", lambda: W.hypercube(3)),
    ("torus3", lambda: W.torus2d(3)),
    ("K3", W.triangle),
    ("K5", lambda: W.complete(5)),
    ("paley13", lambda: W.paley(13)),
]


@pytest.mark.parametrize("name,make", TINY_SYM, ids=[c[0] for c in TINY_SYM])
def test_closure_orbits_match_explicit_group(name, make):
    g = make()
    u, v, w = oracle.canonical_edges(g.n, g.edges)
    orb, rep, size = oracle.edge_orbits(g.n, u, v, w, g.gens())
    # the same generators, expanded into the whole group by brute force
    grp = group_closure(g.n, g.gens())
    lab = orbits_under(grp, u, v)
    assert np.array_equal(lab, orb)
    assert np.array_equal(rep, [np.nonzero(orb == m)[0].min() for m in range(len(rep))])
    assert np.all(np.diff(rep) > 0) and size.sum() == g.m
    # every class of the supplied subgroup lies inside one class of the full Aut(G)
    aut = automorphism_group(g.n, g.edges)
    full = orbits_under(aut, u, v)
    for m in range(len(rep)):
        assert len(set(full[orb == m].tolist())) == 1
    # every element of the generated group is an automorphism
    aut_set = {tuple(a) for a in aut.tolist()}
    assert all(tuple(h) in aut_set for h in grp.tolist())


def test_subgroup_orbits_can_be_finer():
    # C_6(1,2) is the octahedron: the dihedral subgroup gives 2 edge classes, Aut(G) gives 1
    g = W.circulant(6, (1, 2))
    u, v, w = oracle.canonical_edges(g.n, g.edges)
    _, rep, _ = oracle.edge_orbits(g.n, u, v, w, g.gens())
    full = orbits_under(automorphism_group(g.n, g.edges), u, v)
    assert len(rep) == 2 and len(set(full.tolist())) == 1


@pytest.mark.parametrize("make,count", [(lambda: W.torus2d(7), 1), (lambda: W.hypercube(6), 1),
                                        (lambda: W.circulant(50, (1, 2, 5)), 3),
                                        (lambda: W.circulant(101, (1, 2)), 2),
                                        (lambda: W.random_regular(60, 3, 1), 90)])
def test_orbit_counts_by_construction(make, count):
    g = make()
    u, v, w = oracle.canonical_edges(g.n, g.edges)
    _, rep, _ = oracle.edge_orbits(g.n, u, v, w, g.gens())
    assert len(rep) == count


def test_paper_table_orbit_counts():
    spec = json.load(open(os.path.join(GOLDEN, "paper_table_orbits.json")))
    fam = {"complete": W.complete, "torus2d": W.torus2d, "torus3d": W.torus3d,
           "rook": W.rook, "paley": W.paley}
    for row in spec["rows"]:
        g = fam[row["family"]](row["arg"])
        assert (g.n, g.m) == (row["V"], row["E"]), row["paper_row"]
        u, v, w = oracle.canonical_edges(g.n, g.edges)
        _, rep, _ = oracle.edge_orbits(g.n, u, v, w, g.gens())
        assert len(rep) == row["N_orb"], row["paper_row"]
    for row in spec["trivial_group_rows"]:
        g = W.random_regular(row["n"], row["d"], 1)
        u, v, w = oracle.canonical_edges(g.n, g.edges)
        _, rep, _ = oracle.edge_orbits(g.n, u, v, w, np.zeros((0, g.n)))
        assert g.m == row["E"] and len(rep) == row["N_orb"], row["paper_row"]


def test_weighted_symmetry_must_preserve_weights():
    g = W.circulant(8, (1,))
    w = np.ones(g.m)
    u, v, _ = oracle.canonical_edges(g.n, g.edges)
    oracle.edge_orbits(g.n, u, v, w, g.gens())
    w2 = w.copy()
    w2[0] = 2.0
    with pytest.raises(NotAutomorphism):
        oracle.edge_orbits(g.n, u, v, w2, g.gens())
    # alternating weights are kept by rotation by two but not by rotation by one
    w3 = np.array([1.0 if (min(a, b) % 2 == 0) ^ (abs(int(a) - int(b)) > 1) else -1.0 for a, b in g.edges])
    rot2 = (np.arange(8) + 2) % 8
    orb, rep, _ = oracle.edge_orbits(g.n, u, v, w3, rot2[None, :])
    assert len(rep) == 2
    with pytest.raises(NotAutomorphism):
        oracle.edge_orbits(g.n, u, v, w3, g.gens()[:1])


def test_bad_inputs_rejected():
    with pytest.raises(ProblemError):
        oracle.canonical_edges(3, [[0, 0]])
    with pytest.raises(ProblemError):
        oracle.canonical_edges(3, [[0, 1], [1, 0]])
    with pytest.raises(ProblemError):
        oracle.canonical_edges(3, [[0, 3]])
    g = W.circulant(8, (1,))
    u, v, w = oracle.canonical_edges(g.n, g.edges)
    with pytest.raises(NotAutomorphism):
        oracle.edge_orbits(g.n, u, v, w, np.array([[1, 0, 2, 3, 4, 5, 6, 7]]))
    with pytest.raises(NotAutomorphism):
        oracle.edge_orbits(g.n, u, v, w, np.array([[0, 0, 2, 3, 4, 5, 6, 7]]))


def test_cone_is_radius_p_ball_with_paper_order():
    g = W.torus2d(9)
    pl = oracle.plan(g.n, g.edges, None, g.gens(), 2)
    cone = pl["cones"][0]
    u, v = int(pl["u"][0]), int(pl["v"][0])
    assert cone["nodes"][:2] == [u, v]
    # the radius-2 ball around an edge of the square torus: 2 + 6 + 10 = 18 nodes
    assert cone["k"] == 18
    adj = {x: set() for x in range(g.n)}
    for a, b in g.edges:
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    dist = {u: 0, v: 0}
    for d in (1, 2):
        for x in [y for y in dist if dist[y] == d - 1]:
            for y in adj[x]:
                dist.setdefault(y, d)
    assert set(cone["nodes"]) == set(dist)
    keys = [(dist[x], x) for x in cone["nodes"][2:]]
    assert keys == sorted(keys)
    induced = sum(1 for a, b in g.edges if int(a) in dist and int(b) in dist)
    assert len(cone["edges"]) == induced


# ---------------------------------- the pins catch plausible mistakes planted in the oracle
def test_pins_detect_planted_mistakes(monkeypatch):
    import oracle.statevector as sv
    g = W.random_regular(10, 3, 2)
    ga, be = W.draw_angles(1, 1, 3)
    ref = [oracle.zz_p1(g.n, g.edges, None, int(a), int(b), ga[0, 0], be[0, 0]) for a, b in g.edges]

    def zz_now():
        pl = oracle.plan(g.n, g.edges, None, None, 1, reduce=False)
        return oracle.energy(pl, ga, be)[1][0]

    assert np.abs(zz_now() - ref).max() < 1e-12
    good = sv._apply_x_rotation

    def wrong_sign(psi, k, j, beta):
        return good(psi, k, j, -beta)
    monkeypatch.setattr(sv, "_apply_x_rotation", wrong_sign)
    assert np.abs(zz_now() - ref).max() > 1e-3
    monkeypatch.setattr(sv, "_apply_x_rotation", good)

    good_cut = sv.cut_values

    def dropped_edge(k, edges, weights=None):
        return good_cut(k, list(edges)[1:], None if weights is None else list(weights)[1:])
    import sys
    monkeypatch.setattr(sys.modules["oracle.energy"], "cut_values", dropped_edge)
    assert np.abs(zz_now() - ref).max() > 1e-3
