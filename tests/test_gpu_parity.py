"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (FP32 amplitudes, FP64 accumulation):
  * per term       |zz_gpu - zz_oracle| <= 1e-5
  * energy         |E_gpu - E_oracle|  <= 1e-5 * W_total / 2   (E = sum_m W_m (1 - zz_m) / 2)
  * gradient       ||g_gpu - g_oracle||_inf <= 1e-4 * max(||g_oracle||_inf, 1e-3 * W_total) per point
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ZZ_TOL = 1e-5


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_10296_amd as Q
    return Q


def dev(a):
    return torch.as_tensor(np.asarray(a, np.float64), device="cuda")


def check_energy(Q, g, p, ga, be, reduce=True, weights=None, grad=False, plan_kw=None, sample=None):
    plan_kw = plan_kw or {}
    pl = Q.Plan(g.n, g.edges, p=p, weights=weights, generators=g.gens() if reduce else None, reduce=reduce,
                **plan_kw)
    ref = oracle.plan(g.n, g.edges, weights, g.gens() if reduce else None, p, reduce=reduce, max_k=30)
    E, zz = pl.energy(dev(ga), dev(be), term_zz=True)
    torch.cuda.synchronize()
    E, zz = E.cpu().numpy(), zz.cpu().numpy()
    Wt = float(np.sum(np.abs(ref["W"])))   # |E_gpu - E| <= sum_m |W_m| |dzz_m| / 2 (signed weights too)
    if sample is None:
        Eo, zzo = oracle.energy(ref, ga, be)
        assert np.abs(zz - zzo).max() <= ZZ_TOL, np.abs(zz - zzo).max()
        assert np.abs(E - Eo).max() <= ZZ_TOL * Wt / 2 + 1e-12
    else:   # sampled terms (large plans): oracle term by term
        rng = np.random.default_rng(0)
        ms = rng.choice(len(ref["rep"]), size=min(sample, len(ref["rep"])), replace=False)
        sub = dict(ref, cones=[ref["cones"][m] for m in ms], rep=ref["rep"][ms], W=ref["W"][ms])
        _, zzo = oracle.energy(sub, ga, be)
        assert np.abs(zz[:, ms] - zzo).max() <= ZZ_TOL
        # the energy is the orbit-weighted sum of the GPU's own terms
        np.testing.assert_allclose(E, (ref["W"][None, :] * (1 - zz) / 2).sum(1), rtol=1e-12, atol=1e-9)
    if grad:
        E2, dg, db = pl.energy_grad(dev(ga), dev(be))
        torch.cuda.synchronize()
        # the adjoint kernels use their own register layout, so E agrees to rounding only
        assert np.abs(E2.cpu().numpy() - E).max() <= ZZ_TOL * Wt / 2 + 1e-12
        Eo, dgo, dbo, _ = oracle.energy_grad(ref, ga, be)
        dg, db = dg.cpu().numpy(), db.cpu().numpy()
        for i in range(ga.shape[0]):
            ref_inf = max(np.abs(dgo[i]).max(), np.abs(dbo[i]).max())
            err = max(np.abs(dg[i] - dgo[i]).max(), np.abs(db[i] - dbo[i]).max())
            assert err <= 1e-4 * max(ref_inf, 1e-3 * Wt), (i, err, ref_inf)
    return pl, E, zz


def test_config1_n16_p1(Q):
    (g, p), = W.workload("c1")[0]
    _, ga, be = W.workload("c1")
    pl, E, zz = check_energy(Q, g, p, ga, be, reduce=False, grad=True)
    Eb, zzb = oracle.bruteforce_full(g.n, g.edges, None, ga[0], be[0])
    assert abs(E[0] - Eb) <= ZZ_TOL * g.m / 2
    cf = [oracle.zz_p1(g.n, g.edges, None, int(a), int(b), ga[0, 0], be[0, 0]) for a, b in g.edges]
    assert np.abs(zz[0] - np.array(cf)).max() <= ZZ_TOL


def test_single_edge_and_triangle(Q):
    ga, be = W.draw_angles(7, 1, 3)
    check_energy(Q, W.single_edge(), 1, ga, be, grad=True)
    check_energy(Q, W.triangle(), 1, ga, be, grad=True)
    ga, be = W.draw_angles(5, 2, 4)
    check_energy(Q, W.triangle(), 2, ga, be, grad=True)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_random_regular_small(Q, p):
    g = W.random_regular(12, 3, 31)
    ga, be = W.draw_angles(9, p, 10 + p)
    check_energy(Q, g, p, ga, be, reduce=False, grad=True)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_every_workgroup_cone_size(Q, p):
    # star K_{1,m}: every cone is the whole star, k = m + 1 = 2 .. 14 qubits
    for m in range(1, 14):
        g = W.star(m)
        ga, be = W.draw_angles(3, p, 50 + m)
        pl, _, _ = check_energy(Q, g, p, ga, be, reduce=(m % 2 == 0), grad=True)
        assert pl.info()["max_k"] == m + 1


def test_mixed_cone_sizes_one_plan(Q):
    g = W.random_regular(40, 3, 7)
    ga, be = W.draw_angles(6, 2, 77)
    pl, _, _ = check_energy(Q, g, 2, ga, be, reduce=False, grad=True)
    assert len([c for c in pl.info()["k_hist"] if c]) >= 3


def test_reduced_equals_unreduced_and_theorem1(Q):
    g = W.circulant(50, (1, 2))
    ga, be = W.draw_angles(11, 2, 7)
    pr = Q.Plan(g.n, g.edges, p=2, generators=g.gens())
    pu = Q.Plan(g.n, g.edges, p=2, reduce=False)
    Er, zr = pr.energy(dev(ga), dev(be), term_zz=True)
    Eu, zu = pu.energy(dev(ga), dev(be), term_zz=True)
    eo, rep, _ = pr.orbits()
    zu, zr = zu.cpu().numpy(), zr.cpu().numpy()
    # Theorem 1 on the GPU's own unreduced terms (FP32 rounding only)
    for m in range(len(rep)):
        assert np.abs(zu[:, eo == m] - zr[:, m:m + 1]).max() <= 1e-6
    np.testing.assert_allclose(Er.cpu().numpy(), Eu.cpu().numpy(), rtol=1e-6)


def test_weighted_integer(Q):
    rng = np.random.default_rng(5)
    g = W.random_regular(14, 3, 9)
    w = rng.choice([-1.0, 1.0, 2.0], size=g.m)
    ga, be = W.draw_angles(4, 2, 12)
    check_energy(Q, g, 2, ga, be, reduce=False, weights=w, grad=True)


def test_angle_edge_cases(Q):
    g = W.random_regular(16, 3, 4)
    ga = np.array([[0.0, 0.3], [1.1, 0.0], [np.pi / 2, np.pi], [-0.7, 2.9], [7.0, -4.0]])
    be = np.array([[0.2, 0.0], [0.0, 0.0], [np.pi / 4, np.pi / 4], [np.pi / 2, -0.1], [3.0, 1.0]])
    check_energy(Q, g, 2, ga, be, reduce=False, grad=True)


def test_deterministic_and_plain_path_identical(Q):
    g = W.random_regular(60, 3, 8)
    ga, be = W.draw_angles(5, 2, 1)
    pl = Q.Plan(g.n, g.edges, p=2)
    E1, dg1, db1 = pl.energy_grad(dev(ga), dev(be))
    E2, dg2, db2 = pl.energy_grad(dev(ga), dev(be))
    plain = Q.Plan(g.n, g.edges, p=2, one_cone_at_a_time=True)
    E3, dg3, db3 = plain.energy_grad(dev(ga), dev(be))
    for a, b, c in ((E1, E2, E3), (dg1, dg2, dg3), (db1, db2, db3)):
        assert torch.equal(a, b) and torch.equal(a, c)


def test_ragged_batches(Q):
    g = W.random_regular(20, 3, 3)
    pl = Q.Plan(g.n, g.edges, p=2)
    ref = oracle.plan(g.n, g.edges, None, None, 2)
    for P in (1, 3, 63, 65, 130):
        ga, be = W.draw_angles(P, 2, P)
        E = pl.energy(dev(ga), dev(be)).cpu().numpy()
        Eo, _ = oracle.energy(ref, ga, be)
        assert np.abs(E - Eo).max() <= ZZ_TOL * g.m / 2


def test_autograd_function(Q):
    # the autograd Function's backward, with a weighted upstream gradient, against the
    # oracle's forward-mode gradient (and the oracle energy for its forward)
    g = W.circulant(40, (1, 2))
    pl = Q.Plan(g.n, g.edges, p=2, generators=g.gens())
    ga, be = W.draw_angles(3, 2, 2)
    gt = dev(ga).requires_grad_(True)
    bt = dev(be).requires_grad_(True)
    E = Q.qaoa_energy(pl, gt, bt)
    wts = np.array([1.0, -2.0, 0.5])
    (E * dev(wts)).sum().backward()
    ref = oracle.plan(g.n, g.edges, None, g.gens(), 2, reduce=True)
    Eo, dgo, dbo, _ = oracle.energy_grad(ref, ga, be)
    assert np.abs(E.detach().cpu().numpy() - Eo).max() <= ZZ_TOL * g.m / 2
    got_g, got_b = gt.grad.cpu().numpy(), bt.grad.cpu().numpy()
    for i in range(3):
        want_g, want_b = wts[i] * dgo[i], wts[i] * dbo[i]
        scale = max(np.abs(want_g).max(), np.abs(want_b).max(), 1e-3 * g.m * abs(wts[i]))
        assert max(np.abs(got_g[i] - want_g).max(), np.abs(got_b[i] - want_b).max()) <= 1e-4 * scale, i


def test_config2_circulant_reduced(Q):
    (g, p), = W.workload("c2i")[0]
    _, ga, be = W.workload("c2i")
    check_energy(Q, g, p, ga[:32], be[:32], grad=True)


def test_config3_full_gradient_one_point(Q):
    # random 3-regular n=1000, p=2: every one of the 1500 cone gradients at one angle point
    (g, p), = W.workload("c3")[0]
    _, ga, be = W.workload("c3")
    check_energy(Q, g, p, ga[:1], be[:1], grad=True)


def test_config3_gradient_all_points(Q):
    # the same workload at all 64 angle points against stored oracle energies and gradients
    # (tests/golden/make_oracle_golden.py), and against FP64 central differences of the
    # oracle at two of them
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.json")) as f:
        c = {x["name"]: x for x in json.load(f)["cases"]}["c3_rand3_n1000_p2_all"]
    (g, p), = W.workload("c3")[0]
    _, ga, be = W.workload("c3")
    assert c["points"] == 64 and np.array_equal(W.draw_angles(64, 2, c["seed"])[0], ga)
    pl = Q.Plan(g.n, g.edges, p=p)
    E, dg, db = (x.cpu().numpy() for x in pl.energy_grad(dev(ga), dev(be)))
    Eo, dgo, dbo = np.array(c["energy"]), np.array(c["dgamma"]), np.array(c["dbeta"])
    assert np.abs(E - Eo).max() <= ZZ_TOL * g.m / 2
    for i in range(64):
        ref_inf = max(np.abs(dgo[i]).max(), np.abs(dbo[i]).max())
        err = max(np.abs(dg[i] - dgo[i]).max(), np.abs(db[i] - dbo[i]).max())
        assert err <= 1e-4 * max(ref_inf, 1e-3 * g.m), (i, err, ref_inf)
    # central differences (h = 1e-6) of the oracle energy on a sample of 60 terms, through
    # the per-term gradients the library returns
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False)
    ms = np.random.default_rng(30).choice(g.m, size=60, replace=False)
    sub = dict(ref, cones=[ref["cones"][m] for m in ms], rep=ref["rep"][ms], W=np.ones(len(ms)))
    fdg, fdb = oracle.energy_fd(sub, ga[:2], be[:2])
    _, _, _, _, tg = pl.energy_grad_terms(dev(ga[:2]), dev(be[:2]))
    tg = tg.cpu().numpy()[:, :, ms]
    got = -0.5 * tg.sum(axis=2)
    want = np.concatenate([fdg, fdb], axis=1)
    assert np.abs(got - want).max() <= 1e-4 * max(np.abs(want).max(), 1e-3 * len(ms))


def test_config2ii_full_batch_sampled_terms(Q):
    # the bench workload at its full size (15000 cones x 256 points), 40 terms checked
    (g, p), = W.workload("c2ii")[0]
    _, ga, be = W.workload("c2ii")
    pl, E, zz = check_energy(Q, g, p, ga, be, sample=40)
    E2, dg, db, zzg, tg = pl.energy_grad_terms(dev(ga), dev(be))
    assert np.abs(E2.cpu().numpy() - E).max() <= ZZ_TOL * g.m / 2
    # the full-size gradient call, checked on 40 sampled terms at 16 of its points against
    # the oracle's forward-mode term gradients; the energy gradient is their orbit-weighted
    # sum (Sec. 3) over all terms
    rng = np.random.default_rng(22)
    ms = rng.choice(g.m, size=40, replace=False)
    pts = rng.choice(256, size=16, replace=False)
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False)
    tg_np = tg.cpu().numpy()
    for m in ms:
        cone = ref["cones"][m]
        cut = oracle.cut_values(cone["k"], cone["edges"], cone["weights"])
        for i in pts:
            z, dzg, dzb = oracle.zz_and_grad(cone["k"], cut, ga[i], be[i])
            want = np.concatenate([dzg, dzb])
            assert abs(zzg[i, m].item() - z) <= ZZ_TOL
            assert np.abs(tg_np[i, :, m] - want).max() <= 1e-4 * max(np.abs(want).max(), 1e-3), (m, i)
    want = -0.5 * tg_np.sum(axis=2)
    got = torch.cat([dg, db], dim=1).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-9 * g.m


def test_batches_beyond_one_grid(Q):
    # 15000 cones x 600 points = 9.0 M workgroups of 512 threads at 14 qubits: more
    # work-items than one grid holds (2^32), so the launch is split.  Points whose items
    # fall on either side of the split must come out identical to a small call.
    (g, p), = W.workload("c2ii")[0]
    ga, be = W.draw_angles(600, p, 91)
    pl = Q.Plan(g.n, g.edges, p=p)
    assert pl.info()["k_hist"][14] * 600 * 512 > 2 ** 32
    E, dg, db = pl.energy_grad(dev(ga), dev(be))
    idx = [0, 6, 7, 8, 599]   # the split falls inside one cone's run of points (item 2^32 / 512)
    E2, dg2, db2 = pl.energy_grad(dev(ga[idx]), dev(be[idx]))
    assert torch.equal(E[idx], E2) and torch.equal(dg[idx], dg2) and torch.equal(db[idx], db2)
    Ef = pl.energy(dev(ga), dev(be))
    assert torch.equal(Ef[idx], pl.energy(dev(ga[idx]), dev(be[idx])))


def test_points_beyond_one_grid(Q):
    # 2^24 + 5 points: the per-point combination kernel needs more than one grid
    g = W.single_edge()
    P = (1 << 24) + 5
    ga, be = W.draw_angles(P, 1, 17)
    pl = Q.Plan(g.n, g.edges, p=1)
    E, dg, db = pl.energy_grad(dev(ga), dev(be))
    idx = [0, (1 << 24) - 2, (1 << 24) - 1, 1 << 24, P - 1]
    E2, dg2, db2 = pl.energy_grad(dev(ga[idx]), dev(be[idx]))
    assert torch.equal(E[idx], E2) and torch.equal(dg[idx], dg2) and torch.equal(db[idx], db2)
    ref = oracle.plan(g.n, g.edges, None, None, 1)
    Eo, _ = oracle.energy(ref, ga[idx], be[idx])
    assert np.abs(E2.cpu().numpy() - Eo).max() <= ZZ_TOL / 2


def test_discovered_generators(Q):
    # graphs handed over without generators: the library's own search finds them, and the
    # reduced evaluation with them matches the unreduced one and the oracle
    rng = np.random.default_rng(4)
    torus = W.torus2d(8)
    for g in (W.relabel(torus, rng.permutation(torus.n)), W.circulant(200, (1, 2, 5))):
        gens, complete = Q.find_generators(g.n, g.edges)
        assert complete and len(gens) > 0
        ga, be = W.draw_angles(4, 1, 9)
        red = Q.Plan(g.n, g.edges, p=1, generators=gens)
        unr = Q.Plan(g.n, g.edges, p=1, reduce=False)
        assert red.info()["n_orbits"] < unr.info()["n_orbits"]
        Er, dgr, dbr = red.energy_grad(dev(ga), dev(be))
        Eu, dgu, dbu = unr.energy_grad(dev(ga), dev(be))
        tol = ZZ_TOL * g.m / 2
        assert (Er - Eu).abs().max().item() <= tol
        scale = max(dgu.abs().max().item(), dbu.abs().max().item())
        assert max((dgr - dgu).abs().max().item(), (dbr - dbu).abs().max().item()) <= 1e-4 * scale
        Eo, _ = oracle.energy(oracle.plan(g.n, g.edges, None, None, 1, reduce=False), ga, be)
        assert np.abs(Er.cpu().numpy() - Eo).max() <= tol


def test_input_errors(Q):
    g = W.random_regular(12, 3, 1)
    pl = Q.Plan(g.n, g.edges, p=2)
    with pytest.raises(ValueError):
        pl.energy(dev(np.zeros((2, 2))), dev(np.zeros((3, 2))))


@pytest.mark.parametrize("p", [4, 5, 6])
def test_deep_circuits(Q, p):
    # more layers than the workloads use: both stage orders of the layer loop, many layers
    # undone by the adjoint; cones of 4-10 qubits and the 6- and 14-qubit stars
    g = W.random_regular(10, 3, 5)
    ga, be = W.draw_angles(2, p, 60 + p)
    check_energy(Q, g, p, ga, be, reduce=False, grad=True)
    for m in (5, 13):
        check_energy(Q, W.star(m), p, ga, be, grad=True)


def test_adam_training_matches_oracle(Q):
    # multi-start Adam ascent (the library's trainer against the same rule on the oracle):
    # random 3-regular n=16 at p=2, four starts, 25 steps
    from paper_2101_10296_amd.train import adam_ascent
    g = W.random_regular(16, 3, 0)
    ga, be = W.draw_angles(4, 2, 123)
    ref = oracle.plan(g.n, g.edges, None, None, 2, reduce=False)
    go, bo, Eo, histo = oracle.adam_ascent(ref, ga, be, steps=25, lr=0.02)
    for graph in (False, True):
        pl = Q.Plan(g.n, g.edges, p=2, graph=graph)
        gg, bb, E, hist = adam_ascent(pl, dev(ga), dev(be), steps=25, lr=0.02)
        torch.cuda.synchronize()
        assert np.abs(gg.cpu().numpy() - go).max() <= 1e-4
        assert np.abs(bb.cpu().numpy() - bo).max() <= 1e-4
        assert np.abs(E.cpu().numpy() - Eo).max() <= ZZ_TOL * g.m / 2
        assert np.abs(hist.cpu().numpy() - histo).max() <= 1e-4 * g.m
        assert np.all(Eo > histo[0])
        if graph:
            assert pl.info()["graph_replays"] == 24


@pytest.mark.parametrize("case", ["ring", "torus", "rand_p1", "rand_p2"])
def test_rqaoa_matches_oracle(Q, case):
    # recursive QAOA: the library (GPU correlations, symmetry-reduced where generators
    # survive) against the oracle's plain recursion (FP64, every edge its own cone): the
    # same pairs and signs in the same order, and the same cut
    from paper_2101_10296_amd.rqaoa import rqaoa
    if case == "ring":
        g, p, ang = W.circulant(12, (1,)), 1, ([np.pi / 4], [np.pi / 8])
    elif case == "torus":
        g, p, ang = W.torus2d(4), 1, ([0.55], [0.35])
    elif case == "rand_p1":
        g, p, ang = W.random_regular(14, 3, 44), 1, ([0.6], [0.4])
    else:
        g, p, ang = W.random_regular(14, 3, 45), 2, ([0.5, 0.8], [0.45, 0.2])

    def angles(k, n):
        return ang

    z, cut, steps = rqaoa(g.n, g.edges, None, p, angles, n_stop=6, generators=g.gens())
    zo, cuto, stepso = oracle.rqaoa.rqaoa(g.n, g.edges.tolist(), None, p, angles, n_stop=6)
    assert [tuple(map(int, s)) for s in steps] == [tuple(map(int, s)) for s in stepso]
    assert cut == cuto
    assert set(z.tolist()) <= {1, -1}


def test_rational_weights(Q):
    # weights with a common unit other than 1 (cut values counted in that unit): 1/2 and
    # signed quarters, unreduced, energy and gradient against the oracle
    g = W.random_regular(14, 3, 9)
    rng = np.random.default_rng(3)
    ga, be = W.draw_angles(4, 2, 31)
    for choices, unit in (([0.5, 1.0, 1.5], 0.5), ([-0.25, 0.75, 0.5], 0.25)):
        w = rng.choice(choices, size=g.m)
        pl, _, _ = check_energy(Q, g, 2, ga, be, reduce=False, weights=w, grad=True)
        assert pl.info()["weight_unit"] == unit


def test_rational_weights_with_symmetry(Q):
    # C_40(1,2) with weight 1/2 on the step-1 edges and 5/4 on the step-2 edges: the
    # rotation and reflection preserve the weights, two orbits
    g = W.circulant(40, (1, 2))
    d = (g.edges[:, 1] - g.edges[:, 0]) % g.n
    step = np.minimum(d, g.n - d)
    w = np.where(step == 1, 0.5, 1.25)
    ga, be = W.draw_angles(3, 2, 32)
    pl, _, _ = check_energy(Q, g, 2, ga, be, reduce=True, weights=w, grad=True)
    assert pl.info()["n_orbits"] == 2 and pl.info()["weight_unit"] == 0.25


def test_deep_circuits_phase_rows_in_device_memory(Q):
    # phase rows of 64 two- and three-qubit items per workgroup at p = 150 / 120 do not fit
    # in LDS: the kernels read them from the table in device memory instead
    ga, be = W.draw_angles(2, 150, 91)
    check_energy(Q, W.single_edge(), 150, ga, be, grad=True)
    ga, be = W.draw_angles(2, 120, 92)
    check_energy(Q, W.triangle(), 120, ga, be, grad=True)


def test_real_weights_irrational_with_symmetry(Q):
    # C_40(1,2) with weight 1 on the step-1 edges and sqrt(2) on the step-2 edges (an Ising
    # instance with an edge-colour symmetry, Sec. 4): no common unit, so the phase of every
    # amplitude comes from its own real cut value; the rotation and reflection preserve the
    # weights, two orbits
    g = W.circulant(40, (1, 2))
    d = (g.edges[:, 1] - g.edges[:, 0]) % g.n
    w = np.where(np.minimum(d, g.n - d) == 1, 1.0, 2 ** 0.5)
    ga, be = W.draw_angles(5, 2, 41)
    pl, _, _ = check_energy(Q, g, 2, ga, be, reduce=True, weights=w, grad=True)
    assert pl.info()["real_weights"] == 1 and pl.info()["n_orbits"] == 2


@pytest.mark.parametrize("p", [1, 2, 3])
def test_real_weights_gaussian_unreduced(Q, p):
    # Gaussian couplings (no symmetry survives: every edge its own term), cones of 4-12 qubits
    g = W.random_regular(12, 3, 21)
    w = np.random.default_rng(p).normal(size=g.m)
    ga, be = W.draw_angles(4, p, 42 + p)
    pl, _, _ = check_energy(Q, g, p, ga, be, reduce=False, weights=w, grad=True)
    assert pl.info()["real_weights"] == 1


def test_real_weights_every_cone_size_and_wide_range(Q):
    # stars K_{1,m} (one cone of m + 1 = 2..14 qubits, every workgroup kernel size) with
    # Gaussian weights at p = 2; and integer weights whose cut values span more than 255
    # units (3 x 3 rook graph, weight 30 per edge), which also take the real-weight path
    rng = np.random.default_rng(5)
    for m in range(1, 14):
        g = W.star(m)
        ga, be = W.draw_angles(2, 2, 60 + m)
        check_energy(Q, g, 2, ga, be, reduce=False, weights=rng.normal(size=g.m), grad=True)
    g = W.rook(3)
    ga, be = W.draw_angles(3, 2, 44)
    pl, _, _ = check_energy(Q, g, 2, ga, be, reduce=True, weights=np.full(g.m, 30.0), grad=True)
    assert pl.info()["real_weights"] == 1


def test_real_weights_in_a_batch_and_terms(Q):
    # a batch plan with one real-weight instance: every instance takes the real-weight path;
    # each block equals its own plan, and the per-term gradients combine to the gradient
    g1, g2 = W.random_regular(14, 3, 22), W.circulant(30, (1, 2))
    w1 = np.random.default_rng(7).normal(size=g1.m)
    ga, be = W.draw_angles(3, 2, 45)
    bp = Q.Plan.batch([(g1.n, g1.edges, w1, None), (g2.n, g2.edges, None, g2.gens())], 2)
    assert bp.info()["real_weights"] == 1
    E, dg, db, zz, tg = (x.cpu().numpy() for x in bp.energy_grad_terms(dev(ga), dev(be)))
    for j, (g, w, gens) in enumerate(((g1, w1, None), (g2, None, g2.gens()))):
        ref = oracle.plan(g.n, g.edges, w, gens, 2, reduce=gens is not None)
        Eo, dgo, dbo, _ = oracle.energy_grad(ref, ga, be)
        Wt = float(np.sum(np.abs(ref["W"])))
        assert np.abs(E[j] - Eo).max() <= ZZ_TOL * Wt / 2
        scale = max(np.abs(dgo).max(), np.abs(dbo).max(), 1e-3 * Wt)
        assert max(np.abs(dg[j] - dgo).max(), np.abs(db[j] - dbo).max()) <= 1e-4 * scale
