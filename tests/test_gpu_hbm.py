"""GPU parity of cones held in device memory (more than k_lds_max qubits) against the oracle.

Same tolerances as test_gpu_parity.py.  Covered: one, two and three pass groups of stored
qubits (a k-qubit cone stores k - 1 qubits: group 0 holds 13, each further group up to 9,
so three groups start at 24 stored qubits, k = 25), depths 1-5, every pass kind (asserted
through the plan's per-kind launch counters), the p = 1 path that needs no state buffers,
the smallest device-memory cones (15 and 16 qubits: one and two tile pairs), reduced plans
and batching under a small memory budget.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import ZZ_TOL, check_energy, dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_10296_amd as Q
    return Q


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("m", [14, 15])
def test_hbm_star_all_depths(Q, p, m):
    # star K_{1,m}: one orbit whose cone holds all m + 1 qubits (15 or 16: the smallest
    # cones kept in device memory, one or two tile pairs of the stored half)
    g = W.star(m)
    ga, be = W.draw_angles(3, p, 70 + p)
    pl, _, _ = check_energy(Q, g, p, ga, be, grad=True)
    assert pl.info()["n_hbm_cones"] == 1 and pl.info()["max_k"] == m + 1


def test_workgroup_and_device_classes_one_plan_p3(Q):
    # C_40(1,2) at p = 3: a 14-qubit cone (workgroup kernel) and a 15-qubit one (passes)
    g = W.circulant(40, (1, 2))
    ga, be = W.draw_angles(3, 3, 17)
    pl, _, _ = check_energy(Q, g, 3, ga, be, grad=True)
    assert pl.info()["n_hbm_cones"] == 1 and pl.info()["min_k"] == 14


def test_torus_k18_p2_reduced(Q):
    g = W.torus2d(7)
    ga, be = W.draw_angles(3, 2, 11)
    pl, _, _ = check_energy(Q, g, 2, ga, be, grad=True)
    assert pl.info()["max_k"] == 18 and pl.info()["n_orbits"] == 1


def test_several_hbm_classes_one_plan(Q):
    # C_60(1,2,3) at p = 2: three orbits with 14-, 15- and 16-qubit cones
    g = W.circulant(60, (1, 2, 3))
    ga, be = W.draw_angles(3, 2, 12)
    pl, _, _ = check_energy(Q, g, 2, ga, be, grad=True)
    assert pl.info()["n_hbm_cones"] == 2 and pl.info()["max_k"] == 16


def test_hypercube_q10_p1_k20(Q):
    g = W.hypercube(10)
    ga, be = W.draw_angles(4, 1, 13)
    pl, _, zz = check_energy(Q, g, 1, ga, be, grad=True)
    assert pl.info()["max_k"] == 20


def test_q12_p1_k24_closed_form(Q):
    # config: hypercube Q_12, p = 1, one orbit, a 24-qubit cone; the p = 1 closed form
    # gives zz, and central differences of it (FP64) give the gradient
    (g, p), = W.workload("c5i")[0]
    _, ga, be = W.workload("c5i")
    pl = Q.Plan(g.n, g.edges, p=1, generators=g.gens())
    assert pl.info()["max_k"] == 24 and pl.info()["n_orbits"] == 1
    E, zz = pl.energy(dev(ga), dev(be), term_zz=True)
    E2, dg, db = pl.energy_grad(dev(ga), dev(be))
    u, v = (int(x) for x in g.edges[0])
    cf = lambda a, b: oracle.zz_p1(g.n, g.edges, None, u, v, a, b)  # noqa: E731
    h = 1e-6
    for i in range(ga.shape[0]):
        z = cf(ga[i, 0], be[i, 0])
        assert abs(zz[i, 0].item() - z) <= ZZ_TOL
        dz_g = (cf(ga[i, 0] + h, be[i, 0]) - cf(ga[i, 0] - h, be[i, 0])) / (2 * h)
        dz_b = (cf(ga[i, 0], be[i, 0] + h) - cf(ga[i, 0], be[i, 0] - h)) / (2 * h)
        ref = np.array([-0.5 * g.m * dz_g, -0.5 * g.m * dz_b])
        got = np.array([dg[i, 0].item(), db[i, 0].item()])
        assert np.abs(got - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-3 * g.m)
        assert abs(E2[i].item() - g.m * (1 - z) / 2) <= ZZ_TOL * g.m / 2


def test_small_memory_budget_batches(Q):
    g = W.torus2d(7)
    ga, be = W.draw_angles(5, 2, 15)
    full = Q.Plan(g.n, g.edges, p=2, reduce=False)
    tight = Q.Plan(g.n, g.edges, p=2, reduce=False, mem_budget_bytes=3 * (8 << 18))
    Ef, dgf, dbf = full.energy_grad(dev(ga), dev(be))
    Et, dgt, dbt = tight.energy_grad(dev(ga), dev(be))
    assert torch.equal(Ef, Et) and torch.equal(dgf, dgt) and torch.equal(dbf, dbt)
    with pytest.raises(Q.QaoaError) as ei:
        Q.Plan(g.n, g.edges, p=2, mem_budget_bytes=1 << 20).energy_grad(dev(ga), dev(be))
    assert ei.value.status == Q.QAOA_ENOMEM


def _golden_cases():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.json")
    with open(path) as f:
        return {c["name"]: c for c in json.load(f)["cases"]}


# pass kinds (index into Plan.info()["pass_launches"])
FWD_GEN_MIX, FWD_GEN_FINAL, FWD_MIX, FWD_BND_MIX, FWD_BND_FINAL = 0, 1, 2, 3, 4
GR_GEN_FINAL, GR_BND_FINAL, RV_GEN_MIX, RV_MIX, RV_BND_MIX = 5, 6, 7, 8, 9

# stored case -> (pass kinds of the forward call, pass kinds of the gradient call)
STORED = {
    # a 23-qubit cone (22 stored qubits: two pass groups) at p = 2 and 18-20-qubit ones
    "spider5_5_p2": ({FWD_GEN_MIX, FWD_BND_FINAL}, {FWD_GEN_MIX, GR_BND_FINAL, RV_GEN_MIX}),
    # 20-22-qubit cones (two groups) at p = 3: the layer-boundary passes in both directions
    "C60_1_2_3_p3": ({FWD_GEN_MIX, FWD_BND_MIX, FWD_BND_FINAL},
                     {FWD_GEN_MIX, FWD_BND_MIX, GR_BND_FINAL, RV_BND_MIX, RV_GEN_MIX}),
    # a 25-qubit cone (24 stored qubits: three groups) at p = 2: the mixer-only passes
    "spider5_6_p2": ({FWD_GEN_MIX, FWD_MIX, FWD_BND_FINAL}, {FWD_GEN_MIX, FWD_MIX, GR_BND_FINAL, RV_MIX, RV_GEN_MIX}),
    # four 25-qubit cones at p = 3: every multi-pass kind, both snake directions
    "spider5_6_p3": ({FWD_GEN_MIX, FWD_MIX, FWD_BND_MIX, FWD_BND_FINAL},
                     {FWD_GEN_MIX, FWD_MIX, FWD_BND_MIX, GR_BND_FINAL, RV_MIX, RV_BND_MIX, RV_GEN_MIX}),
    # the 25-qubit cone with real weights sqrt(deg u + deg v) (kept by the generators)
    "spider5_6_p2_rootw": ({FWD_GEN_MIX, FWD_MIX, FWD_BND_FINAL},
                           {FWD_GEN_MIX, FWD_MIX, GR_BND_FINAL, RV_MIX, RV_GEN_MIX}),
}


@pytest.mark.parametrize("ckpt", [0, 1])
@pytest.mark.parametrize("name", list(STORED))
def test_stored_oracle_cases(Q, name, ckpt):
    # oracle values stored by tests/golden/make_oracle_golden.py; every term, the energy and
    # the gradient at every stored point, and the pass kinds that produced them; with the
    # adjoint recovering the forward states by inverse layers (ckpt 0) and reading them
    # from stored checkpoints (ckpt 1)
    c = _golden_cases()[name]
    g = getattr(W, c["family"])(*c["args"])
    w = getattr(W, c["weights"])(g) if c.get("weights") else None
    ga, be = W.draw_angles(c["points"], c["p"], c["seed"])
    pl = Q.Plan(g.n, g.edges, p=c["p"], weights=w, generators=g.gens() if c["reduce"] else None,
                reduce=c["reduce"], checkpoint_mode=ckpt)
    eo, rep, _ = pl.orbits()
    assert list(rep) == c["rep"]
    assert pl.info()["real_weights"] == (1 if w is not None else 0)
    kinds_fwd, kinds_grad = STORED[name]
    E, zz = pl.energy(dev(ga), dev(be), term_zz=True)
    ran = {i for i, n in enumerate(pl.info()["pass_launches"]) if n}
    assert ran == kinds_fwd, ran
    E2, dg, db = pl.energy_grad(dev(ga), dev(be))
    ran = {i for i, n in enumerate(pl.info()["pass_launches"]) if n}
    assert ran == kinds_grad, ran
    assert (pl.info()["checkpointed_classes"] > 0) == bool(ckpt)
    zz = zz.cpu().numpy()
    Wt = float(np.sum(np.abs(c["W"])))
    assert np.abs(zz - np.array(c["zz"])).max() <= ZZ_TOL
    assert np.abs(E.cpu().numpy() - np.array(c["energy"])).max() <= ZZ_TOL * Wt / 2
    assert np.abs(E2.cpu().numpy() - np.array(c["energy"])).max() <= ZZ_TOL * Wt / 2
    dgo, dbo = np.array(c["dgamma"]), np.array(c["dbeta"])
    dg, db = dg.cpu().numpy(), db.cpu().numpy()
    for i in range(ga.shape[0]):
        ref_inf = max(np.abs(dgo[i]).max(), np.abs(dbo[i]).max())
        err = max(np.abs(dg[i] - dgo[i]).max(), np.abs(db[i] - dbo[i]).max())
        assert err <= 1e-4 * max(ref_inf, 1e-3 * Wt), (i, err, ref_inf)


@pytest.mark.parametrize("ckpt", [0, 1])
@pytest.mark.parametrize("p", [4, 5])
def test_deep_circuits_device_memory(Q, p, ckpt):
    # the 15- and 16-qubit stars at p = 4, 5: several boundary passes per group, both snake
    # directions, and the rescale of psi read as the forward sweep left it at deeper layers
    # (the first reverse pass, or with stored checkpoints every reverse pass)
    ga, be = W.draw_angles(2, p, 80 + p)
    for m in (14, 15):
        pl, _, _ = check_energy(Q, W.star(m), p, ga, be, grad=True, plan_kw=dict(checkpoint_mode=ckpt))
        assert (pl.info()["checkpointed_classes"] > 0) == bool(ckpt)


def test_checkpoint_auto_and_budget(Q):
    # auto stores the forward states where the budget holds them at the same batch size:
    # it does under the default budget, not under a budget that fits the uncompute batch only
    # (C_60(1,2,3) at p = 3: cones of 20-22 qubits, two stored states per item)
    g = W.circulant(60, (1, 2, 3))
    ga, be = W.draw_angles(2, 3, 13)
    ref = Q.Plan(g.n, g.edges, p=3, generators=g.gens())
    E0, dg0, db0 = ref.energy_grad(dev(ga), dev(be))
    auto = Q.Plan(g.n, g.edges, p=3, generators=g.gens(), checkpoint_mode=2)
    E1, dg1, db1 = auto.energy_grad(dev(ga), dev(be))
    assert auto.info()["checkpointed_classes"] == auto.info()["n_hbm_cones"] > 0
    tight = Q.Plan(g.n, g.edges, p=3, generators=g.gens(), checkpoint_mode=2,
                   mem_budget_bytes=2 * (8 << 21) + (8 << 20))
    E2, dg2, db2 = tight.energy_grad(dev(ga), dev(be))
    assert tight.info()["checkpointed_classes"] < tight.info()["n_hbm_cones"]
    for E, dg, db in ((E1, dg1, db1), (E2, dg2, db2)):
        assert (E - E0).abs().max().item() <= ZZ_TOL * g.m / 2
        scale = max(dg0.abs().max().item(), db0.abs().max().item())
        assert max((dg - dg0).abs().max().item(), (db - db0).abs().max().item()) <= 1e-4 * scale


def test_deep_weighted_star_rows_in_device_memory(Q):
    # a 15-qubit cone (device-memory passes) with weight 17 on each of its 14 edges: cut
    # range 239, so p = 45 phase rows (86 KB) do not fit beside the pass kernels' LDS
    g = W.star(14)
    w = np.full(g.m, 17.0)
    ga, be = W.draw_angles(2, 45, 93)
    check_energy(Q, g, 45, ga, be, weights=w)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_real_weights_device_memory_star(Q, p):
    # the 16-qubit star (two tile pairs) with Gaussian couplings: real cut values in the
    # device-memory passes, every depth's pass kinds
    g = W.star(15)
    w = np.random.default_rng(20 + p).normal(size=g.m)
    ga, be = W.draw_angles(3, p, 75 + p)
    pl, _, _ = check_energy(Q, g, p, ga, be, reduce=False, weights=w, grad=True)
    assert pl.info()["real_weights"] == 1 and pl.info()["n_hbm_cones"] == g.m


@pytest.mark.parametrize("ckpt", [0, 1])
def test_real_weights_device_memory_circulant(Q, ckpt):
    # C_60(1,2,3) with weights 1, sqrt 2, sqrt 3 by step (the rotation and reflection keep
    # them: three orbits) at p = 3: 20-22-qubit cones in two pass groups, both adjoint modes
    g = W.circulant(60, (1, 2, 3))
    d = (g.edges[:, 1] - g.edges[:, 0]) % g.n
    step = np.minimum(d, g.n - d)
    w = np.sqrt(step.astype(float))
    ga, be = W.draw_angles(1, 3, 79)
    pl, _, _ = check_energy(Q, g, 3, ga, be, reduce=True, weights=w, grad=True,
                            plan_kw=dict(checkpoint_mode=ckpt))
    assert pl.info()["real_weights"] == 1 and pl.info()["n_orbits"] == 3
