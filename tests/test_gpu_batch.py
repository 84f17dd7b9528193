"""GPU parity of plans over several graphs (Plan.batch / qaoa_plan_batch).

A batch plan runs the cones of every instance in the same launches; each instance's
energy, gradient and terms must equal those of its own plan (same kernels, so to rounding
of the orbit-weighted sums only) and the oracle within the tolerances of
test_gpu_parity.py.  Covered: workgroup and device-memory cones in one batch, instances
with different weight units, shared and per-instance angle points, the per-term outputs
and the autograd Function.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_gpu_parity import ZZ_TOL, dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_10296_amd as Q
    return Q


def _instances():
    # C_40(1,2) reduced (10-11-qubit cones), an unreduced random 3-regular graph, the star
    # K_{1,15} (one 16-qubit cone in device memory) with weight 1/2 (unit 1/2), and the
    # 7 x 7 torus (18-qubit cones in device memory)
    star = W.star(15)
    return [(W.circulant(40, (1, 2)), True, None), (W.random_regular(24, 3, 6), False, None),
            (star, True, np.full(star.m, 0.5)), (W.torus2d(7), True, None)]


def test_batch_matches_single_plans_and_oracle(Q):
    graphs = _instances()
    p, P = 2, 3
    N = len(graphs)
    bp = Q.Plan.batch([(g.n, g.edges, w, g.gens() if red else None) for g, red, w in graphs], p)
    assert bp.info()["n_hbm_cones"] >= 2
    ga = np.stack([W.draw_angles(P, p, 700 + j)[0] for j in range(N)])
    be = np.stack([W.draw_angles(P, p, 700 + j)[1] for j in range(N)])
    E, dg, db = (x.cpu().numpy() for x in bp.energy_grad(dev(ga), dev(be)))
    Ef, zz = bp.energy(dev(ga), dev(be), term_zz=True)
    Ef, zz = Ef.cpu().numpy(), zz.cpu().numpy()
    assert E.shape == (N, P) and dg.shape == (N, P, p)
    o0 = 0
    for j, (g, red, w) in enumerate(graphs):
        single = Q.Plan(g.n, g.edges, p=p, weights=w, generators=g.gens() if red else None)
        Es, dgs, dbs = (x.cpu().numpy() for x in single.energy_grad(dev(ga[j]), dev(be[j])))
        _, zzs = single.energy(dev(ga[j]), dev(be[j]), term_zz=True)
        zzs = zzs.cpu().numpy()
        M = zzs.shape[1]
        assert np.abs(zz[:, o0:o0 + M] - zzs).max() <= 1e-12
        Wt = float(np.sum(w)) if w is not None else float(g.m)
        assert np.abs(E[j] - Es).max() <= 1e-12 * max(1.0, Wt) and np.abs(Ef[j] - Es).max() <= ZZ_TOL * Wt
        assert np.abs(dg[j] - dgs).max() <= 1e-12 * max(1.0, Wt) and np.abs(db[j] - dbs).max() <= 1e-12 * max(1.0, Wt)
        ref = oracle.plan(g.n, g.edges, w, g.gens() if red else None, p, reduce=red, max_k=30)
        Eo, dgo, dbo, _ = oracle.energy_grad(ref, ga[j], be[j])
        assert np.abs(E[j] - Eo).max() <= ZZ_TOL * Wt / 2
        for i in range(P):
            scale = max(np.abs(dgo[i]).max(), np.abs(dbo[i]).max(), 1e-3 * Wt)
            assert max(np.abs(dg[j, i] - dgo[i]).max(), np.abs(db[j, i] - dbo[i]).max()) <= 1e-4 * scale, (j, i)
        o0 += M
    assert o0 == bp.n_orbits


def test_batch_shared_points_terms_and_autograd(Q):
    graphs = _instances()
    p, P = 2, 4
    bp = Q.Plan.batch([(g.n, g.edges, w, g.gens() if red else None) for g, red, w in graphs], p)
    ga, be = W.draw_angles(P, p, 710)
    E, dg, db = bp.energy_grad(dev(ga), dev(be))                  # shared [P, p] points
    N = len(graphs)
    E3, dg3, db3 = bp.energy_grad(dev(np.broadcast_to(ga, (N, P, p)).copy()),
                                  dev(np.broadcast_to(be, (N, P, p)).copy()))
    assert torch.equal(E, E3) and torch.equal(dg, dg3) and torch.equal(db, db3)
    # per-term gradients combine to the energy gradient (units of each instance applied)
    E4, dg4, db4, zz, tg = bp.energy_grad_terms(dev(ga), dev(be))
    assert torch.equal(E4, E)
    tg = tg.cpu().numpy()
    o0 = 0
    for j, (g, red, w) in enumerate(graphs):
        single = Q.Plan(g.n, g.edges, p=p, weights=w, generators=g.gens() if red else None)
        M = single.n_orbits
        # orbit weights W_m of instance j: the sum of its edges' weights
        wj = np.ones(g.m) if w is None else np.asarray(w)
        seo = single.orbits()[0]
        Wm = np.array([wj[seo == m].sum() for m in range(M)])
        want = -0.5 * np.einsum("m,ilm->il", Wm, tg[:, :, o0:o0 + M])
        got = np.concatenate([dg[j].cpu().numpy(), db[j].cpu().numpy()], axis=1)
        assert np.abs(got - want).max() <= 1e-9 * max(1.0, Wm.sum()), j
        o0 += M
    # autograd: shared angles receive the sum over instances of the weighted gradients
    gt = dev(ga).requires_grad_(True)
    bt = dev(be).requires_grad_(True)
    Et = Q.qaoa_energy(bp, gt, bt)
    wts = torch.linspace(-1.0, 2.0, N * P, dtype=torch.float64, device="cuda").reshape(N, P)
    (Et * wts).sum().backward()
    torch.testing.assert_close(gt.grad, (wts[:, :, None] * dg).sum(0))
    torch.testing.assert_close(bt.grad, (wts[:, :, None] * db).sum(0))
