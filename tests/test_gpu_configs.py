"""GPU parity at the full sizes of the mixed-graph and large-cone workloads.

* the 48-graph mix (tori, hypercubes, circulants C_n(1,2,5), random 3- and 4-regular
  graphs; p = 1 or 2; 32 angle points each), every graph reduced by its generators:
  sampled orbit terms against the oracle, the full oracle gradient on five graphs, and
  the energy / gradient consistency of every plan;
* random 3-regular n=200 at p=3 (300 cones of 20-30 qubits) at its first two angle points
  (bench.py times them): every cone of up to 22 qubits term by term against the oracle,
  stored oracle terms of sampled 24-, 25-, 26- and 29-qubit cones (three pass groups) and
  stored oracle term gradients of a 24- and a 25-qubit cone; for all of it, the invariance
  of energy and gradient under a relabelling of the nodes (which changes every cone's qubit
  order, so every kernel data path differs).
Tolerances as in test_gpu_parity.py.
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


def _golden(kind):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.json")
    with open(path) as f:
        return {c["name"]: c for c in json.load(f)[kind]}


def _grad_close(dg, db, dgo, dbo, Wt):
    for i in range(dgo.shape[0]):
        ref_inf = max(np.abs(dgo[i]).max(), np.abs(dbo[i]).max())
        err = max(np.abs(dg[i] - dgo[i]).max(), np.abs(db[i] - dbo[i]).max())
        assert err <= 1e-4 * max(ref_inf, 1e-3 * Wt), (i, err, ref_inf)


def test_config4_mixed_graphs(Q):
    graphs, ga, be = W.workload("c4")
    assert len(graphs) == 48
    full_oracle = {"torus32x32", "Q8"}
    rng = np.random.default_rng(4)
    n_full = 0
    single = {}
    for gi, (g, p) in enumerate(graphs):
        gam, bet = ga[:, :p], be[:, :p]
        pl = Q.Plan(g.n, g.edges, p=p, generators=g.gens())
        E, zz = pl.energy(dev(gam), dev(bet), term_zz=True)
        E2, dg, db = pl.energy_grad(dev(gam), dev(bet))
        E, zz, E2 = E.cpu().numpy(), zz.cpu().numpy(), E2.cpu().numpy()
        dg, db = dg.cpu().numpy(), db.cpu().numpy()
        single[gi] = (E2, dg, db)
        ref = oracle.plan(g.n, g.edges, None, g.gens(), p, reduce=True, max_k=30)
        Wt = float(np.sum(ref["W"]))
        assert np.array_equal(pl.orbits()[1], ref["rep"])
        np.testing.assert_allclose(E, (ref["W"][None, :] * (1 - zz) / 2).sum(1), rtol=1e-12, atol=1e-9)
        assert np.abs(E2 - E).max() <= ZZ_TOL * Wt / 2
        assert np.isfinite(dg).all() and np.isfinite(db).all()
        # a few orbit terms with cones the oracle runs quickly, at two points
        small = [m for m, c in enumerate(ref["cones"]) if c["k"] <= 14]
        ms = rng.choice(small, size=min(3, len(small)), replace=False) if small else []
        if len(ms):
            sub = dict(ref, cones=[ref["cones"][m] for m in ms], rep=ref["rep"][ms], W=ref["W"][ms])
            _, zzo = oracle.energy(sub, gam[:2], bet[:2])
            assert np.abs(zz[:2, ms] - zzo).max() <= ZZ_TOL, g.name
        if g.name == "C100(1,2,5)":   # 20-22-qubit cones: energy terms at one point
            _, zzo = oracle.energy(ref, gam[:1], bet[:1])
            assert np.abs(zz[:1] - zzo).max() <= ZZ_TOL
        # the whole gradient against the oracle on graphs with few or small orbits
        if g.name in full_oracle or (g.n <= 150 and max(c["k"] for c in ref["cones"]) <= 14):
            Eo, dgo, dbo, _ = oracle.energy_grad(ref, gam[:2], bet[:2])
            assert np.abs(E[:2] - Eo).max() <= ZZ_TOL * Wt / 2
            _grad_close(dg[:2], db[:2], dgo, dbo, Wt)
            n_full += 1
    assert n_full >= 5
    # the same 48 graphs as two batch plans (one per depth, one call each): every graph's
    # block equals its own plan's result up to the rounding of the orbit-weighted sums
    for p in (1, 2):
        ids = [gi for gi, (g, pg) in enumerate(graphs) if pg == p]
        bp = Q.Plan.batch([(graphs[gi][0].n, graphs[gi][0].edges, None, graphs[gi][0].gens()) for gi in ids], p)
        Eb, dgb, dbb = (x.cpu().numpy() for x in bp.energy_grad(dev(ga[:, :p]), dev(be[:, :p])))
        for j, gi in enumerate(ids):
            Es, dgs, dbs = single[gi]
            m = graphs[gi][0].m
            assert np.abs(Eb[j] - Es).max() <= 1e-12 * m
            assert max(np.abs(dgb[j] - dgs).max(), np.abs(dbb[j] - dbs).max()) <= 1e-12 * m


def test_config5ii_full_size(Q):
    (g, p), = W.workload("c5ii")[0]
    _, ga, be = W.workload("c5ii")
    ga, be = ga[:2], be[:2]
    pl = Q.Plan(g.n, g.edges, p=p)
    info = pl.info()
    assert info["max_k"] == 30 and info["n_hbm_cones"] == 300
    E, zz = pl.energy(dev(ga), dev(be), term_zz=True)
    E2, dg, db, zzg, tg = pl.energy_grad_terms(dev(ga), dev(be))
    assert pl.info()["pass_launches"][8] > 0   # the three-group reverse mixer passes ran
    E, zz, E2 = E.cpu().numpy(), zz.cpu().numpy(), E2.cpu().numpy()
    dg, db, zzg, tg = dg.cpu().numpy(), db.cpu().numpy(), zzg.cpu().numpy(), tg.cpu().numpy()
    assert np.isfinite(zz).all() and np.abs(zz).max() <= 1 + 1e-5
    assert np.abs(zzg - zz).max() <= ZZ_TOL
    # stored oracle values (tests/golden/make_oracle_golden.py) of cones too large to rerun
    gold = _golden("term_cases")["c5ii_terms_k24_29"]
    for j, e in enumerate(gold["edges"]):
        assert pl.cone(e)[0] == gold["k"][j]
        assert np.abs(zz[:gold["points"], e] - np.array(gold["zz"])[:, j]).max() <= ZZ_TOL, e
    gold = _golden("term_grad_cases")["c5ii_term_grads_k24_25"]
    for j, e in enumerate(gold["edges"]):
        assert pl.cone(e)[0] == gold["k"][j]
        for i in range(gold["points"]):
            assert abs(zzg[i, e] - gold["zz"][j][i]) <= ZZ_TOL
            ref = np.array(gold["dzz"][j][i])
            assert np.abs(tg[i, :, e] - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-3), (e, i)
    np.testing.assert_allclose(E, ((1 - zz) / 2).sum(1), rtol=1e-12, atol=1e-9)
    assert np.abs(E2 - E).max() <= ZZ_TOL * g.m / 2
    # term by term where the oracle can: every cone of at most 22 qubits, at two points
    ref = oracle.plan(g.n, g.edges, None, None, p, reduce=False, max_k=30)
    ms = np.array([m for m, c in enumerate(ref["cones"]) if c["k"] <= 22])
    assert len(ms) >= 5
    sub = dict(ref, cones=[ref["cones"][m] for m in ms], rep=ref["rep"][ms], W=ref["W"][ms])
    _, zzo = oracle.energy(sub, ga[:1], be[:1])
    assert np.abs(zz[:1, ms] - zzo).max() <= ZZ_TOL
    pl.close()   # frees the state buffers (most of the device memory)
    # the adjoint reading stored forward states (checkpoint_mode 1: up to five 4 GiB states
    # per 30-qubit item): the same terms and gradient within the tolerances, and the stored
    # oracle term gradients
    plc = Q.Plan(g.n, g.edges, p=p, checkpoint_mode=1)
    Ec, dgc, dbc, zzc, tgc = (x.cpu().numpy() for x in plc.energy_grad_terms(dev(ga), dev(be)))
    assert plc.info()["checkpointed_classes"] > 0
    plc.close()
    assert np.abs(zzc - zzg).max() <= ZZ_TOL and np.abs(Ec - E).max() <= ZZ_TOL * g.m / 2
    ginf = max(np.abs(dg).max(), np.abs(db).max())
    assert max(np.abs(dgc - dg).max(), np.abs(dbc - db).max()) <= 1e-4 * max(ginf, 1e-3 * g.m)
    for j, e in enumerate(gold["edges"]):
        for i in range(gold["points"]):
            ref = np.array(gold["dzz"][j][i])
            assert np.abs(tgc[i, :, e] - ref).max() <= 1e-4 * max(np.abs(ref).max(), 1e-3), (e, i)
    # relabelled graph: same energies and gradients
    perm = np.random.default_rng(7).permutation(g.n)
    gr = W.relabel(g, perm)
    plr = Q.Plan(gr.n, gr.edges, p=p)
    Er, dgr, dbr = plr.energy_grad(dev(ga[:2]), dev(be[:2]))
    assert np.abs(Er.cpu().numpy() - E[:2]).max() <= ZZ_TOL * g.m / 2
    ginf = max(np.abs(dg[:2]).max(), np.abs(db[:2]).max())
    err = max(np.abs(dgr.cpu().numpy() - dg[:2]).max(), np.abs(dbr.cpu().numpy() - db[:2]).max())
    assert err <= 1e-4 * max(ginf, 1e-3 * g.m)
