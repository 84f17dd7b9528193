"""The run-time tuner and the layout variants it chooses between (GPU).

Every workgroup layout variant (one register bit fewer per LDS stage; workgroups of at
least 256 threads; the register/lane exchange layouts of the 14-qubit adjoint kernel) is
compared with the oracle on every cone size; plans built with
tune=True are compared with the default layout to the parity tolerances, and the tuner's
record lists a choice with a time for every candidate of each class it met.
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


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("p", [2, 3])
def test_layout_variants_every_cone_size(Q, variant, p):
    # stars K_{1,m}: one cone of m + 1 = 2..14 qubits, forced layout variant (tune = 2 + v)
    for m in range(1, 14):
        g = W.star(m)
        ga, be = W.draw_angles(3, p, 90 + m)
        check_energy(Q, g, p, ga, be, reduce=(m % 2 == 0), grad=True, plan_kw=dict(tune=2 + variant))


def test_layout_variants_many_items(Q):
    # random 3-regular n = 160 at p = 2: cones of 10-14 qubits, 720 items with ragged tails
    g = W.random_regular(160, 3, 12)
    ga, be = W.draw_angles(3, 2, 93)
    for variant in (1, 2, 3):
        check_energy(Q, g, 2, ga, be, reduce=False, grad=True, plan_kw=dict(tune=2 + variant))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_exchange_layouts_every_depth(Q, p):
    # the 14-qubit star (one 14-qubit cone) in the exchange layouts at p = 1..5: both layer
    # directions, the walk over several undone layers and the last one; unit weights and
    # Gaussian couplings (per-amplitude phases)
    g = W.star(13)
    ga, be = W.draw_angles(3, p, 130 + p)
    check_energy(Q, g, p, ga, be, reduce=True, grad=True, plan_kw=dict(tune=5))
    w = np.random.default_rng(p).normal(size=g.m)
    check_energy(Q, g, p, ga, be, reduce=False, weights=w, grad=True, plan_kw=dict(tune=5))


def test_tuned_plans_match_defaults(Q):
    # workgroup classes (random 3-regular, p = 2) and device-memory classes (the 7 x 7 torus,
    # 18-qubit cones) with the tuner on: the same results as the default layouts to the
    # tolerances, and a record per class
    for g, p, gens in ((W.random_regular(2000, 3, 14), 2, None), (W.torus2d(7), 2, W.torus2d(7).gens())):
        ga, be = W.draw_angles(16, p, 95)
        ref = Q.Plan(g.n, g.edges, p=p, generators=gens)
        tuned = Q.Plan(g.n, g.edges, p=p, generators=gens, tune=True)
        E0, dg0, db0 = ref.energy_grad(dev(ga), dev(be))
        for _ in range(2):   # the first call tunes, the second uses the cached choices
            E1, dg1, db1 = tuned.energy_grad(dev(ga), dev(be))
            assert (E1 - E0).abs().max().item() <= ZZ_TOL * g.m / 2
            scale = max(dg0.abs().max().item(), db0.abs().max().item(), 1e-3 * g.m)
            assert max((dg1 - dg0).abs().max().item(), (db1 - db0).abs().max().item()) <= 1e-4 * scale
    rep = Q.tuning_report()
    lines = [ln for ln in rep.splitlines() if ln]
    assert any("workgroup-variant k=14 p=2 grad=1" in ln for ln in lines), rep
    assert any("passes-tiles-per-workgroup k=18 p=2 grad=1" in ln for ln in lines), rep
    for ln in lines:
        choice = int(ln.split("choice=")[1].split()[0])
        times = dict(kv.split("=") for kv in ln.split("ms:")[1].split())
        assert str(choice) in times and all(float(t) > 0 for t in times.values())
