"""Graph replay (opts.graph): captured launch sequences replayed with new angle values.

Every replay is checked bit for bit against an eager plan on the same inputs, with eager
torch work and synchronisations between the replays.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2101_10296_amd as Q
    return Q


@pytest.mark.parametrize("grad", [True, False])
def test_graph_replay_matches_eager(Q, grad):
    # C_60(1,2,3) at p = 2: 14-qubit cones (workgroup kernel) and 15-16-qubit cones (passes)
    g, p, P = W.circulant(60, (1, 2, 3)), 2, 4
    eager = Q.Plan(g.n, g.edges, p=p, generators=g.gens())
    rep = Q.Plan(g.n, g.edges, p=p, generators=g.gens(), graph=True)
    M = rep.n_orbits
    dev = torch.device("cuda")
    gt = torch.zeros((P, p), dtype=torch.float64, device=dev)
    bt = torch.zeros((P, p), dtype=torch.float64, device=dev)
    E = torch.empty(P, dtype=torch.float64, device=dev)
    A = torch.empty((P, p), dtype=torch.float64, device=dev)
    B = torch.empty((P, p), dtype=torch.float64, device=dev)
    Z = torch.empty((P, M), dtype=torch.float64, device=dev)
    for it in range(5):
        ga, be = W.draw_angles(P, p, 900 + it)
        gt.copy_(torch.as_tensor(ga))
        bt.copy_(torch.as_tensor(be))
        if grad:
            rep.energy_grad(gt, bt, out=(E, A, B))
        else:
            rep.energy(gt, bt, term_zz=True, out=(E, Z))
        torch.cuda.synchronize()
        junk = torch.randn(4096, device=dev).cumsum(0)      # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
        if grad:
            Ee, Ae, Be = eager.energy_grad(gt, bt)
            torch.cuda.synchronize()
            assert torch.equal(E, Ee) and torch.equal(A, Ae) and torch.equal(B, Be), it
        else:
            Ee, Ze = eager.energy(gt, bt, term_zz=True)
            torch.cuda.synchronize()
            assert torch.equal(E, Ee) and torch.equal(Z, Ze), it
    assert rep.info()["graph_replays"] == 4      # the first call captures, the rest replay
    # a call with other output buffers captures again and is still correct
    Ee2 = rep.energy(gt, bt) if not grad else rep.energy_grad(gt, bt)[0]
    torch.cuda.synchronize()
    assert torch.equal(Ee2, Ee)

