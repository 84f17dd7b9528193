"""The allocation-free energy + gradient entry point against qaoa_energy_grad (GPU).

qaoa_energy_grad_noalloc keeps its per-call scratch in a file-scope device array of the
library (QAOA_NOALLOC_SCRATCH_BYTES = 32 MiB per GPU) and allocates nothing.  Called through the C ABI twice in a row
(the second call with fewer points, so stale contents of the shared array from the first
call would show), on a plan large enough that the points run in several chunks, and on a
small plan; each result must match the allocating entry point on the same plan to the
parity tolerances (per point |dE| <= 1e-5 W/2, gradient 1e-4 relative to its inf-norm).
"""
import ctypes as C

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


def _lib(Q):
    L = Q._capi.lib()
    L.qaoa_energy_grad_noalloc.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 6
    L.qaoa_energy_grad_noalloc.restype = C.c_int32
    return L


def _noalloc(Q, pl, ga, be):
    g = torch.as_tensor(ga, dtype=torch.float64, device="cuda").contiguous()
    b = torch.as_tensor(be, dtype=torch.float64, device="cuda").contiguous()
    P = g.shape[0]
    E = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
    dg = torch.full((P, pl.p), float("nan"), dtype=torch.float64, device="cuda")
    db = torch.full((P, pl.p), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    rc = _lib(Q).qaoa_energy_grad_noalloc(pl._h, P, g.data_ptr(), b.data_ptr(), E.data_ptr(), dg.data_ptr(),
                                          db.data_ptr(), st)
    assert rc == 0, Q._capi.lib().qaoa_last_error()
    torch.cuda.synchronize()
    return E.cpu().numpy(), dg.cpu().numpy(), db.cpu().numpy()


def _check(Q, pl, ga, be, Wt):
    E0, dg0, db0 = (x.cpu().numpy() for x in pl.energy_grad(torch.as_tensor(ga, device="cuda"),
                                                           torch.as_tensor(be, device="cuda")))
    E1, dg1, db1 = _noalloc(Q, pl, ga, be)
    assert np.abs(E1 - E0).max() <= 1e-5 * Wt / 2
    for i in range(ga.shape[0]):
        ref = max(np.abs(dg0[i]).max(), np.abs(db0[i]).max(), 1e-3 * Wt)
        assert max(np.abs(dg1[i] - dg0[i]).max(), np.abs(db1[i] - db0[i]).max()) <= 1e-4 * ref, i


def test_noalloc_matches_energy_grad_two_calls(Q):
    # random 3-regular n = 10000, p = 2: 15000 orbits, 600 KB of scratch per point, so 256
    # points take five chunks of the 32 MiB array; the second call has 37 points
    g = W.random_regular(10000, 3, 202)
    pl = Q.Plan(g.n, g.edges, p=2)
    ga, be = W.draw_angles(256, 2, 201)
    _check(Q, pl, ga, be, g.m)
    ga2, be2 = W.draw_angles(37, 2, 209)
    _check(Q, pl, ga2, be2, g.m)
    # and a different, smaller plan on the same array (the ring at p = 3: 8-qubit cones)
    h = W.circulant(30, (1,))
    pl2 = Q.Plan(h.n, h.edges, p=3, generators=h.gens())
    ga3, be3 = W.draw_angles(5, 3, 210)
    _check(Q, pl2, ga3, be3, h.m)


def test_noalloc_rejects_what_it_cannot_hold(Q):
    # a plan that has not been evaluated on the device yet, and one with a cone of more than
    # 14 qubits (its state would need device memory), are refused with EINVAL
    L = _lib(Q)
    g = W.star(15)
    pl = Q.Plan(g.n, g.edges, p=2, generators=g.gens())
    x = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    args = (x.data_ptr(), x.data_ptr(), out.data_ptr(), out.data_ptr(), out.data_ptr(), st)
    assert L.qaoa_energy_grad_noalloc(pl._h, 1, *args) == Q.QAOA_EINVAL
    assert b"not resident" in L.qaoa_last_error()
    pl.energy_grad(x, x)
    assert L.qaoa_energy_grad_noalloc(pl._h, 1, *args) == Q.QAOA_EINVAL
    assert b"device memory" in L.qaoa_last_error()
    # one point of 2100 two-qubit orbits at p = 1024 needs (2p + 1) 2100 doubles of per-term
    # values, more than the array holds
    n = 4200
    edges = np.stack([np.arange(0, n, 2), np.arange(1, n, 2)], axis=1)
    big = Q.Plan(n, edges, p=1024, reduce=False)
    y = torch.full((1, 1024), 0.3, dtype=torch.float64, device="cuda")
    o2 = torch.zeros(2048, dtype=torch.float64, device="cuda")
    big.energy_grad(y, y)
    assert L.qaoa_energy_grad_noalloc(big._h, 1, y.data_ptr(), y.data_ptr(), o2.data_ptr(), o2.data_ptr(),
                                      o2.data_ptr(), st) == Q.QAOA_EINVAL
    assert b"bytes of scratch" in L.qaoa_last_error()
