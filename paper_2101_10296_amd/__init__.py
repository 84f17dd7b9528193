"""Symmetry-reduced light-cone QAOA MaxCut energy and gradient on AMD Instinct MI355X.

Python binding of libqaoa.so (include/qaoa.h).  Every step of the computation runs in
the library's HIP kernels; this module only marshals arguments.  PyTorch supplies device
memory and the current HIP stream.

    plan = Plan(n, edges, p=2, generators=gens)        # orbits + light cones (host)
    E = plan.energy(gamma, beta)                         # gamma, beta: cuda float64 [P, p]
    E, dgamma, dbeta = plan.energy_grad(gamma, beta)
    E = qaoa_energy(plan, gamma, beta)                   # differentiable (autograd)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _capi
from ._capi import (QAOA_EHIP, QAOA_ECONE, QAOA_EINVAL, QAOA_ENOMEM, QAOA_ENOTAUT,  # noqa: F401
                    QAOA_OK, STATUS_NAMES)

__all__ = ["Plan", "QaoaError", "qaoa_energy", "QAOAEnergyFn", "library_path", "tuning_report", "find_generators"]


def library_path() -> str:
    return _capi.LIB_PATH


class QaoaError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _check(st: int):
    if st != QAOA_OK:
        raise QaoaError(st, _capi.lib().qaoa_last_error().decode(errors="replace"))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _problem(n_nodes, edges, p, weights, generators, keep):
    """A qaoa_problem over host arrays that `keep` holds alive."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    u, v = _i32(e[:, 0]), _i32(e[:, 1])
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    g = None if generators is None else _i32(generators).reshape(-1, int(n_nodes))
    keep.extend([u, v, w, g])
    pr = _capi.Problem()
    pr.n_nodes = int(n_nodes)
    pr.n_edges = int(e.shape[0])
    pr.edge_u = u.ctypes.data_as(C.POINTER(C.c_int32))
    pr.edge_v = v.ctypes.data_as(C.POINTER(C.c_int32))
    pr.edge_w = None if w is None else w.ctypes.data_as(C.POINTER(C.c_double))
    pr.n_generators = 0 if g is None else int(g.shape[0])
    pr.generators = None if g is None or g.size == 0 else g.ctypes.data_as(C.POINTER(C.c_int32))
    pr.p = int(p)
    return pr


class Plan:
    """A planned problem: canonical edges, edge orbits and one light cone per orbit.

    Plan.batch([...], p) plans several graphs together (one launch per cone size for all of
    them); its evaluations take and return one block per instance (see energy())."""

    def __init__(self, n_nodes: int, edges, p: int, weights=None, generators=None, *, reduce: bool = True,
                 max_cone_qubits: int = 30, k_lds_max: int = 14, mem_budget_bytes: int = 0,
                 checkpoint_mode: int = 0, one_cone_at_a_time: bool = False, profile: bool = False,
                 graph: bool = False, tune: bool = False, _instances=None):
        L = _capi.lib()
        o = _capi.PlanOpts()
        L.qaoa_plan_opts_default(C.byref(o))
        o.reduce = int(bool(reduce))
        o.max_cone_qubits = int(max_cone_qubits)
        o.k_lds_max = int(k_lds_max)
        o.mem_budget_bytes = int(mem_budget_bytes)
        o.checkpoint_mode = int(checkpoint_mode)
        o.one_cone_at_a_time = int(bool(one_cone_at_a_time))
        o.profile = int(bool(profile))
        o.graph = int(bool(graph))
        o.tune = int(tune)
        keep = []
        h = C.c_void_p()
        if _instances is None:
            pr = _problem(n_nodes, edges, p, weights, generators, keep)
            _check(L.qaoa_plan_lightcones(C.byref(pr), C.byref(o), C.byref(h)))
        else:
            arr = (_capi.Problem * len(_instances))()
            for j, inst in enumerate(_instances):
                arr[j] = _problem(inst[0], inst[1], p, inst[2] if len(inst) > 2 else None,
                                  inst[3] if len(inst) > 3 else None, keep)
            _check(L.qaoa_plan_batch(arr, len(_instances), C.byref(o), C.byref(h)))
        self._h = h
        self.p = int(p)
        inf = self.info()
        self.n_nodes = int(inf["n_nodes"])
        self.n_edges = int(inf["n_edges"])
        self.n_orbits = int(inf["n_orbits"])
        self.n_instances = int(inf["n_instances"])

    @classmethod
    def batch(cls, instances, p: int, **opts):
        """One plan over several graphs of depth p: instances = [(n_nodes, edges[, weights[,
        generators]]), ...].  Nodes, edges and orbits are numbered instance after instance."""
        return cls(0, None, p, _instances=list(instances), **opts)

    # ---------------------------------------------------------------- host queries
    def info(self) -> dict:
        inf = _capi.PlanInfo()
        _check(_capi.lib().qaoa_plan_query(self._h, C.byref(inf)))
        d = {f: getattr(inf, f) for f, _ in _capi.PlanInfo._fields_ if f not in ("k_hist", "pass_launches")}
        d["k_hist"] = list(inf.k_hist)
        d["pass_launches"] = list(inf.pass_launches)
        return d

    def orbits(self):
        """(edge_orbit int32 [m], rep int64 [M], size int64 [M])."""
        M = self.info()["n_orbits"]
        eo = np.zeros(self.n_edges, np.int32)
        rep = np.zeros(M, np.int64)
        size = np.zeros(M, np.int64)
        _check(_capi.lib().qaoa_plan_orbits(self._h, eo.ctypes.data_as(C.POINTER(C.c_int32)),
                                            rep.ctypes.data_as(C.POINTER(C.c_int64)),
                                            size.ctypes.data_as(C.POINTER(C.c_int64))))
        return eo, rep, size

    def cone(self, m: int):
        """(k, nodes int32 [k], n_cone_edges) of the cone of orbit m."""
        k = C.c_int32()
        ne = C.c_int32()
        nodes = np.zeros(31, np.int32)
        _check(_capi.lib().qaoa_plan_cone(self._h, int(m), C.byref(k), nodes.ctypes.data_as(C.POINTER(C.c_int32)),
                                          31, C.byref(ne)))
        return int(k.value), nodes[: k.value].copy(), int(ne.value)

    def kernel_times(self):
        """[(k, items, ms)] per kernel group of the last call (plans built with profile=True);
        k = -1 is the angle-table kernel, k = -2 the orbit-weighted combination."""
        cap = 64
        ks = np.zeros(cap, np.int32)
        it = np.zeros(cap, np.int64)
        ms = np.zeros(cap, np.float64)
        n = C.c_int32()
        _check(_capi.lib().qaoa_plan_kernel_times(self._h, cap, ks.ctypes.data_as(C.POINTER(C.c_int32)),
                                                  it.ctypes.data_as(C.POINTER(C.c_int64)),
                                                  ms.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        return [(int(ks[i]), int(it[i]), float(ms[i])) for i in range(min(n.value, cap))]

    # ---------------------------------------------------------------- device evaluation
    def _angles(self, gamma, beta):
        """(gamma, beta) as contiguous float64 [N * P, p] with N = n_instances: [P, p] inputs
        are shared by every instance, [N, P, p] inputs give each instance its own points."""
        import torch
        if not (isinstance(gamma, torch.Tensor) and isinstance(beta, torch.Tensor)):
            raise TypeError("gamma and beta must be torch tensors on a HIP device")
        if gamma.device.type != "cuda" or beta.device.type != "cuda":
            raise ValueError("gamma and beta must live on the GPU")
        if gamma.shape != beta.shape:
            raise ValueError("gamma and beta must have the same shape")
        N = self.n_instances
        g = gamma.detach().to(torch.float64)
        b = beta.detach().to(torch.float64)
        if N > 1 and g.dim() == 3:
            if g.shape[0] != N or g.shape[2] != self.p:
                raise ValueError(f"per-instance angles must have shape [{N}, P, {self.p}]")
        else:
            g = g.reshape(-1, self.p)
            b = b.reshape(-1, self.p)
            if N > 1:
                g = g.unsqueeze(0).expand(N, -1, -1)
                b = b.unsqueeze(0).expand(N, -1, -1)
        P = g.shape[-2]
        return g.reshape(-1, self.p).contiguous(), b.reshape(-1, self.p).contiguous(), P

    def _shape(self, P, *rest):
        return (P, *rest) if self.n_instances == 1 else (self.n_instances, P, *rest)

    @staticmethod
    def _out(t, shape, device):
        import torch
        if t is None:
            return torch.empty(shape, dtype=torch.float64, device=device)
        if tuple(t.shape) != tuple(shape) or t.dtype != torch.float64 or not t.is_contiguous() or t.device != device:
            raise ValueError(f"output tensor must be contiguous float64 {tuple(shape)} on {device}")
        return t

    def energy(self, gamma, beta, term_zz: bool = False, out=None):
        """E [P] (and per-orbit <ZZ> [P, M] if term_zz) as cuda float64 tensors; for a plan over
        N > 1 instances E is [N, P] (gamma, beta [P, p] shared or [N, P, p] per instance).

        out: optional preallocated E (or (E, zz) with term_zz), e.g. to keep device pointers
        fixed for graph replay."""
        g, b, P = self._angles(gamma, beta)
        o = out if isinstance(out, (tuple, list)) else (out, None)
        E = self._out(o[0], self._shape(P), g.device)
        zz = self._out(o[1], (P, max(self.n_orbits, 1)), g.device) if term_zz else None
        import torch
        stream = torch.cuda.current_stream(g.device).cuda_stream
        _check(_capi.lib().qaoa_energy(self._h, P, g.data_ptr(), b.data_ptr(), E.data_ptr(),
                                       None if zz is None else zz.data_ptr(), stream))
        return (E, zz[:, : self.n_orbits]) if term_zz else E

    def energy_grad(self, gamma, beta, out=None):
        """(E [P], dE/dgamma [P, p], dE/dbeta [P, p]) as cuda float64 tensors.

        out: optional preallocated (E, dgamma, dbeta)."""
        import torch
        g, b, P = self._angles(gamma, beta)
        o = out if out is not None else (None, None, None)
        E = self._out(o[0], self._shape(P), g.device)
        dg = self._out(o[1], self._shape(P, self.p), g.device)
        db = self._out(o[2], self._shape(P, self.p), g.device)
        stream = torch.cuda.current_stream(g.device).cuda_stream
        _check(_capi.lib().qaoa_energy_grad(self._h, P, g.data_ptr(), b.data_ptr(), E.data_ptr(),
                                            dg.data_ptr(), db.data_ptr(), stream))
        return E, dg, db

    def energy_grad_terms(self, gamma, beta):
        """(E [P], dE/dgamma [P, p], dE/dbeta [P, p], zz [P, M], d zz / d(gamma, beta) [P, 2p, M]):
        the energy gradient together with every orbit term and its own gradient."""
        import torch
        g, b, P = self._angles(gamma, beta)
        dev = g.device
        M = max(self.n_orbits, 1)
        E = torch.empty(self._shape(P), dtype=torch.float64, device=dev)
        dg = torch.empty(self._shape(P, self.p), dtype=torch.float64, device=dev)
        db = torch.empty(self._shape(P, self.p), dtype=torch.float64, device=dev)
        zz = torch.empty((P, M), dtype=torch.float64, device=dev)
        tg = torch.empty((P, 2 * self.p, M), dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        _check(_capi.lib().qaoa_energy_grad_terms(self._h, P, g.data_ptr(), b.data_ptr(), E.data_ptr(), dg.data_ptr(),
                                                  db.data_ptr(), zz.data_ptr(), tg.data_ptr(), stream))
        return E, dg, db, zz[:, : self.n_orbits], tg[:, :, : self.n_orbits]

    def close(self):
        if getattr(self, "_h", None):
            _capi.lib().qaoa_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tuning_report() -> str:
    """The run-time tuner's choices so far in this process (plans built with tune=True)."""
    L = _capi.lib()
    n = C.c_int64()
    _check(L.qaoa_tuning_report(None, 0, C.byref(n)))
    buf = C.create_string_buffer(n.value + 1)
    _check(L.qaoa_tuning_report(buf, n.value + 1, C.byref(n)))
    return buf.value.decode()


def find_generators(n_nodes: int, edges, weights=None, max_generators: int = 256, time_limit: float = 30.0):
    """Automorphism generators of a graph whose symmetry is not known (edge weights act as
    colours): (generators int32 [g, n], complete).  Every row is a verified automorphism;
    complete is False when the time limit or the capacity ended the search (the rows then
    generate a subgroup, which the orbit reduction accepts)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    u, v = _i32(e[:, 0]), _i32(e[:, 1])
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    pr = _capi.Problem()
    pr.n_nodes = int(n_nodes)
    pr.n_edges = int(e.shape[0])
    pr.edge_u = u.ctypes.data_as(C.POINTER(C.c_int32))
    pr.edge_v = v.ctypes.data_as(C.POINTER(C.c_int32))
    pr.edge_w = None if w is None else w.ctypes.data_as(C.POINTER(C.c_double))
    pr.n_generators = 0
    pr.generators = None
    pr.p = 1
    out = np.zeros((int(max_generators), int(n_nodes)), np.int32)
    nf = C.c_int32()
    done = C.c_int32()
    _check(_capi.lib().qaoa_find_generators(C.byref(pr), int(max_generators), float(time_limit),
                                            out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nf), C.byref(done)))
    return out[: nf.value].copy(), bool(done.value)


def _autograd_fn():
    import torch

    class QAOAEnergyFn(torch.autograd.Function):
        """E(gamma, beta) with the adjoint gradient computed in the same library call."""

        @staticmethod
        def forward(ctx, gamma, beta, plan):
            E, dg, db = plan.energy_grad(gamma, beta)
            ctx.save_for_backward(dg, db)
            ctx.shapes = (gamma.shape, beta.shape, gamma.dtype, beta.dtype)
            return E

        @staticmethod
        def backward(ctx, grad_out):
            dg, db = ctx.saved_tensors
            gs, bs, gdt, bdt = ctx.shapes
            go = grad_out.to(torch.float64).unsqueeze(-1)
            gg, gb = go * dg, go * db
            if gg.dim() == 3 and len(gs) < 3:   # angles shared by every instance of a batch plan
                gg, gb = gg.sum(0), gb.sum(0)
            return gg.reshape(gs).to(gdt), gb.reshape(bs).to(bdt), None

    return QAOAEnergyFn


_FN = None


def QAOAEnergyFn():  # noqa: N802 - returns the autograd Function class
    global _FN
    if _FN is None:
        _FN = _autograd_fn()
    return _FN


def qaoa_energy(plan: Plan, gamma, beta):
    """Differentiable energy: gamma, beta [P, p] (cuda) -> E [P]."""
    return QAOAEnergyFn().apply(gamma, beta, plan)
