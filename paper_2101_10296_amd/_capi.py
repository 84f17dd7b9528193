"""ctypes declarations of libqaoa.so (the C ABI in include/qaoa.h)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqaoa.so")

QAOA_OK, QAOA_EINVAL, QAOA_ENOTAUT, QAOA_ECONE, QAOA_ENOMEM, QAOA_EHIP = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "QAOA_OK", -1: "QAOA_EINVAL", -2: "QAOA_ENOTAUT", -3: "QAOA_ECONE",
                -4: "QAOA_ENOMEM", -5: "QAOA_EHIP"}


class Problem(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_edges", C.c_int64),
                ("edge_u", C.POINTER(C.c_int32)), ("edge_v", C.POINTER(C.c_int32)),
                ("edge_w", C.POINTER(C.c_double)),
                ("n_generators", C.c_int32), ("generators", C.POINTER(C.c_int32)),
                ("p", C.c_int32)]


class PlanOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("reduce", C.c_int32), ("max_cone_qubits", C.c_int32),
                ("k_lds_max", C.c_int32), ("checkpoint_mode", C.c_int32), ("one_cone_at_a_time", C.c_int32),
                ("profile", C.c_int32), ("graph", C.c_int32), ("tune", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("p", C.c_int32), ("n_edges", C.c_int64), ("n_orbits", C.c_int64),
                ("min_k", C.c_int32), ("max_k", C.c_int32), ("k_hist", C.c_int64 * 31),
                ("total_weight", C.c_double), ("cut_min", C.c_int32), ("cut_max", C.c_int32),
                ("n_hbm_cones", C.c_int64), ("device_bytes", C.c_int64),
                ("graph_replays", C.c_int64), ("weight_unit", C.c_double),
                ("pass_launches", C.c_int64 * 10), ("checkpointed_classes", C.c_int32),
                ("n_instances", C.c_int32), ("checkpointed_k_mask", C.c_uint32),
                ("real_weights", C.c_int32)]


_lib = None


def lib():
    """Load libqaoa.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2101_10296_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.qaoa_plan_opts_default.argtypes = [C.POINTER(PlanOpts)]
        L.qaoa_plan_opts_default.restype = None
        L.qaoa_plan_lightcones.argtypes = [C.POINTER(Problem), C.POINTER(PlanOpts), C.POINTER(vp)]
        L.qaoa_plan_lightcones.restype = i32
        L.qaoa_plan_batch.argtypes = [C.POINTER(Problem), i32, C.POINTER(PlanOpts), C.POINTER(vp)]
        L.qaoa_plan_batch.restype = i32
        L.qaoa_plan_query.argtypes = [vp, C.POINTER(PlanInfo)]
        L.qaoa_plan_query.restype = i32
        L.qaoa_plan_orbits.argtypes = [vp, C.POINTER(i32), C.POINTER(i64), C.POINTER(i64)]
        L.qaoa_plan_orbits.restype = i32
        L.qaoa_plan_cone.argtypes = [vp, i64, C.POINTER(i32), C.POINTER(i32), i32, C.POINTER(i32)]
        L.qaoa_plan_cone.restype = i32
        L.qaoa_energy.argtypes = [vp, i64, vp, vp, vp, vp, vp]
        L.qaoa_energy.restype = i32
        L.qaoa_energy_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
        L.qaoa_energy_grad.restype = i32
        L.qaoa_energy_grad_terms.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.qaoa_energy_grad_terms.restype = i32
        L.qaoa_plan_kernel_times.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i64), C.POINTER(C.c_double),
                                             C.POINTER(i32)]
        L.qaoa_plan_kernel_times.restype = i32
        L.qaoa_find_generators.argtypes = [C.POINTER(Problem), i32, C.c_double, C.POINTER(i32), C.POINTER(i32),
                                           C.POINTER(i32)]
        L.qaoa_find_generators.restype = i32
        L.qaoa_tuning_report.argtypes = [C.c_char_p, i64, C.POINTER(i64)]
        L.qaoa_tuning_report.restype = i32
        L.qaoa_plan_destroy.argtypes = [vp]
        L.qaoa_plan_destroy.restype = None
        L.qaoa_last_error.argtypes = []
        L.qaoa_last_error.restype = C.c_char_p
        _lib = L
    return _lib
