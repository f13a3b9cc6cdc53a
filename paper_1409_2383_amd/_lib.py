"""ctypes binding of libntf_admm.so (argument marshalling only).

Every computation happens in the HIP library; this module only mirrors the C
structs of include/ntf_admm.h and loads the shared object built in-tree by
``paper_1409_2383_amd/build.py``.  There is no fallback: if the library is
missing or cannot be loaded, ``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libntf_admm.so")

# status codes
NTF_OK = 0
NTF_NOT_CONVERGED = 1
NTF_E_INVAL = -1
NTF_E_WORKSPACE = -2
NTF_E_HIP = -3
NTF_E_NUMERIC = -4
NTF_E_UNSUPPORTED = -5

PREC_F32, PREC_BF16_MIXED, PREC_F64 = 0, 1, 3
RHO_TRACE, RHO_FIXED, RHO_ADAPTIVE = 0, 1, 2


class Problem(ctypes.Structure):
    _fields_ = [
        ("dims", c_int64 * 3),
        ("F", c_int32),
        ("x_dtype", c_int32),
        ("X", c_void_p),
        ("H", c_void_p * 3),
        ("U", c_void_p * 3),
    ]


class SparseProblem(ctypes.Structure):
    _fields_ = [
        ("dims", c_int64 * 3),
        ("F", c_int32),
        ("x_dtype", c_int32),
        ("nnz", c_int64),
        ("idx", c_void_p),
        ("val", c_void_p),
        ("H", c_void_p * 3),
        ("U", c_void_p * 3),
    ]


MAX_ORDER = 8


class NwayProblem(ctypes.Structure):
    _fields_ = [
        ("order", c_int32),
        ("F", c_int32),
        ("dims", c_int64 * MAX_ORDER),
        ("x_dtype", c_int32),
        ("reserved", c_int32),
        ("X", c_void_p),
        ("H", c_void_p * MAX_ORDER),
        ("U", c_void_p * MAX_ORDER),
    ]


class NwayStats(ctypes.Structure):
    _fields_ = [
        ("outer", c_int64),
        ("rho", c_double * MAX_ORDER),
        ("prim", c_double * MAX_ORDER),
        ("dual", c_double * MAX_ORDER),
        ("norm_h", c_double * MAX_ORDER),
        ("norm_p", c_double * MAX_ORDER),
        ("norm_y", c_double * MAX_ORDER),
        ("inner_iters_mean", c_double * MAX_ORDER),
        ("numeric_error", c_int32),
        ("converged", c_int32),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class Opts(ctypes.Structure):
    _fields_ = [
        ("inner_iters", c_int32),
        ("rho_policy", c_int32),
        ("rho0", c_double),
        ("mu", c_double),
        ("tau_incr", c_double),
        ("tau_decr", c_double),
        ("inner_eps_abs", c_double),
        ("inner_eps_rel", c_double),
        ("stop_eps_abs", c_double),
        ("stop_eps_rel", c_double),
        ("precision", c_int32),
        ("factor_source", c_int32),
        ("rescale_dual_on_rho_change", c_int32),
        ("paper_init", c_int32),
        ("warm_hidden", c_int32),
        ("reserved", c_int32 * 3),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("outer", c_int64),
        ("rho", c_double * 3),
        ("prim", c_double * 3),
        ("dual", c_double * 3),
        ("norm_h", c_double * 3),
        ("norm_p", c_double * 3),
        ("norm_y", c_double * 3),
        ("inner_iters_mean", c_double * 3),
        ("rfe_cheap", c_double),
        ("warm_taken", c_int64 * 3),
        ("numeric_error", c_int32),
        ("converged", c_int32),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class Mlp(ctypes.Structure):
    _fields_ = [
        ("F", c_int32),
        ("hidden", c_int32),
        ("dtype", c_int32),
        ("reserved", c_int32),
        ("params", c_void_p),
    ]


class Constraints(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32 * 3),
        ("reserved", c_int32),
        ("lo", c_double * 3),
        ("hi", c_double * 3),
        ("card", c_int64 * 3),
    ]


CONS_NONNEG, CONS_BOX, CONS_PMF_ROWS, CONS_CARDINALITY = 0, 1, 2, 3


class BatchTile(ctypes.Structure):
    _fields_ = [
        ("kind", c_int32),
        ("ft", c_int32),
        ("qbucket", c_int32),
        ("mt", c_int32),
        ("item_elems", c_int64),
        ("us", c_double),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("n_problems", c_int32),
        ("grid", c_int32),
        ("lds_bytes", c_int32),
        ("n_items", c_int32),
        ("items_by_kind", c_int64 * 9),
        ("x_bytes", c_int64),
        ("t_bytes", c_int64),
    ]


# (name, restype, argtypes) of every exported function
SIGNATURES = [
    ("ntf_status_str", c_char_p, [c_int32]),
    ("ntf_admm_last_error", c_char_p, [c_void_p]),
    ("ntf_admm_workspace_bytes", c_size_t, [POINTER(Problem), POINTER(Opts)]),
    ("ntf_admm_init", c_int32, [POINTER(c_void_p), POINTER(Problem), POINTER(Opts), c_void_p, c_size_t, c_void_p]),
    ("ntf_admm_sparse_workspace_bytes", c_size_t, [POINTER(SparseProblem), POINTER(Opts)]),
    ("ntf_admm_init_sparse", c_int32, [POINTER(c_void_p), POINTER(SparseProblem), POINTER(Opts), c_void_p,
                                       c_size_t, c_void_p]),
    ("ntf_nway_workspace_bytes", c_size_t, [POINTER(NwayProblem), POINTER(Opts)]),
    ("ntf_nway_init", c_int32, [POINTER(c_void_p), POINTER(NwayProblem), POINTER(Opts), c_void_p, c_size_t,
                                c_void_p]),
    ("ntf_nway_step", c_int32, [c_void_p, POINTER(NwayStats)]),
    ("ntf_nway_run", c_int32, [c_void_p, c_int32, c_int32, POINTER(NwayStats)]),
    ("ntf_nway_fit", c_int32, [c_void_p, POINTER(c_double)]),
    ("ntf_nway_mttkrp", c_int32, [c_void_p, c_int32, c_void_p]),
    ("ntf_nway_last_error", c_char_p, [c_void_p]),
    ("ntf_nway_destroy", c_int32, [c_void_p]),
    ("ntf_admm_step", c_int32, [c_void_p, POINTER(Stats)]),
    ("ntf_admm_run", c_int32, [c_void_p, c_int32, c_int32, POINTER(Stats)]),
    ("ntf_admm_fit", c_int32, [c_void_p, POINTER(c_double)]),
    ("ntf_admm_state_bytes", c_size_t, [c_void_p]),
    ("ntf_admm_get_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("ntf_admm_set_state", c_int32, [c_void_p, c_void_p, c_size_t]),
    ("ntf_admm_mttkrp", c_int32, [c_void_p, c_int32, c_void_p]),
    ("ntf_admm_launch_pass", c_int32, [c_void_p, c_int32]),
    ("ntf_admm_destroy", c_int32, [c_void_p]),
    ("ntf_inner_workspace_bytes", c_size_t, [c_int64, c_int32]),
    ("ntf_inner_update", c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p,
                                   c_double, c_int32, c_double, c_double, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]),
    ("ntf_inner_static_scratch_bytes", c_size_t, [c_int32]),
    ("ntf_inner_update_noalloc", c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_int32,
                                           c_void_p, c_double, c_int32, c_double, c_double, c_void_p,
                                           c_void_p, c_void_p]),
    ("ntf_gram_workspace_bytes", c_size_t, [c_int64, c_int32]),
    ("ntf_gram", c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    ("ntf_admm_set_warmstart", c_int32, [c_void_p, POINTER(Mlp)]),
    ("ntf_mlp_param_count", c_size_t, [c_int32, c_int32]),
    ("ntf_mlp_features", c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    ("ntf_mlp_forward", c_int32, [POINTER(Mlp), c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    ("ntf_mlp_backward", c_int32, [POINTER(Mlp), c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                   c_void_p, c_void_p]),
    ("ntf_mlp_mse", c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    ("ntf_mlp_adam", c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, c_int32, c_void_p, c_void_p]),
    ("ntf_gather_rows", c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    ("ntf_mlp_targets", c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    ("ntf_admm_mode_problem", c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    ("ntf_admm_set_constraints", c_int32, [c_void_p, POINTER(Constraints)]),
    ("ntf_batch_workspace_bytes", c_size_t, [POINTER(Problem), c_int32, POINTER(Opts)]),
    ("ntf_batch_init", c_int32, [POINTER(c_void_p), POINTER(Problem), c_int32, POINTER(Opts), c_void_p,
                                 c_size_t, c_void_p]),
    ("ntf_batch_step", c_int32, [c_void_p, c_int32]),
    ("ntf_batch_sync", c_int32, [c_void_p, POINTER(c_int32)]),
    ("ntf_batch_fit", c_int32, [c_void_p, POINTER(c_double)]),
    ("ntf_batch_mttkrp", c_int32, [c_void_p, c_int32, c_int32, c_void_p]),
    ("ntf_batch_launch_kind", c_int32, [c_void_p, c_int32]),
    ("ntf_batch_autotune", c_int32, [c_void_p, c_int32, POINTER(BatchTile), c_int32, POINTER(c_int32)]),
    ("ntf_batch_set_tiles", c_int32, [c_void_p, POINTER(BatchTile), c_int32]),
    ("ntf_batch_get_tiles", c_int32, [c_void_p, POINTER(BatchTile), c_int32, POINTER(c_int32)]),
    ("ntf_batch_info_get", c_int32, [c_void_p, POINTER(BatchInfo)]),
    ("ntf_batch_profile", c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int64)]),
    ("ntf_batch_last_error", c_char_p, [c_void_p]),
    ("ntf_batch_destroy", c_int32, [c_void_p]),
]

_LIB = None


def lib():
    """The loaded library with typed entry points (raises if not built)."""
    global _LIB
    if _LIB is None:
        # Load PyTorch's HIP runtime first so the library binds to the same
        # libamdhip64 instance as the tensors and streams it is handed.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


class NtfError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = lib().ntf_status_str(status).decode()
        super().__init__(f"{where}: {msg} ({status})" + (f": {detail}" if detail else ""))


def check(status: int, where: str, ctx=None, ok=(NTF_OK,), batch=False, nway=False):
    if status not in ok:
        err = (lib().ntf_batch_last_error if batch else
               lib().ntf_nway_last_error if nway else lib().ntf_admm_last_error)
        detail = err(ctx).decode(errors="replace")
        raise NtfError(status, where, detail)
    return status
