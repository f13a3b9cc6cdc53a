"""MI355X (gfx950) ADMoM non-negative CP factorisation.

Thin Python front end of libntf_admm.so.  PyTorch provides device memory and
the stream; every step of the method runs in the library's HIP kernels.  The
names follow the paper (Liavas & Sidiropoulos): H_n are the non-negative
factors (A-tilde, B-tilde, C-tilde), U_n the scaled duals (-Y_n / rho_n).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

from . import _lib
from ._lib import (PREC_BF16_MIXED, PREC_F32, PREC_F64, RHO_ADAPTIVE, RHO_FIXED, RHO_TRACE,
                   NtfError)

__all__ = ["NtfAdmm", "NtfAdmmSparse", "NtfNway", "NtfBatch", "AdmmOptions", "inner_update", "gram", "PREC_F32", "PREC_BF16_MIXED",
           "PREC_F64", "RHO_TRACE", "RHO_FIXED", "RHO_ADAPTIVE", "NtfError", "library_path"]


def library_path() -> str:
    _lib.lib()
    return _lib.LIB_PATH


@dataclass
class AdmmOptions:
    inner_iters: int = 1
    rho_policy: int = RHO_TRACE
    rho0: float = 1.0
    mu: float = 8.0
    tau_incr: float = 4.0
    tau_decr: float = 2.0
    inner_eps_abs: float = 0.0
    inner_eps_rel: float = 0.0
    stop_eps_abs: float = 0.0
    stop_eps_rel: float = 0.0
    precision: int = PREC_F32
    factor_source: int = 0
    rescale_dual_on_rho_change: int = 0
    paper_init: int = 0
    warm_hidden: int = 0

    def to_c(self) -> _lib.Opts:
        o = _lib.Opts()
        for name, _ in _lib.Opts._fields_:
            if name == "reserved":
                continue
            setattr(o, name, getattr(self, name))
        return o


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> int:
    return t.data_ptr()


class NtfAdmm:
    """ADMoM NTF solver bound to one tensor and one set of factor buffers.

    X: CUDA tensor [I, J, K], float32 (F32 / BF16_MIXED) or float64 (F64), C order.
    H: three CUDA tensors [d_n, F] (float32, or float64 for F64): initial
       factors, updated in place.  U: three duals of the same shape (zeros if
       omitted).  The workspace is a torch uint8 tensor owned by this object, or
    the caller's (`workspace`: at least ntf_admm_workspace_bytes long; an
    earlier solver's `.workspace.numel()` for the same shape and options).
    """

    def __init__(self, X, H: Sequence, U: Optional[Sequence] = None,
                 opts: Optional[AdmmOptions] = None, stream=None, workspace=None):
        torch = _torch()
        self.opts = opts or AdmmOptions()
        fdt = torch.float64 if self.opts.precision == PREC_F64 else torch.float32
        if not X.is_cuda or not X.is_contiguous() or X.dim() != 3:
            raise ValueError("X must be a contiguous 3-way CUDA tensor")
        if X.dtype != fdt:
            raise ValueError(f"X must be {fdt} for this precision")
        F = H[0].shape[1]
        self.X = X
        self.H = list(H)
        for n in range(3):
            h = self.H[n]
            if (not h.is_cuda or h.dtype != fdt or not h.is_contiguous()
                    or tuple(h.shape) != (X.shape[n], F)):
                raise ValueError(f"H[{n}] must be a contiguous CUDA {fdt} tensor of shape "
                                 f"({X.shape[n]}, {F})")
        self.U = list(U) if U is not None else [torch.zeros_like(h) for h in self.H]
        for n in range(3):
            if self.U[n].shape != self.H[n].shape or self.U[n].dtype != fdt or not self.U[n].is_contiguous():
                raise ValueError(f"U[{n}] must match H[{n}]")
        self.F = F
        self.dims = tuple(int(d) for d in X.shape)
        self.device = X.device
        self.stream = stream
        L = _lib.lib()
        pr = _lib.Problem()
        for n in range(3):
            pr.dims[n] = X.shape[n]
            pr.H[n] = _ptr(self.H[n])
            pr.U[n] = _ptr(self.U[n])
        pr.F = F
        pr.x_dtype = 1 if self.opts.precision == PREC_F64 else 0
        pr.X = _ptr(X)
        self._prob = pr
        self._copts = self.opts.to_c()
        nbytes = L.ntf_admm_workspace_bytes(ctypes.byref(pr), ctypes.byref(self._copts))
        if nbytes == 0:
            ctx = ctypes.c_void_p()
            st = L.ntf_admm_init(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts),
                                 None, 0, _stream_handle(stream))
            _lib.check(st, "ntf_admm_init")
        if workspace is not None:
            if (not workspace.is_cuda or workspace.dtype != torch.uint8 or not workspace.is_contiguous()
                    or workspace.numel() < nbytes):
                raise ValueError(f"workspace must be a contiguous CUDA uint8 tensor of >= {nbytes} bytes")
            self.workspace = workspace
        else:
            self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=X.device)
        ctx = ctypes.c_void_p()
        st = L.ntf_admm_init(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts),
                             ctypes.c_void_p(_ptr(self.workspace)), nbytes, _stream_handle(stream))
        _lib.check(st, "ntf_admm_init", None)
        self._ctx = ctx

    # -- solver
    def step(self, stats: bool = False):
        L = _lib.lib()
        if stats:
            s = _lib.Stats()
            _lib.check(L.ntf_admm_step(self._ctx, ctypes.byref(s)), "ntf_admm_step", self._ctx)
            return s.as_dict()
        _lib.check(L.ntf_admm_step(self._ctx, None), "ntf_admm_step", self._ctx)
        return None

    def run(self, max_outer: int, check_every: int = 1, stats: bool = True):
        L = _lib.lib()
        s = _lib.Stats()
        st = L.ntf_admm_run(self._ctx, int(max_outer), int(check_every),
                            ctypes.byref(s) if stats else None)
        _lib.check(st, "ntf_admm_run", self._ctx, ok=(_lib.NTF_OK, _lib.NTF_NOT_CONVERGED))
        out = s.as_dict() if stats else {}
        out["status"] = st
        return out

    def fit(self) -> float:
        r = ctypes.c_double()
        _lib.check(_lib.lib().ntf_admm_fit(self._ctx, ctypes.byref(r)), "ntf_admm_fit", self._ctx)
        return r.value

    def mttkrp(self, mode: int):
        torch = _torch()
        W = torch.empty((self.dims[mode], self.F), dtype=torch.float64, device=self.device)
        _lib.check(_lib.lib().ntf_admm_mttkrp(self._ctx, int(mode), ctypes.c_void_p(_ptr(W))),
                   "ntf_admm_mttkrp", self._ctx)
        return W

    def launch_pass(self, which: int):
        """Enqueue one MTTKRP kernel only (0: pass 1, 1: mode 2 from T, 2: pass 3)."""
        _lib.check(_lib.lib().ntf_admm_launch_pass(self._ctx, int(which)), "ntf_admm_launch_pass",
                   self._ctx)

    def plan_info(self) -> dict:
        """Algorithmic bytes of each MTTKRP kernel launch."""
        return pass_bytes(tuple(self.X.shape), self.F, self.opts.precision, self.X.element_size())

    def set_constraints(self, constraints=None):
        """Per-mode set constraints: a sequence of three entries, each None or
        "nonneg", ("box", lo, hi), "pmf_rows" or ("cardinality", c) (Section
        IV-E, Section VI-D)."""
        c = _lib.Constraints()
        for m, spec in enumerate(constraints or (None, None, None)):
            if spec is None or spec == "nonneg":
                c.kind[m] = _lib.CONS_NONNEG
            elif spec == "pmf_rows":
                c.kind[m] = _lib.CONS_PMF_ROWS
            elif isinstance(spec, tuple) and spec[0] == "box":
                c.kind[m] = _lib.CONS_BOX
                c.lo[m], c.hi[m] = float(spec[1]), float(spec[2])
            elif isinstance(spec, tuple) and spec[0] == "cardinality":
                c.kind[m] = _lib.CONS_CARDINALITY
                c.card[m] = int(spec[1])
            else:
                raise ValueError(f"unknown constraint {spec!r}")
        _lib.check(_lib.lib().ntf_admm_set_constraints(self._ctx, ctypes.byref(c)),
                   "ntf_admm_set_constraints", self._ctx)

    def get_state(self) -> bytes:
        L = _lib.lib()
        n = L.ntf_admm_state_bytes(self._ctx)
        buf = ctypes.create_string_buffer(n)
        _lib.check(L.ntf_admm_get_state(self._ctx, buf, n), "ntf_admm_get_state", self._ctx)
        return buf.raw

    def set_state(self, blob: bytes):
        L = _lib.lib()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _lib.check(L.ntf_admm_set_state(self._ctx, buf, len(blob)), "ntf_admm_set_state", self._ctx)

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.lib().ntf_admm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NtfAdmmSparse(NtfAdmm):
    """ADMoM NTF of a sparse tensor given by its non-zeros (Section IV-A,
    item 1).

    idx: CUDA int32 tensor [nnz, 3] of distinct coordinates (any order);
    val: CUDA tensor [nnz], float32 (F32) or float64 (F64); dims: (I, J, K).
    The library sorts three copies of the non-zeros into its workspace at
    set-up; idx and val are not used afterwards.  Every other method is the
    dense solver's.
    """

    def __init__(self, idx, val, dims, H: Sequence, U: Optional[Sequence] = None,
                 opts: Optional[AdmmOptions] = None, stream=None):
        torch = _torch()
        self.opts = opts or AdmmOptions()
        fdt = torch.float64 if self.opts.precision == PREC_F64 else torch.float32
        nnz = int(idx.shape[0]) if idx.dim() == 2 else -1
        if (not idx.is_cuda or idx.dtype != torch.int32 or idx.dim() != 2 or idx.shape[1] != 3
                or not idx.is_contiguous()):
            raise ValueError("idx must be a contiguous CUDA int32 tensor of shape (nnz, 3)")
        if not val.is_cuda or val.dtype != fdt or tuple(val.shape) != (nnz,) or not val.is_contiguous():
            raise ValueError(f"val must be a contiguous CUDA {fdt} tensor of shape ({nnz},)")
        self.X = None
        self.dims = tuple(int(d) for d in dims)
        self.device = val.device
        F = H[0].shape[1]
        self.H = list(H)
        for n in range(3):
            h = self.H[n]
            if (not h.is_cuda or h.dtype != fdt or not h.is_contiguous()
                    or tuple(h.shape) != (self.dims[n], F)):
                raise ValueError(f"H[{n}] must be a contiguous CUDA {fdt} tensor of shape "
                                 f"({self.dims[n]}, {F})")
        self.U = list(U) if U is not None else [torch.zeros_like(h) for h in self.H]
        for n in range(3):
            if self.U[n].shape != self.H[n].shape or self.U[n].dtype != fdt or not self.U[n].is_contiguous():
                raise ValueError(f"U[{n}] must match H[{n}]")
        self.F = F
        self.nnz = nnz
        self.stream = stream
        L = _lib.lib()
        pr = _lib.SparseProblem()
        for n in range(3):
            pr.dims[n] = self.dims[n]
            pr.H[n] = _ptr(self.H[n])
            pr.U[n] = _ptr(self.U[n])
        pr.F = F
        pr.x_dtype = 1 if self.opts.precision == PREC_F64 else 0
        pr.nnz = nnz
        pr.idx = _ptr(idx) if nnz > 0 else None
        pr.val = _ptr(val) if nnz > 0 else None
        self._prob = pr
        self._copts = self.opts.to_c()
        nbytes = L.ntf_admm_sparse_workspace_bytes(ctypes.byref(pr), ctypes.byref(self._copts))
        if nbytes == 0:
            ctx = ctypes.c_void_p()
            st = L.ntf_admm_init_sparse(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts),
                                        None, 0, _stream_handle(stream))
            _lib.check(st, "ntf_admm_init_sparse")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        st = L.ntf_admm_init_sparse(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts),
                                    ctypes.c_void_p(_ptr(self.workspace)), nbytes, _stream_handle(stream))
        _lib.check(st, "ntf_admm_init_sparse", None)
        self._ctx = ctx

    def plan_info(self) -> dict:
        """Algorithmic bytes of one sparse MTTKRP launch per mode."""
        return sparse_pass_bytes(self.dims, self.F, self.nnz, self.opts.precision)


class NtfNway:
    """ADMoM NTF of a dense tensor of order N = 3..8 (Appendix A).

    X: contiguous CUDA tensor with N dims, float32 (F32) or float64 (F64);
    H: N factor tensors [I_n, F], updated in place; U: duals (zeros if
    omitted).  Same options as NtfAdmm (mixed precision and the learned warm
    start excepted)."""

    def __init__(self, X, H: Sequence, U: Optional[Sequence] = None,
                 opts: Optional[AdmmOptions] = None, stream=None):
        torch = _torch()
        self.opts = opts or AdmmOptions()
        fdt = torch.float64 if self.opts.precision == PREC_F64 else torch.float32
        N = X.dim()
        if not X.is_cuda or not X.is_contiguous() or not 3 <= N <= _lib.MAX_ORDER:
            raise ValueError(f"X must be a contiguous CUDA tensor with 3..{_lib.MAX_ORDER} dims")
        if X.dtype != fdt:
            raise ValueError(f"X must be {fdt} for this precision")
        if len(H) != N:
            raise ValueError("one factor per mode")
        F = H[0].shape[1]
        self.X, self.H, self.N, self.F = X, list(H), N, F
        self.dims = tuple(int(d) for d in X.shape)
        for n in range(N):
            h = self.H[n]
            if not h.is_cuda or h.dtype != fdt or not h.is_contiguous() or tuple(h.shape) != (self.dims[n], F):
                raise ValueError(f"H[{n}] must be a contiguous CUDA {fdt} tensor of shape ({self.dims[n]}, {F})")
        self.U = list(U) if U is not None else [torch.zeros_like(h) for h in self.H]
        for n in range(N):
            if self.U[n].shape != self.H[n].shape or self.U[n].dtype != fdt or not self.U[n].is_contiguous():
                raise ValueError(f"U[{n}] must match H[{n}]")
        L = _lib.lib()
        pr = _lib.NwayProblem()
        pr.order = N
        pr.F = F
        for n in range(N):
            pr.dims[n] = self.dims[n]
            pr.H[n] = _ptr(self.H[n])
            pr.U[n] = _ptr(self.U[n])
        pr.x_dtype = 1 if self.opts.precision == PREC_F64 else 0
        pr.X = _ptr(X)
        self._prob = pr
        self._copts = self.opts.to_c()
        nbytes = L.ntf_nway_workspace_bytes(ctypes.byref(pr), ctypes.byref(self._copts))
        if nbytes == 0:
            ctx = ctypes.c_void_p()
            st = L.ntf_nway_init(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts), None, 0,
                                 _stream_handle(stream))
            _lib.check(st, "ntf_nway_init", None, nway=True)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=X.device)
        ctx = ctypes.c_void_p()
        st = L.ntf_nway_init(ctypes.byref(ctx), ctypes.byref(pr), ctypes.byref(self._copts),
                             ctypes.c_void_p(_ptr(self.workspace)), nbytes, _stream_handle(stream))
        _lib.check(st, "ntf_nway_init", None, nway=True)
        self._ctx = ctx

    def _stats(self, s):
        d = s.as_dict()
        for k, v in d.items():
            if isinstance(v, list):
                d[k] = v[:self.N]
        return d

    def step(self, stats: bool = False):
        L = _lib.lib()
        if stats:
            s = _lib.NwayStats()
            _lib.check(L.ntf_nway_step(self._ctx, ctypes.byref(s)), "ntf_nway_step", self._ctx, nway=True)
            return self._stats(s)
        _lib.check(L.ntf_nway_step(self._ctx, None), "ntf_nway_step", self._ctx, nway=True)
        return None

    def run(self, max_outer: int, check_every: int = 1, stats: bool = True):
        s = _lib.NwayStats()
        st = _lib.lib().ntf_nway_run(self._ctx, int(max_outer), int(check_every),
                                     ctypes.byref(s) if stats else None)
        _lib.check(st, "ntf_nway_run", self._ctx, ok=(_lib.NTF_OK, _lib.NTF_NOT_CONVERGED), nway=True)
        out = self._stats(s) if stats else {}
        out["status"] = st
        return out

    def fit(self) -> float:
        r = ctypes.c_double()
        _lib.check(_lib.lib().ntf_nway_fit(self._ctx, ctypes.byref(r)), "ntf_nway_fit", self._ctx, nway=True)
        return r.value

    def mttkrp(self, mode: int):
        torch = _torch()
        W = torch.empty((self.dims[mode], self.F), dtype=torch.float64, device=self.X.device)
        _lib.check(_lib.lib().ntf_nway_mttkrp(self._ctx, int(mode), ctypes.c_void_p(_ptr(W))),
                   "ntf_nway_mttkrp", self._ctx, nway=True)
        return W

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.lib().ntf_nway_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sparse_pass_bytes(dims, F: int, nnz: int, precision: int) -> dict:
    """Bytes one sparse MTTKRP launch of each mode must move at least: the
    sorted non-zeros (three int32 indices and the value), the two other
    factors once, and W (FP64) written once."""
    es = 8 if precision == PREC_F64 else 4
    out = {}
    for m, name in enumerate(("mode1", "mode2", "mode3")):
        others = [d for q, d in enumerate(dims) if q != m]
        out[name] = nnz * (12 + es) + (others[0] + others[1]) * F * es + dims[m] * F * 8
    return out


def inner_update(W, H, U, G, rho: float = 0.0, T: int = 1, eps_abs: float = 0.0,
                 eps_rel: float = 0.0, want_iters: bool = False, want_ht: bool = False,
                 stream=None):
    """One mode update on given W (float64 [rows,F]) and G (float64 [F,F]):
    (G + rho I)^{-1} on the device, then up to T inner iterations per row
    on H, U (in place).  rho <= 0 selects trace(G)/F."""
    torch = _torch()
    rows, F = H.shape
    dtype = 1 if H.dtype == torch.float64 else 0
    L = _lib.lib()
    nb = L.ntf_inner_workspace_bytes(rows, F)
    ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=H.device)
    iters = torch.zeros(rows, dtype=torch.int32, device=H.device) if want_iters else None
    ht = torch.empty_like(H) if want_ht else None
    st = L.ntf_inner_update(_ptr(W), _ptr(H), _ptr(U), rows, F, dtype, _ptr(G), float(rho), int(T),
                            float(eps_abs), float(eps_rel),
                            ctypes.c_void_p(_ptr(iters)) if iters is not None else None,
                            ctypes.c_void_p(_ptr(ht)) if ht is not None else None,
                            ctypes.c_void_p(_ptr(ws)), nb, _stream_handle(stream))
    _lib.check(st, "ntf_inner_update")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return iters, ht


def inner_update_noalloc(W, H, U, G, rho: float = 0.0, T: int = 1, eps_abs: float = 0.0,
                         eps_rel: float = 0.0, iters=None, ht=None, stream=None):
    """inner_update without a workspace: the library keeps its scratch in a
    fixed device array per GPU (calls overlapping on one GPU race).  `iters`
    (int32 [rows]) and `ht` (like H) are optional caller-owned outputs; this
    call allocates nothing and does not synchronise."""
    torch = _torch()
    rows, F = H.shape
    dtype = 1 if H.dtype == torch.float64 else 0
    st = _lib.lib().ntf_inner_update_noalloc(
        _ptr(W), _ptr(H), _ptr(U), rows, F, dtype, _ptr(G), float(rho), int(T), float(eps_abs),
        float(eps_rel), ctypes.c_void_p(_ptr(iters)) if iters is not None else None,
        ctypes.c_void_p(_ptr(ht)) if ht is not None else None, _stream_handle(stream))
    _lib.check(st, "ntf_inner_update_noalloc")


def gram(H, stream=None):
    """H^T H accumulated in FP64 on the device."""
    torch = _torch()
    rows, F = H.shape
    dtype = 1 if H.dtype == torch.float64 else 0
    L = _lib.lib()
    nb = L.ntf_gram_workspace_bytes(rows, F)
    ws = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=H.device)
    G = torch.empty((F, F), dtype=torch.float64, device=H.device)
    st = L.ntf_gram(_ptr(H), rows, F, dtype, _ptr(G), ctypes.c_void_p(_ptr(ws)), nb,
                    _stream_handle(stream))
    _lib.check(st, "ntf_gram")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return G


def pass_bytes(dims, F: int, precision: int, x_elem_bytes: int = 4) -> dict:
    """Algorithmic HBM bytes of one launch of each MTTKRP kernel: the tensor
    copy the kernel streams (BF16 in the mixed-precision mode, else X itself)
    and the I x J x F intermediate X x_3 H_3 that the first pass writes and the
    mode-2 kernel reads.  Factor reads (at most a few MB, L2-resident) are
    not counted."""
    I, J, K = dims
    x_bytes = I * J * K * (2 if precision == PREC_BF16_MIXED else x_elem_bytes)
    t_bytes = I * J * F * (8 if precision == PREC_F64 else 4)
    return {"pass1": x_bytes + t_bytes, "mode2": t_bytes, "pass3": x_bytes}


class NtfBatch:
    """Many independent NTF problems of uneven shapes, factorised together:
    one persistent kernel per outer iteration over a global work list, each
    outer iteration one replay of a captured HIP graph (mixed precision only:
    BF16 MTTKRP with FP32 accumulation, FP32 Grams, FP64 inverse/solves).

    Xs: CUDA float32 tensors [I, J, K]; Hs: per problem three CUDA float32
    factors [d_n, F] (updated in place); Us: duals (zeros if omitted).
    """

    KIND_PASS1, KIND_MODE2, KIND_PASS3 = 0, 4, 7

    def __init__(self, Xs: Sequence, Hs: Sequence[Sequence], Us=None,
                 opts: Optional[AdmmOptions] = None, stream=None):
        torch = _torch()
        self.opts = opts or AdmmOptions(precision=PREC_BF16_MIXED)
        if self.opts.precision != PREC_BF16_MIXED:
            raise ValueError("the batched solver runs in PREC_BF16_MIXED only")
        n = len(Xs)
        if n < 1 or len(Hs) != n:
            raise ValueError("need one factor triple per tensor")
        self.X, self.H = list(Xs), [list(h) for h in Hs]
        self.U = [list(u) for u in Us] if Us is not None else \
            [[torch.zeros_like(h) for h in hs] for hs in self.H]
        probs = (_lib.Problem * n)()
        for p in range(n):
            X, H, U = self.X[p], self.H[p], self.U[p]
            if not X.is_cuda or X.dtype != torch.float32 or X.dim() != 3 or not X.is_contiguous():
                raise ValueError(f"X[{p}] must be a contiguous 3-way CUDA float32 tensor")
            F = H[0].shape[1]
            for m in range(3):
                for t, nm in ((H[m], "H"), (U[m], "U")):
                    if (not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous()
                            or tuple(t.shape) != (X.shape[m], F)):
                        raise ValueError(f"{nm}[{p}][{m}] must be contiguous CUDA float32 "
                                         f"({X.shape[m]}, {F})")
                probs[p].dims[m] = X.shape[m]
                probs[p].H[m] = _ptr(H[m])
                probs[p].U[m] = _ptr(U[m])
            probs[p].F = F
            probs[p].x_dtype = 0
            probs[p].X = _ptr(X)
        self.n = n
        self.Fs = [h[0].shape[1] for h in self.H]
        self._probs = probs
        self._copts = self.opts.to_c()
        L = _lib.lib()
        nbytes = L.ntf_batch_workspace_bytes(probs, n, ctypes.byref(self._copts))
        if nbytes == 0:
            ctx = ctypes.c_void_p()
            _lib.check(L.ntf_batch_init(ctypes.byref(ctx), probs, n, ctypes.byref(self._copts), None, 0,
                                        _stream_handle(stream)), "ntf_batch_init", None, batch=True)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.X[0].device)
        ctx = ctypes.c_void_p()
        _lib.check(L.ntf_batch_init(ctypes.byref(ctx), probs, n, ctypes.byref(self._copts),
                                    ctypes.c_void_p(_ptr(self.workspace)), nbytes,
                                    _stream_handle(stream)), "ntf_batch_init", None, batch=True)
        self._ctx = ctx

    def _check(self, st, where):
        return _lib.check(st, where, self._ctx, batch=True)

    def step(self, n_outer: int = 1):
        self._check(_lib.lib().ntf_batch_step(self._ctx, int(n_outer)), "ntf_batch_step")

    def sync(self) -> int:
        flags = ctypes.c_int32(0)
        st = _lib.lib().ntf_batch_sync(self._ctx, ctypes.byref(flags))
        self._check(st, "ntf_batch_sync")
        return flags.value

    def fit(self):
        import numpy as np
        out = (ctypes.c_double * self.n)()
        self._check(_lib.lib().ntf_batch_fit(self._ctx, out), "ntf_batch_fit")
        return np.array(out[:], dtype=np.float64)

    def mttkrp(self, prob: int, mode: int):
        torch = _torch()
        rows = self.X[prob].shape[mode]
        W = torch.empty((rows, self.Fs[prob]), dtype=torch.float64, device=self.X[prob].device)
        self._check(_lib.lib().ntf_batch_mttkrp(self._ctx, int(prob), int(mode), _ptr(W)),
                    "ntf_batch_mttkrp")
        return W

    def launch_kind(self, kind: int):
        self._check(_lib.lib().ntf_batch_launch_kind(self._ctx, int(kind)), "ntf_batch_launch_kind")

    @staticmethod
    def _tiles_to_list(arr, n):
        return [{"kind": t.kind, "ft": t.ft, "qbucket": t.qbucket, "mt": t.mt,
                 "item_elems": t.item_elems, "us": t.us} for t in arr[:n]]

    def autotune(self, reps: int = 3, cache_path: Optional[str] = None):
        """Times tile candidates per bucket, keeps the fastest; with a cache
        file, writes the choices there (JSON) for set_tiles on a later run."""
        cap = 64
        arr = (_lib.BatchTile * cap)()
        nout = ctypes.c_int32(0)
        self._check(_lib.lib().ntf_batch_autotune(self._ctx, int(reps), arr, cap, ctypes.byref(nout)),
                    "ntf_batch_autotune")
        tiles = self._tiles_to_list(arr, nout.value)
        if cache_path:
            import json
            with open(cache_path, "w") as fh:
                json.dump(tiles, fh, indent=1)
        return tiles

    def set_tiles(self, tiles):
        arr = (_lib.BatchTile * max(1, len(tiles)))()
        for i, t in enumerate(tiles):
            for k in ("kind", "ft", "qbucket", "mt", "item_elems", "us"):
                setattr(arr[i], k, t.get(k, 0))
        self._check(_lib.lib().ntf_batch_set_tiles(self._ctx, arr, len(tiles)), "ntf_batch_set_tiles")

    def tiles(self):
        cap = 64
        arr = (_lib.BatchTile * cap)()
        nout = ctypes.c_int32(0)
        self._check(_lib.lib().ntf_batch_get_tiles(self._ctx, arr, cap, ctypes.byref(nout)),
                    "ntf_batch_get_tiles")
        return self._tiles_to_list(arr, nout.value)

    KIND_NAMES = ("pass1", "prep1", "inner1", "prep2", "mode2", "inner2", "prep3", "pass3", "inner3")

    def profile(self) -> dict:
        """One instrumented outer iteration: per item kind, summed block time
        busy and waiting (microseconds) and the item count."""
        busy, wait, items = (ctypes.c_double * 9)(), (ctypes.c_double * 9)(), (ctypes.c_int64 * 9)()
        self._check(_lib.lib().ntf_batch_profile(self._ctx, busy, wait, items), "ntf_batch_profile")
        return {k: {"busy_us": busy[q], "wait_us": wait[q], "items": items[q]}
                for q, k in enumerate(self.KIND_NAMES)}

    def info(self) -> dict:
        i = _lib.BatchInfo()
        self._check(_lib.lib().ntf_batch_info_get(self._ctx, ctypes.byref(i)), "ntf_batch_info_get")
        return {"n_problems": i.n_problems, "grid": i.grid, "lds_bytes": i.lds_bytes,
                "n_items": i.n_items, "items_by_kind": list(i.items_by_kind),
                "x_bytes": i.x_bytes, "t_bytes": i.t_bytes}

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _lib.lib().ntf_batch_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

