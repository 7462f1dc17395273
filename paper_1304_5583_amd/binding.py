"""Thin ctypes binding of the gfx950 DFC-LRR library (include/lrr.h, include/lrr_diag.h,
include/lrr_segment.h, include/lrr_slr.h).

Argument marshalling only: every step of the solve runs in the HIP library.
Matrices are torch tensors on the GPU.  The library is column-major; a
column-major m x n matrix is exactly a row-major (n, m) tensor, so the helpers
below take and return *row-major tensors of the transposed shape* (``Mt`` of
shape (n, m) holds M).  ``to_device_colmajor`` / ``from_device_colmajor``
convert from/to ordinary (rows, cols) numpy arrays.

The library must be built (``python -m paper_1304_5583_amd.build``); loading
fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrr.so")

LRR_OK, LRR_NOT_CONVERGED = 0, 1
LRR_EINVAL, LRR_ENOMEM, LRR_EDEVICE, LRR_ENUMERIC, LRR_ENOTAPE = -1, -2, -3, -4, -5
LRR_FP64, LRR_FP32, LRR_MIXED_BF16 = 0, 1, 2
LRR_COORDS_AUTO, LRR_COORDS_FULL, LRR_COORDS_REDUCED = 0, 1, 2
LRR_SOLVE_AUTO, LRR_SOLVE_LITERAL, LRR_SOLVE_PUSHTHROUGH = 0, 1, 2
LRR_IO_FP64, LRR_IO_FP32 = 0, 1
STATUS_NAMES = {0: "LRR_OK", 1: "LRR_NOT_CONVERGED", -1: "LRR_EINVAL", -2: "LRR_ENOMEM",
                -3: "LRR_EDEVICE", -4: "LRR_ENUMERIC", -5: "LRR_ENOTAPE"}


class lrr_opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int), ("solve_form", C.c_int),
        ("mu0", C.c_double), ("rho", C.c_double), ("mu_max", C.c_double), ("tol", C.c_double),
        ("max_iter", C.c_int), ("fixed_iters", C.c_int), ("check_every", C.c_int),
        ("max_sweeps", C.c_int), ("save_for_backward", C.c_int), ("checkpoint_every", C.c_int),
        ("eig_block", C.c_int), ("use_graph", C.c_int), ("coords", C.c_int), ("tune", C.c_int),
        ("io_type", C.c_int), ("reserved", C.c_int * 3),
    ]


class lrr_seg_info(C.Structure):
    _fields_ = [
        ("rank", C.c_int), ("range_rank", C.c_int), ("sketch", C.c_int), ("embed_iters", C.c_int),
        ("embed_resid", C.c_double), ("theta_k", C.c_double), ("theta_k1", C.c_double),
        ("kmeans_iters", C.c_int), ("n_keep", C.c_int),
    ]


class lrr_slr_info(C.Structure):
    _fields_ = [("max_steps", C.c_int), ("not_converged", C.c_int), ("max_kkt", C.c_double),
                ("large_support", C.c_int), ("max_support", C.c_int)]


class lrr_info(C.Structure):
    _fields_ = [
        ("iters", C.POINTER(C.c_int)), ("rank", C.POINTER(C.c_int)),
        ("res_primal", C.POINTER(C.c_double)), ("res_coupling", C.POINTER(C.c_double)),
        ("batch_iters", C.c_int), ("combine_rank", C.c_int),
    ]


class LRRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblrr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1304_5583_amd.build`")
    lib = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    ip = C.POINTER(C.c_int)
    lib.lrr_version.restype = C.c_char_p
    lib.lrr_opts_default.argtypes = [C.POINTER(lrr_opts)]
    lib.lrr_opts_default.restype = None
    lib.lrr_ctx_create.argtypes = [i, C.POINTER(vp)]
    lib.lrr_ctx_create.restype = i
    lib.lrr_ctx_destroy.argtypes = [vp]
    lib.lrr_ctx_destroy.restype = None
    lib.lrr_last_error.argtypes = [vp]
    lib.lrr_last_error.restype = C.c_char_p
    lib.lrr_tune_load.argtypes = [vp, C.c_char_p]
    lib.lrr_tune_load.restype = i
    lib.lrr_check_partition.argtypes = [i, i, ip, ip]
    lib.lrr_check_partition.restype = i
    lib.lrr_workspace_bytes.argtypes = [i, i, i, ip, C.POINTER(lrr_opts), C.POINTER(C.c_size_t)]
    lib.lrr_workspace_bytes.restype = i
    lib.lrr_solve.argtypes = [vp, i, i, i, vp, i, vp, i, d, C.POINTER(lrr_opts), vp, i, vp, i,
                              C.POINTER(lrr_info), vp]
    lib.lrr_solve.restype = i
    lib.dfc_lrr_solve.argtypes = [vp, i, i, vp, i, d, i, ip, ip, C.POINTER(lrr_opts), vp, i, vp, i,
                                  C.POINTER(lrr_info), vp]
    lib.dfc_lrr_solve.restype = i
    lib.dfc_lrr_backward.argtypes = [vp, vp, i, C.POINTER(C.c_double), vp, i, vp]
    lib.dfc_lrr_backward.restype = i
    lib.lrr_diag_dgemm.argtypes = [vp, i, i, i, i, i, d, vp, i, vp, i, d, vp, i, vp]
    lib.lrr_diag_dgemm.restype = i
    lib.lrr_diag_gemm.argtypes = [vp, i, i, i, i, i, i, d, vp, i, vp, i, d, vp, i, vp]
    lib.lrr_diag_gemm.restype = i
    lib.lrr_diag_spd_inverse.argtypes = [vp, i, i, vp, i, vp, i, vp]
    lib.lrr_diag_spd_inverse.restype = i
    lib.lrr_diag_spd_inverse_noalloc.argtypes = [vp, i, i, vp, i, vp, i, vp]
    lib.lrr_diag_spd_inverse_noalloc.restype = i
    lib.lrr_diag_syevj.argtypes = [vp, i, ip, vp, i, C.c_long, vp, i, vp, i, ip, vp]
    lib.lrr_diag_syevj.restype = i
    lib.lrr_diag_plan_rounds.argtypes = [ip, i, i, ip, ip]
    lib.lrr_diag_plan_rounds.restype = i
    lib.dfc_lrr_solve_local.argtypes = [vp, i, i, vp, i, d, i, ip, ip, i, C.POINTER(lrr_opts), vp, i, vp, i,
                                        C.POINTER(lrr_info), vp]
    lib.dfc_lrr_solve_local.restype = i
    lib.lrr_slr_graph.argtypes = [vp, i, i, vp, i, vp, i, i, d, vp, vp, vp, C.POINTER(lrr_slr_info), vp]
    lib.lrr_slr_graph.restype = i
    lib.lrr_segment.argtypes = [vp, i, vp, i, i, vp, d, i, vp, C.POINTER(lrr_seg_info), vp]
    lib.lrr_segment.restype = i
    lib.lrr_outlier_flags.argtypes = [vp, i, i, vp, i, vp, i, d, vp, ip, vp]
    lib.lrr_outlier_flags.restype = i
    _lib = lib
    return lib


def lrr_version() -> str:
    return load_library().lrr_version().decode()


def lrr_opts_default(**overrides) -> lrr_opts:
    o = lrr_opts()
    load_library().lrr_opts_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


TUNE_TABLE = os.path.join(HERE, "tune_table.txt")


def lrr_tune_load(path: str | None = TUNE_TABLE, ctx: Context | None = None):
    """Load the autotuner's schedule table into the context (None clears it);
    solves with opts.tune = 1 then use the entry for their shape."""
    ctx = ctx or get_context(0)
    st = load_library().lrr_tune_load(ctx.handle, path.encode() if path is not None else None)
    _check(st, ctx, allow_nc=False)


def lrr_check_partition(n: int, perm, offsets) -> int:
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    return load_library().lrr_check_partition(int(n), len(offsets) - 1, _ip(perm), _ip(offsets))


def lrr_last_error(ctx=None) -> str:
    r = load_library().lrr_last_error(ctx.handle if ctx is not None else None)
    return r.decode() if r else ""


class Context:
    """Owns an lrr_ctx (device workspace) for one HIP device."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = C.c_void_p()
        st = lib.lrr_ctx_create(int(device), C.byref(h))
        if st != LRR_OK:
            raise LRRError(st, lib.lrr_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            load_library().lrr_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


_ctx_cache: dict[int, Context] = {}


def get_context(device: int = 0) -> Context:
    if device not in _ctx_cache:
        _ctx_cache[device] = Context(device)
    return _ctx_cache[device]


@dataclass
class SolveInfo:
    status: int
    iters: np.ndarray
    rank: np.ndarray
    res_primal: np.ndarray
    res_coupling: np.ndarray
    batch_iters: int
    combine_rank: int


def _make_info(t: int):
    it = np.zeros(t, dtype=np.int32)
    rk = np.zeros(t, dtype=np.int32)
    r1 = np.zeros(t, dtype=np.float64)
    r2 = np.zeros(t, dtype=np.float64)
    info = lrr_info(_ip(it), _ip(rk), r1.ctypes.data_as(C.POINTER(C.c_double)),
                    r2.ctypes.data_as(C.POINTER(C.c_double)), 0, 0)
    return info, (it, rk, r1, r2)


def _check(st: int, ctx: Context, allow_nc: bool = True):
    if st == LRR_OK or (allow_nc and st == LRR_NOT_CONVERGED):
        return
    raise LRRError(st, load_library().lrr_last_error(ctx.handle).decode())


def _stream(torch, device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_cuda_f64(torch, *ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError("expected contiguous float64 CUDA tensors")


def _io(torch, opts, *ts):
    """Element type of a forward call from its input tensors: float64 (the
    default) or float32 (opts.io_type = LRR_IO_FP32, float32 outputs); returns
    (opts to pass, output dtype)."""
    dts = {t.dtype for t in ts if t is not None}
    if dts == {torch.float32}:
        o = lrr_opts()
        C.pointer(o)[0] = opts
        o.io_type = LRR_IO_FP32
        for t in ts:
            if t is not None and (not t.is_cuda or not t.is_contiguous()):
                raise TypeError("expected contiguous float32 CUDA tensors")
        return o, torch.float32
    _require_cuda_f64(torch, *ts)
    return opts, torch.float64


def lrr_solve(At, Xt, lam: float, opts: lrr_opts | None = None, ctx: Context | None = None,
              want_E: bool = True):
    """Eq. (2) with one block.  At: (n, m) tensor holding A (m x n); Xt: (l, m)
    holding X (m x l).  Returns (Zt (l, n) holding Z, Et (l, m) or None, info).
    float32 A and X select FP32 I/O (float32 outputs, FP64 state)."""
    import torch
    opts, odt = _io(torch, opts or lrr_opts_default(), At, Xt)
    n, m = At.shape
    l, m2 = Xt.shape
    if m2 != m:
        raise ValueError("A and X must have the same number of rows")
    ctx = ctx or get_context(At.device.index or 0)
    Zt = torch.empty((l, n), dtype=odt, device=At.device)
    Et = torch.empty((l, m), dtype=odt, device=At.device) if want_E else None
    info, arrs = _make_info(1)
    st = load_library().lrr_solve(ctx.handle, m, n, l, C.c_void_p(At.data_ptr()), m,
                                  C.c_void_p(Xt.data_ptr()), m, float(lam), C.byref(opts),
                                  C.c_void_p(Zt.data_ptr()), n,
                                  C.c_void_p(Et.data_ptr()) if Et is not None else None, m,
                                  C.byref(info), _stream(torch, At.device))
    _check(st, ctx)
    return Zt, Et, SolveInfo(st, *arrs, info.batch_iters, info.combine_rank)


def dfc_lrr_solve(Mt, lam: float, perm, offsets, opts: lrr_opts | None = None,
                  ctx: Context | None = None, want_S: bool = True, Zt=None):
    """Algorithm 1.  Mt: (n, m) tensor holding M (m x n).  Returns
    (Zt (n, n) holding Z, St (n, m) holding S or None, info).  A float32 Mt
    selects FP32 I/O (float32 outputs, FP64 state inside)."""
    import torch
    opts, odt = _io(torch, opts or lrr_opts_default(), Mt)
    n, m = Mt.shape
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    t = len(offsets) - 1
    ctx = ctx or get_context(Mt.device.index or 0)
    if Zt is None:
        Zt = torch.empty((n, n), dtype=odt, device=Mt.device)
    elif Zt.dtype != odt or Zt.shape != (n, n) or not Zt.is_contiguous():
        raise TypeError("Zt must be a contiguous (n, n) tensor of the input's dtype")
    St = torch.empty((n, m), dtype=odt, device=Mt.device) if want_S else None
    info, arrs = _make_info(t)
    st = load_library().dfc_lrr_solve(ctx.handle, m, n, C.c_void_p(Mt.data_ptr()), m, float(lam), t,
                                      _ip(perm), _ip(offsets), C.byref(opts),
                                      C.c_void_p(Zt.data_ptr()), n,
                                      C.c_void_p(St.data_ptr()) if St is not None else None, m,
                                      C.byref(info), _stream(torch, Mt.device))
    _check(st, ctx)
    return Zt, St, SolveInfo(st, *arrs, info.batch_iters, info.combine_rank)


def dfc_lrr_solve_local(Mt, lam: float, perm, offsets, combine_rank: int = 0, opts: lrr_opts | None = None,
                        ctx: Context | None = None, want_S: bool = True, Zt=None):
    """Footnote variant of Section 2.2 (every block its own dictionary, truncated-SVD
    combine of diag(J_1..J_t)).  Same tensors and return value as dfc_lrr_solve."""
    import torch
    opts, odt = _io(torch, opts or lrr_opts_default(), Mt)
    n, m = Mt.shape
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    t = len(offsets) - 1
    ctx = ctx or get_context(Mt.device.index or 0)
    if Zt is None:
        Zt = torch.empty((n, n), dtype=odt, device=Mt.device)
    elif Zt.dtype != odt or Zt.shape != (n, n) or not Zt.is_contiguous():
        raise TypeError("Zt must be a contiguous (n, n) tensor of the input's dtype")
    St = torch.empty((n, m), dtype=odt, device=Mt.device) if want_S else None
    info, arrs = _make_info(t)
    st = load_library().dfc_lrr_solve_local(ctx.handle, m, n, C.c_void_p(Mt.data_ptr()), m, float(lam), t,
                                            _ip(perm), _ip(offsets), int(combine_rank), C.byref(opts),
                                            C.c_void_p(Zt.data_ptr()), n,
                                            C.c_void_p(St.data_ptr()) if St is not None else None, m,
                                            C.byref(info), _stream(torch, Mt.device))
    _check(st, ctx)
    return Zt, St, SolveInfo(st, *arrs, info.batch_iters, info.combine_rank)


def dfc_lrr_backward(dZt, ctx: Context | None = None, want_dM: bool = True, m: int | None = None):
    """Gradient of the last recorded dfc_lrr_solve: dZt (n, n) holds dL/dZ."""
    import torch
    _require_cuda_f64(torch, dZt)
    n = dZt.shape[0]
    ctx = ctx or get_context(dZt.device.index or 0)
    dlam = C.c_double(0.0)
    dMt = torch.empty((n, m), dtype=torch.float64, device=dZt.device) if (want_dM and m) else None
    st = load_library().dfc_lrr_backward(ctx.handle, C.c_void_p(dZt.data_ptr()), n, C.byref(dlam),
                                         C.c_void_p(dMt.data_ptr()) if dMt is not None else None,
                                         m or 1, _stream(torch, dZt.device))
    _check(st, ctx, allow_nc=False)
    return dlam.value, dMt


# ---------------------------------------------------------------- diagnostics

def lrr_diag_dgemm(ta: bool, tb: bool, A, B, Cm, M: int, N: int, K: int, lda: int, ldb: int, ldc: int,
                   alpha: float = 1.0, beta: float = 0.0, ctx: Context | None = None):
    import torch
    ctx = ctx or get_context(A.device.index or 0)
    st = load_library().lrr_diag_dgemm(ctx.handle, int(ta), int(tb), M, N, K, float(alpha),
                                       C.c_void_p(A.data_ptr()), lda, C.c_void_p(B.data_ptr()), ldb,
                                       float(beta), C.c_void_p(Cm.data_ptr()), ldc,
                                       _stream(torch, A.device))
    _check(st, ctx, allow_nc=False)


def lrr_diag_gemm(precision: int, ta: bool, tb: bool, A, B, Cm, M: int, N: int, K: int, lda: int, ldb: int,
                  ldc: int, alpha: float = 1.0, beta: float = 0.0, ctx: Context | None = None):
    import torch
    ctx = ctx or get_context(A.device.index or 0)
    st = load_library().lrr_diag_gemm(ctx.handle, int(precision), int(ta), int(tb), M, N, K, float(alpha),
                                      C.c_void_p(A.data_ptr()), lda, C.c_void_p(B.data_ptr()), ldb,
                                      float(beta), C.c_void_p(Cm.data_ptr()), ldc,
                                      _stream(torch, A.device))
    _check(st, ctx, allow_nc=False)


def lrr_diag_spd_inverse(At, ctx: Context | None = None):
    """At: (n, m) holding A (m x n).  Returns (m, m) tensor holding (I + A A^T)^{-1}
    (symmetric, so the layout question does not arise)."""
    import torch
    n, m = At.shape
    ctx = ctx or get_context(At.device.index or 0)
    K = torch.empty((m, m), dtype=torch.float64, device=At.device)
    st = load_library().lrr_diag_spd_inverse(ctx.handle, m, n, C.c_void_p(At.data_ptr()), m,
                                             C.c_void_p(K.data_ptr()), m, _stream(torch, At.device))
    _check(st, ctx, allow_nc=False)
    return K


def lrr_diag_plan_rounds(need, cap: int):
    """Round schedule of a targeted Jacobi pass for the nb x nb marks `need`
    (host only).  Returns (rounds, pairs) with pairs an int array (cap, nb/2, 2)
    of which the first `rounds` rows are used; rounds = -1 if cap is too small."""
    need = np.ascontiguousarray(need, dtype=np.int32)
    nb = need.shape[0]
    out = np.zeros(max(cap, 1) * max(nb // 2, 1), dtype=np.int32)
    r = np.zeros(1, dtype=np.int32)
    st = load_library().lrr_diag_plan_rounds(_ip(need), nb, cap, _ip(out), _ip(r))
    if st != LRR_OK:
        raise LRRError(st, "lrr_diag_plan_rounds: invalid arguments")
    v = out[:cap * (nb // 2)].reshape(cap, nb // 2)
    return int(r[0]), np.stack([v & 0xffff, v >> 16], axis=-1)


def lrr_diag_syevj(Bs, ls, eig_block: int = 16, ctx: Context | None = None):
    """Bs: (count, ld, ld) symmetric matrices (row/col-major agree); ls: orders.
    Returns (lam (count, ld), W (count, ld, ld) with W[b].T[:, j] the j-th
    eigenvector of the leading ls[b] block, sweeps)."""
    import torch
    count, ld, ld2 = Bs.shape
    assert ld == ld2
    ctx = ctx or get_context(Bs.device.index or 0)
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    lam = torch.zeros((count, ld), dtype=torch.float64, device=Bs.device)
    W = torch.zeros_like(Bs)
    sw = C.c_int(0)
    st = load_library().lrr_diag_syevj(ctx.handle, count, _ip(ls), C.c_void_p(Bs.data_ptr()), ld,
                                       ld * ld, C.c_void_p(lam.data_ptr()), ld,
                                       C.c_void_p(W.data_ptr()), eig_block, C.byref(sw),
                                       _stream(torch, Bs.device))
    _check(st, ctx, allow_nc=False)
    return lam, W, sw.value


def lrr_segment(Zt, k: int, exclude=None, rank_tol: float = 1e-6, rank_bound: int = 0,
                ctx: Context | None = None):
    """Cluster labels of the n points from Z (Section 4.1.2 pipeline, include/lrr_segment.h).

    Zt: (n, n) float64 CUDA tensor holding the column-major Z (as returned by
    ``lrr_solve`` / ``dfc_lrr_solve``).  exclude: None or a length-n bool/uint8
    array or tensor (True: point left out, label -1).  Returns (labels, info)
    with labels an int64 CUDA tensor of length n and info a dict of
    ``lrr_seg_info``; info["converged"] is False when the call returned
    LRR_NOT_CONVERGED."""
    import torch
    _require_cuda_f64(torch, Zt)
    n = Zt.shape[0]
    if Zt.shape != (n, n):
        raise ValueError("Zt must be square")
    ctx = ctx or get_context(Zt.device.index or 0)
    ex = None
    if exclude is not None:
        ex = torch.as_tensor(np.asarray(exclude.cpu() if torch.is_tensor(exclude) else exclude).astype(np.uint8),
                             device=Zt.device)
        if ex.numel() != n:
            raise ValueError("exclude must have n entries")
    labels = torch.empty(n, dtype=torch.int64, device=Zt.device)
    info = lrr_seg_info()
    st = load_library().lrr_segment(ctx.handle, n, C.c_void_p(Zt.data_ptr()), int(Zt.stride(0)), int(k),
                                    C.c_void_p(ex.data_ptr()) if ex is not None else None, float(rank_tol),
                                    int(rank_bound), C.c_void_p(labels.data_ptr()), C.byref(info),
                                    _stream(torch, Zt.device))
    _check(st, ctx, allow_nc=True)
    out = {f: getattr(info, f) for f, _ in lrr_seg_info._fields_}
    out["converged"] = st == LRR_OK
    return labels, out


def lrr_outlier_flags(Mt, St, delta: float, ctx: Context | None = None):
    """Columns the outlier estimate marks (include/lrr_segment.h): Mt and St are
    (n, m) tensors holding M and S (m x n).  Returns (flags, count) with flags a
    bool CUDA tensor of length n: ||S[:, j]|| > delta ||M[:, j]||."""
    import torch
    _require_cuda_f64(torch, Mt, St)
    n, m = Mt.shape
    if St.shape != (n, m):
        raise ValueError("M and S must have the same shape")
    ctx = ctx or get_context(Mt.device.index or 0)
    flags = torch.empty(n, dtype=torch.uint8, device=Mt.device)
    cnt = C.c_int(0)
    st = load_library().lrr_outlier_flags(ctx.handle, m, n, C.c_void_p(Mt.data_ptr()), m,
                                          C.c_void_p(St.data_ptr()), m, float(delta),
                                          C.c_void_p(flags.data_ptr()), C.byref(cnt), _stream(torch, Mt.device))
    _check(st, ctx, allow_nc=False)
    return flags.bool(), cnt.value


def lrr_slr_graph(Mt, Zt, nk: int, alpha: float = 0.05, want_obj: bool = True, ctx: Context | None = None):
    """SLR-graph of Section 4.2.2 (include/lrr_slr.h).  Mt: (n, m) tensor holding M,
    Zt: (n, n) tensor holding the column-major Z.  Returns (nbr (n, nk) int32,
    w (n, nk) float64, obj (n,) float64 or None, info dict); row i of nbr / w
    lists sample i's neighbours and edge weights."""
    import torch
    _require_cuda_f64(torch, Mt, Zt)
    n, m = Mt.shape
    if Zt.shape != (n, n):
        raise ValueError("Zt must be n x n")
    ctx = ctx or get_context(Mt.device.index or 0)
    nbr = torch.empty((n, nk), dtype=torch.int32, device=Mt.device)
    w = torch.empty((n, nk), dtype=torch.float64, device=Mt.device)
    obj = torch.empty(n, dtype=torch.float64, device=Mt.device) if want_obj else None
    info = lrr_slr_info()
    st = load_library().lrr_slr_graph(ctx.handle, m, n, C.c_void_p(Mt.data_ptr()), m, C.c_void_p(Zt.data_ptr()),
                                      int(Zt.stride(0)), int(nk), float(alpha), C.c_void_p(nbr.data_ptr()),
                                      C.c_void_p(w.data_ptr()), C.c_void_p(obj.data_ptr()) if obj is not None else None,
                                      C.byref(info), _stream(torch, Mt.device))
    _check(st, ctx, allow_nc=True)
    out = {f: getattr(info, f) for f, _ in lrr_slr_info._fields_}
    out["converged"] = st == LRR_OK
    return nbr, w, obj, out


# ---------------------------------------------------------------- layout helpers

def to_device_colmajor(A: np.ndarray, device="cuda"):
    """(rows, cols) numpy array -> (cols, rows) float64 tensor = column-major A."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).to(device)


def from_device_colmajor(t) -> np.ndarray:
    """(cols, rows) tensor holding a column-major matrix -> (rows, cols) numpy."""
    return t.detach().cpu().numpy().T.copy()
