"""MI355X-native HODLRdD matrix-vector product.

Thin ctypes binding of ``libhodlr.so`` (C ABI in ``include/hodlr.h``).  The
functions below only marshal arguments: every step of the method (tree,
interaction lists, ACA, apply, near field) runs in the library's HIP kernels.
PyTorch supplies device memory and streams.  There is no CPU fallback: if the
library is not built, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhodlr.so")

FP64, FP32, BF16 = 0, 1, 2
KERNELS = {"log": 0, "inv_r": 1, "inv_r2": 2, "gauss": 3, "exp": 4, "r": 5, "sin": 6,
           "inv_sqrt1p": 7}
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EDUPLICATE", 5: "ENONFINITE",
          6: "EUNSUPPORTED"}


class HodlrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_double), ("scale", C.c_double), ("diag", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("level_rule", C.c_int), ("has_domain", C.c_int),
                ("domain_lo", C.c_double * 8), ("domain_side", C.c_double),
                ("storage", C.c_int), ("symmetric", C.c_int), ("max_rank", C.c_int),
                ("skip_aca", C.c_int), ("mem_budget_bytes", C.c_size_t), ("adm_dim", C.c_int),
                ("skeleton", C.c_int)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int64), ("d", C.c_int), ("kappa", C.c_int), ("lmax", C.c_int),
                ("symmetric", C.c_int), ("storage", C.c_int),
                ("domain_lo", C.c_double * 8), ("domain_side", C.c_double),
                ("nboxes", C.c_int64 * 32), ("il_entries", C.c_int64 * 32),
                ("stored_blocks", C.c_int64 * 32), ("rank_min", C.c_int32 * 32),
                ("rank_max", C.c_int32 * 32), ("rank_mean", C.c_double * 32),
                ("factor_elems", C.c_int64 * 32), ("class_blocks", C.c_int64 * 8),
                ("class_factor_elems", C.c_int64 * 8), ("class_vector_elems", C.c_int64 * 8),
                ("split_blocks", C.c_int64), ("split_factor_elems", C.c_int64),
                ("near_entries", C.c_int64),
                ("near_pairs", C.c_int64), ("device_bytes", C.c_size_t),
                ("build_ms", C.c_double * 4),
                ("mfma_proj_jobs", C.c_int64 * 4), ("mfma_proj_factor_elems", C.c_int64 * 4),
                ("mfma_proj_vector_elems", C.c_int64 * 4), ("mfma_expand_factor_elems", C.c_int64),
                ("mfma_proj_elems", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("route", C.c_int), ("class_choice", C.c_int * 8), ("class_ms", C.c_double * 8),
                ("class_route_ms", C.c_double), ("persistent_ms", C.c_double),
                ("seg_side", C.c_int), ("one_stream_ms", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("restart", C.c_int),
                ("max_outer", C.c_int), ("lo_compute", C.c_int), ("use_initial_guess", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("inner_iters", C.c_int), ("converged", C.c_int),
                ("rel_residual", C.c_double), ("history", C.c_double * 64)]


class ServerOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_size_t), ("max_concurrent", C.c_int),
                ("max_batch_cols", C.c_int), ("max_points", C.c_int64), ("multiset", C.c_int)]


class Request(C.Structure):
    _fields_ = [("kind", C.c_int), ("set", C.c_int), ("nrhs", C.c_int), ("X", C.c_void_p),
                ("Y", C.c_void_p), ("alpha", C.c_double), ("beta", C.c_double),
                ("tol", C.c_double), ("stream", C.c_void_p)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("launches", C.c_int64), ("batched_requests", C.c_int64),
                ("multiset_launches", C.c_int64),
                ("max_concurrent", C.c_int64), ("used_bytes", C.c_size_t),
                ("budget_bytes", C.c_size_t), ("sets", C.c_int)]


REQ_MATVEC, REQ_SOLVE = 0, 1

_lib = None
_P = C.c_void_p
_i64 = C.c_int64


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "paper_2209_05819_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.hodlr_default_opts.argtypes = [C.POINTER(Opts)]
        L.hodlr_build.argtypes = [_P, _i64, C.c_int, C.POINTER(Kernel), C.c_int, C.c_double,
                                  C.POINTER(Opts), _P, C.POINTER(_P)]
        L.hodlr_matvec.argtypes = [_P, _P, _i64, C.c_int, C.c_int, _P, _i64, C.c_int, _P]
        L.hodlr_matvec_events.argtypes = [_P, _P, _i64, C.c_int, C.c_int, _P, _i64, C.c_int, _P,
                                          C.POINTER(_P), C.c_int]
        L.hodlr_matvec_noalloc.argtypes = [_P, _P, _i64, C.c_int, C.c_int, _P, _i64, C.c_int, _P]
        L.hodlr_set_route.argtypes = [_P, C.c_int]
        L.hodlr_autotune.argtypes = [_P, C.c_int, C.c_int, C.c_int, C.POINTER(Tuning), _P]
        L.hodlr_matvec_batch.argtypes = [C.c_int, _P, _P, _P, _P, C.c_int, _P, _P, _P]
        L.hodlr_get_info.argtypes = [_P, C.POINTER(Info)]
        L.hodlr_server_default_opts.argtypes = [C.POINTER(ServerOpts)]
        L.hodlr_server_default_opts.restype = None
        L.hodlr_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(_P)]
        L.hodlr_server_add_set.argtypes = [_P, _P, _i64, C.c_int, C.POINTER(Kernel), C.c_int,
                                           C.c_double, C.POINTER(Opts), C.POINTER(C.c_int)]
        L.hodlr_server_submit.argtypes = [_P, C.POINTER(Request), C.POINTER(_i64)]
        L.hodlr_server_wait.argtypes = [_P, _i64, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.hodlr_server_poll.argtypes = [_P, _i64, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.hodlr_server_get_stats.argtypes = [_P, C.POINTER(ServerStats)]
        L.hodlr_server_destroy.argtypes = [_P]
        L.hodlr_server_destroy.restype = None
        L.hodlr_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
        L.hodlr_default_solve_opts.restype = None
        L.hodlr_solve.argtypes = [_P, _P, C.c_double, C.c_double, _P, _i64, C.c_int, _P, _i64,
                                  C.POINTER(SolveOpts), C.POINTER(SolveInfo), _P]
        L.hodlr_export_tree.argtypes = [_P, _P, _P]
        L.hodlr_export_boxes.argtypes = [_P, C.c_int, _P, _P, _P]
        L.hodlr_export_il.argtypes = [_P, C.c_int, C.POINTER(_i64), _P, _P]
        L.hodlr_export_near.argtypes = [_P, C.POINTER(_i64), _P, _P]
        L.hodlr_export_near_level.argtypes = [_P, C.c_int, C.POINTER(_i64), _P, _P]
        L.hodlr_export_box_flags.argtypes = [_P, C.c_int, _P]
        L.hodlr_reserve_workspace.argtypes = [_P, C.c_int, C.c_int]
        L.hodlr_mfma_extent.argtypes = [_i64, _i64, C.c_int, C.POINTER(_i64)]
        L.hodlr_export_factors.argtypes = [_P, C.c_int, _P, C.POINTER(_i64), C.POINTER(_i64),
                                           _P, _P]
        L.hodlr_import_factors.argtypes = [_P, C.c_int, _P, _P, _P]
        L.hodlr_destroy.argtypes = [_P]
        L.hodlr_last_error.restype = C.c_char_p
        for f in ("hodlr_build", "hodlr_matvec", "hodlr_matvec_events", "hodlr_matvec_noalloc",
                  "hodlr_set_route", "hodlr_matvec_batch", "hodlr_autotune",
                  "hodlr_get_info",
                  "hodlr_export_tree",
                  "hodlr_export_boxes", "hodlr_export_il", "hodlr_export_near",
                  "hodlr_export_near_level", "hodlr_export_box_flags", "hodlr_reserve_workspace",
                  "hodlr_mfma_extent",
                  "hodlr_export_factors", "hodlr_import_factors", "hodlr_solve",
                  "hodlr_server_create", "hodlr_server_add_set", "hodlr_server_submit",
                  "hodlr_server_wait", "hodlr_server_poll", "hodlr_server_get_stats"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise HodlrError(st, lib().hodlr_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_opts() -> Opts:
    o = Opts()
    lib().hodlr_default_opts(C.byref(o))
    return o


def make_kernel(kind, h: float = 1.0, scale: float = 1.0, diag: float = 0.0) -> Kernel:
    return Kernel(KERNELS[kind] if isinstance(kind, str) else int(kind), float(h), float(scale),
                  float(diag))


def _stream_ptr(stream):
    """A hipStream_t from None (torch's current stream), a torch stream or an
    integer handle."""
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def hodlr_build(points, kernel: Kernel, leaf_size: int, tol: float,
                opts: Opts | None = None, stream=None) -> int:
    """points: N x d float64, a host array or a contiguous device tensor."""
    if _is_device_tensor(points):
        import torch
        if points.dtype != torch.float64 or points.dim() != 2 or not points.is_contiguous():
            raise TypeError("device points must be a contiguous N x d float64 tensor")
        N, d = points.shape
        ptr = C.c_void_p(points.data_ptr())
    else:
        points = np.ascontiguousarray(points, dtype=np.float64)
        N, d = points.shape
        ptr = _np_ptr(points)
    out = C.c_void_p()
    _check(lib().hodlr_build(ptr, N, d, C.byref(kernel), int(leaf_size), float(tol),
                             C.byref(opts) if opts is not None else None, _stream_ptr(stream),
                             C.byref(out)))
    return out.value


def hodlr_mfma_extent(rank: int, length: int, nrhs: int) -> tuple[int, int]:
    """(status, largest byte offset) of the matrix-core product for one BF16
    factor; host computation, no device needed."""
    ext = _i64()
    st = lib().hodlr_mfma_extent(int(rank), int(length), int(nrhs), C.byref(ext))
    return st, ext.value


def _is_device_tensor(x) -> bool:
    return type(x).__module__.startswith("torch") and getattr(x, "is_cuda", False)


def hodlr_matvec(h: int, X, Y, compute_prec: int = FP64, stream=None) -> None:
    """Y = K~ X for torch tensors on the GPU: N x nrhs, column-major
    (a (nrhs, N) contiguous tensor transposed, or a 1-D vector)."""
    import torch
    if X.dtype != Y.dtype or X.dtype not in (torch.float64, torch.float32):
        raise TypeError("X and Y must both be float64 or float32")
    if not (X.is_cuda and Y.is_cuda):
        raise TypeError("X and Y must be device tensors")
    xp = FP64 if X.dtype == torch.float64 else FP32
    if X.dim() == 1:
        N, nrhs, ldx, ldy = X.shape[0], 1, X.shape[0], Y.shape[0]
    else:
        N, nrhs = X.shape
        if X.stride(0) != 1 or Y.stride(0) != 1:
            raise ValueError("X and Y must be column-major (stride 1 along N)")
        ldx, ldy = X.stride(1) if nrhs > 1 else N, Y.stride(1) if nrhs > 1 else N
    _check(lib().hodlr_matvec(C.c_void_p(h), C.c_void_p(X.data_ptr()), ldx, nrhs, xp,
                              C.c_void_p(Y.data_ptr()), ldy, compute_prec, _stream_ptr(stream)))


def hodlr_matvec_noalloc(h: int, X, Y, compute_prec: int = FP64, stream=None) -> None:
    """hodlr_matvec with the library's static scratch array as workspace and
    the near field on the same stream: allocates nothing (for callers that
    cannot); calls on one GPU must not overlap."""
    import torch
    if X.dtype != Y.dtype or X.dtype not in (torch.float64, torch.float32):
        raise TypeError("X and Y must both be float64 or float32")
    if not (X.is_cuda and Y.is_cuda):
        raise TypeError("X and Y must be device tensors")
    xp = FP64 if X.dtype == torch.float64 else FP32
    if X.dim() == 1:
        nrhs, ldx, ldy = 1, X.shape[0], Y.shape[0]
    else:
        N, nrhs = X.shape
        if X.stride(0) != 1 or Y.stride(0) != 1:
            raise ValueError("X and Y must be column-major (stride 1 along N)")
        ldx, ldy = X.stride(1) if nrhs > 1 else N, Y.stride(1) if nrhs > 1 else N
    _check(lib().hodlr_matvec_noalloc(C.c_void_p(h), C.c_void_p(X.data_ptr()), ldx, nrhs, xp,
                                      C.c_void_p(Y.data_ptr()), ldy, compute_prec,
                                      _stream_ptr(stream)))


def hodlr_set_route(h: int, route: int) -> None:
    """0: per-stage, per-class launches, the near field on a second stream;
    1: one persistent launch per product; 2: the per-class launches on the
    caller's stream only; -1: not chosen (route 0, the default)."""
    _check(lib().hodlr_set_route(C.c_void_p(h), int(route)))


def hodlr_autotune(h: int, nrhs: int = 1, x_prec: int = FP64, compute_prec: int = FP64,
                   stream=None) -> Tuning:
    """Time the block classes' tile shapes and the two product routes on this
    handle and keep the fastest (synchronous)."""
    t = Tuning()
    _check(lib().hodlr_autotune(C.c_void_p(h), int(nrhs), int(x_prec), int(compute_prec),
                                C.byref(t), _stream_ptr(stream)))
    return t


def _cols(X):
    if X.dim() == 1:
        return 1, X.shape[0]
    if X.stride(0) != 1:
        raise ValueError("X and Y must be column-major (stride 1 along N)")
    return X.shape[1], (X.stride(1) if X.shape[1] > 1 else X.shape[0])


def hodlr_matvec_batch(hs, Xs, Ys, stream=None) -> None:
    """Y[t] = K~_t X[t] for several handles in one persistent launch (device
    tensors, all float64 or all float32; handles all FP64 or all FP32)."""
    import torch
    n = len(hs)
    if not (len(Xs) == len(Ys) == n) or n < 1:
        raise ValueError("one X and one Y per handle")
    dt = Xs[0].dtype
    if dt not in (torch.float64, torch.float32):
        raise TypeError("X and Y must be float64 or float32")
    ha = (C.c_void_p * n)(*[C.c_void_p(h) for h in hs])
    xa = (C.c_void_p * n)(*[C.c_void_p(x.data_ptr()) for x in Xs])
    ya = (C.c_void_p * n)(*[C.c_void_p(y.data_ptr()) for y in Ys])
    ldx = (C.c_int64 * n)()
    ldy = (C.c_int64 * n)()
    nr = (C.c_int * n)()
    for t in range(n):
        if Xs[t].dtype != dt or Ys[t].dtype != dt or not (Xs[t].is_cuda and Ys[t].is_cuda):
            raise TypeError("every X and Y a device tensor of one dtype")
        nr[t], ldx[t] = _cols(Xs[t])
        _, ldy[t] = _cols(Ys[t])
    _check(lib().hodlr_matvec_batch(n, ha, xa, ldx, nr, FP64 if dt == torch.float64 else FP32,
                                    ya, ldy, _stream_ptr(stream)))


def hodlr_reserve_workspace(h: int, nrhs: int, compute_prec: int = FP64) -> None:
    """Reserve the product workspace so that later products with at most
    nrhs columns only launch kernels (capturable into a HIP graph)."""
    _check(lib().hodlr_reserve_workspace(C.c_void_p(h), nrhs, compute_prec))


def _mv_args(X, Y):
    import torch
    if X.dtype != Y.dtype or X.dtype not in (torch.float64, torch.float32):
        raise TypeError("X and Y must both be float64 or float32")
    if not (X.is_cuda and Y.is_cuda):
        raise TypeError("X and Y must be device tensors")
    xp = FP64 if X.dtype == torch.float64 else FP32
    if X.dim() == 1:
        return xp, 1, X.shape[0], Y.shape[0]
    N, nrhs = X.shape
    if X.stride(0) != 1 or Y.stride(0) != 1:
        raise ValueError("X and Y must be column-major (stride 1 along N)")
    return xp, nrhs, (X.stride(1) if nrhs > 1 else N), (Y.stride(1) if nrhs > 1 else N)


def hodlr_matvec_events(h: int, X, Y, events, compute_prec: int = FP64, stream=None) -> None:
    """hodlr_matvec recording 5 or 11 torch.cuda.Event (enable_timing=True)
    at the stage boundaries on the stream (see hodlr_matvec_events)."""
    xp, nrhs, ldx, ldy = _mv_args(X, Y)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    for e in events:
        if e.cuda_event == 0:   # torch creates the event lazily
            e.record()
    arr = (C.c_void_p * len(events))(*[C.c_void_p(e.cuda_event) for e in events])
    _check(lib().hodlr_matvec_events(C.c_void_p(h), C.c_void_p(X.data_ptr()), ldx, nrhs, xp,
                                     C.c_void_p(Y.data_ptr()), ldy, compute_prec,
                                     C.c_void_p(int(stream)), arr, len(events)))


def default_solve_opts() -> SolveOpts:
    o = SolveOpts()
    lib().hodlr_default_solve_opts(C.byref(o))
    return o


def hodlr_solve(hi: int, lo: int, alpha: float, beta: float, F, U, opts: SolveOpts | None = None,
                stream=None) -> SolveInfo:
    """(alpha I + beta K~) U = F for float64 device tensors F, U (N or N x nrhs,
    column-major): FP64 refinement with `hi`, inner GMRES with `lo`."""
    import torch
    if F.dtype != torch.float64 or U.dtype != torch.float64 or not (F.is_cuda and U.is_cuda):
        raise TypeError("F and U must be float64 device tensors")
    if F.dim() == 1:
        N, nrhs, ldf, ldu = F.shape[0], 1, F.shape[0], U.shape[0]
    else:
        N, nrhs = F.shape
        if F.stride(0) != 1 or U.stride(0) != 1:
            raise ValueError("F and U must be column-major (stride 1 along N)")
        ldf, ldu = (F.stride(1) if nrhs > 1 else N), (U.stride(1) if nrhs > 1 else N)
    info = SolveInfo()
    _check(lib().hodlr_solve(C.c_void_p(hi), C.c_void_p(lo), C.c_double(alpha), C.c_double(beta),
                             C.c_void_p(F.data_ptr()), C.c_int64(ldf), nrhs,
                             C.c_void_p(U.data_ptr()), C.c_int64(ldu),
                             C.byref(opts) if opts is not None else None, C.byref(info),
                             _stream_ptr(stream)))
    return info


def hodlr_get_info(h: int) -> Info:
    info = Info()
    _check(lib().hodlr_get_info(C.c_void_p(h), C.byref(info)))
    return info


def hodlr_export_tree(h: int, N: int):
    perm = np.empty(N, dtype=np.int64)
    keys = np.empty(N, dtype=np.uint64)
    _check(lib().hodlr_export_tree(C.c_void_p(h), _np_ptr(perm), _np_ptr(keys)))
    return perm, keys


def hodlr_export_boxes(h: int, level: int, nb: int, d: int):
    start = np.empty(nb + 1, dtype=np.int64)
    key = np.empty(max(nb, 1), dtype=np.uint64)
    coord = np.empty((max(nb, 1), d), dtype=np.int32)
    _check(lib().hodlr_export_boxes(C.c_void_p(h), level, _np_ptr(start), _np_ptr(key),
                                    _np_ptr(coord)))
    return start, key[:nb], coord[:nb]


def hodlr_export_il(h: int, level: int, nb: int):
    nnz = C.c_int64()
    _check(lib().hodlr_export_il(C.c_void_p(h), level, C.byref(nnz), None, None))
    ptr = np.empty(nb + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().hodlr_export_il(C.c_void_p(h), level, C.byref(nnz), _np_ptr(ptr), _np_ptr(col)))
    return ptr, col[:nnz.value]


def hodlr_export_near(h: int, nb: int):
    nnz = C.c_int64()
    _check(lib().hodlr_export_near(C.c_void_p(h), C.byref(nnz), None, None))
    ptr = np.empty(nb + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().hodlr_export_near(C.c_void_p(h), C.byref(nnz), _np_ptr(ptr), _np_ptr(col)))
    return ptr, col[:nnz.value]


def hodlr_export_near_level(h: int, level: int, nb: int):
    nnz = C.c_int64()
    _check(lib().hodlr_export_near_level(C.c_void_p(h), level, C.byref(nnz), None, None))
    ptr = np.empty(nb + 1, dtype=np.int64)
    col = np.empty(max(nnz.value, 1), dtype=np.int32)
    _check(lib().hodlr_export_near_level(C.c_void_p(h), level, C.byref(nnz), _np_ptr(ptr),
                                         _np_ptr(col)))
    return ptr, col[:nnz.value]


def hodlr_export_box_flags(h: int, level: int, nb: int):
    f = np.empty(max(nb, 1), dtype=np.uint8)
    _check(lib().hodlr_export_box_flags(C.c_void_p(h), level, _np_ptr(f)))
    return f[:nb]


def hodlr_export_factors(h: int, level: int, nnz: int):
    ranks = np.empty(max(nnz, 1), dtype=np.int32)
    nu, nv = C.c_int64(), C.c_int64()
    _check(lib().hodlr_export_factors(C.c_void_p(h), level, _np_ptr(ranks), C.byref(nu),
                                      C.byref(nv), None, None))
    U = np.empty(max(nu.value, 1))
    V = np.empty(max(nv.value, 1))
    _check(lib().hodlr_export_factors(C.c_void_p(h), level, None, None, None, _np_ptr(U),
                                      _np_ptr(V)))
    return ranks[:nnz], U[:nu.value], V[:nv.value]


def hodlr_export_ranks(h: int, level: int, nnz: int):
    """ranks of the interaction-list entries of a level (any storage form)"""
    ranks = np.empty(max(nnz, 1), dtype=np.int32)
    nu, nv = C.c_int64(), C.c_int64()
    _check(lib().hodlr_export_factors(C.c_void_p(h), level, _np_ptr(ranks), C.byref(nu),
                                      C.byref(nv), None, None))
    return ranks[:nnz]


def hodlr_import_factors(h: int, level: int, ranks, U, V) -> None:
    r = np.ascontiguousarray(ranks, dtype=np.int32)
    Ua = np.ascontiguousarray(U, dtype=np.float64)
    Va = np.ascontiguousarray(V, dtype=np.float64)
    _check(lib().hodlr_import_factors(C.c_void_p(h), level, _np_ptr(r), _np_ptr(Ua), _np_ptr(Va)))


def hodlr_destroy(h: int) -> None:
    if h:
        lib().hodlr_destroy(C.c_void_p(h))


class HODLR:
    """Owning wrapper: build on construction, destroy when collected."""

    def __init__(self, points, kernel: Kernel, leaf_size: int, tol: float, *, level_rule=1,
                 domain=None, storage=FP64, symmetric=True, max_rank=0, skip_aca=False,
                 mem_budget_bytes=0, adm_dim=0, skeleton=False, stream=None):
        o = default_opts()
        o.level_rule = level_rule
        o.adm_dim = int(adm_dim)
        o.skeleton = 1 if skeleton else 0
        if domain is not None:
            o.has_domain = 1
            lo = np.asarray(domain[0], dtype=np.float64)
            for a in range(len(lo)):
                o.domain_lo[a] = lo[a]
            o.domain_side = float(domain[1])
        o.storage = storage
        o.symmetric = 1 if symmetric else 0
        o.max_rank = int(max_rank)
        o.skip_aca = 1 if skip_aca else 0
        o.mem_budget_bytes = int(mem_budget_bytes)
        self.points = points if _is_device_tensor(points) else np.ascontiguousarray(
            points, dtype=np.float64)
        self.N, self.d = self.points.shape
        self.h = hodlr_build(self.points, kernel, leaf_size, tol, o, stream)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                hodlr_destroy(h)
            except Exception:   # interpreter shutdown: the module may be gone
                pass
            self.h = None

    def info(self) -> Info:
        return hodlr_get_info(self.h)

    def matvec(self, X, compute_prec: int = FP64, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty_like(X) if X.dim() == 1 else torch.empty(
                (X.shape[1], X.shape[0]), dtype=X.dtype, device=X.device).t()
        hodlr_matvec(self.h, X, out, compute_prec, stream)
        return out


class Server:
    """Resident point sets and a continuously batched request loop (the C
    library's hodlr_server_*).  Requests take float64 device tensors (N or
    N x nrhs, column-major with leading dimension N) that must stay alive
    until the request completes."""

    def __init__(self, mem_budget_bytes=0, max_concurrent=8, max_batch_cols=64,
                 max_points=1 << 18, multiset=False):
        o = ServerOpts()
        lib().hodlr_server_default_opts(C.byref(o))
        o.mem_budget_bytes = int(mem_budget_bytes)
        o.max_concurrent = int(max_concurrent)
        o.max_batch_cols = int(max_batch_cols)
        o.max_points = int(max_points)
        o.multiset = 1 if multiset else 0
        out = _P()
        _check(lib().hodlr_server_create(C.byref(o), C.byref(out)))
        self.s = out.value
        self._keep = {}

    def add_set(self, points, kernel: Kernel, leaf_size: int, tol: float, *, level_rule=1,
                storage=FP64, domain=None) -> int:
        o = default_opts()
        o.level_rule = level_rule
        o.storage = storage
        if domain is not None:
            o.has_domain = 1
            lo = np.asarray(domain[0], dtype=np.float64)
            for a in range(len(lo)):
                o.domain_lo[a] = lo[a]
            o.domain_side = float(domain[1])
        P = np.ascontiguousarray(points, dtype=np.float64)
        sid = C.c_int()
        _check(lib().hodlr_server_add_set(C.c_void_p(self.s), _np_ptr(P), P.shape[0], P.shape[1],
                                          C.byref(kernel), int(leaf_size), float(tol),
                                          C.byref(o), C.byref(sid)))
        return sid.value

    @staticmethod
    def _shape(X):
        if X.dim() == 1:
            return X.shape[0], 1
        if X.stride(0) != 1 or (X.shape[1] > 1 and X.stride(1) != X.shape[0]):
            raise ValueError("requests take column-major tensors with leading dimension N")
        return X.shape

    def submit(self, kind: int, set_id: int, X, Y, alpha=1.0, beta=1.0, tol=1e-8,
               stream=None) -> int:
        """X is read after the work queued so far on `stream` (default: torch's
        current stream), where it is taken to be produced."""
        import torch
        if X.dtype != torch.float64 or Y.dtype != torch.float64:
            raise TypeError("requests take float64 tensors")
        _, nrhs = self._shape(X)
        if stream is None:
            stream = torch.cuda.current_stream(X.device)
        r = Request(kind, set_id, nrhs, X.data_ptr(), Y.data_ptr(), alpha, beta, tol,
                    _stream_ptr(stream).value)
        rid = _i64()
        _check(lib().hodlr_server_submit(C.c_void_p(self.s), C.byref(r), C.byref(rid)))
        self._keep[rid.value] = (X, Y)
        return rid.value

    def wait(self, rid: int):
        """Blocks; returns (queue_us, run_us); raises on a failed request."""
        qu, ru = C.c_double(), C.c_double()
        try:
            _check(lib().hodlr_server_wait(C.c_void_p(self.s), rid, C.byref(qu), C.byref(ru)))
        finally:
            self._keep.pop(rid, None)
        return qu.value, ru.value

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(lib().hodlr_server_get_stats(C.c_void_p(self.s), C.byref(st)))
        return st

    def close(self):
        if getattr(self, "s", None):
            lib().hodlr_server_destroy(C.c_void_p(self.s))
            self.s = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
