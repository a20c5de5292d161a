"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the FP64 CPU oracle.

The oracle (``hodlr_oracle.c``) is a plain CPU implementation of the HODLRdD
method of Khan, Kandappan and Ambikasaran (arXiv 2209.05819): the direct sum
and the method's steps (sec. 5.2 tree, sec. 5.3 interaction lists, eq. keq1
ACA, Alg. "HODLRdD matrix-vector Product").  Only the tests, the smoke check
and the CPU-baseline leg of the benchmark use it.  It shares no code with the
GPU library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hodlr_oracle.c")
LIB = os.path.join(HERE, "libhodlr_oracle.so")

KERNELS = {"log": 0, "inv_r": 1, "inv_r2": 2, "gauss": 3, "exp": 4, "r": 5,
           "sin": 6, "inv_sqrt1p": 7}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP, no fast-math)."""
    stale = (not os.path.exists(LIB)
             or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                            os.path.getmtime(os.path.join(HERE, "hodlr_oracle.h"))))
    if force or stale:
        cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
               SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("h", C.c_double), ("scale", C.c_double),
                ("diag", C.c_double)]


_lib = None
_P = C.c_void_p
_i64 = C.c_int64


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        L.ohodlr_create_adm.restype = _P
        L.ohodlr_create_adm.argtypes = [_P, _i64, C.c_int, C.c_int, _P, C.c_double, C.c_int,
                                        C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.ohodlr_create.restype = _P
        L.ohodlr_create.argtypes = [_P, _i64, C.c_int, C.c_int, _P, C.c_double,
                                    C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.ohodlr_destroy.argtypes = [_P]
        for f in ("ohodlr_kappa", "ohodlr_lmax"):
            getattr(L, f).argtypes = [_P]
            getattr(L, f).restype = C.c_int
        L.ohodlr_domain.argtypes = [_P, _P, _P]
        L.ohodlr_perm.argtypes = [_P, _P]
        L.ohodlr_keys.argtypes = [_P, _P]
        L.ohodlr_quantized.argtypes = [_P, _P]
        L.ohodlr_nboxes.argtypes = [_P, C.c_int]
        L.ohodlr_nboxes.restype = _i64
        L.ohodlr_boxes.argtypes = [_P, C.c_int, _P, _P, _P]
        L.ohodlr_il_nnz.argtypes = [_P, C.c_int]
        L.ohodlr_il_nnz.restype = _i64
        L.ohodlr_il.argtypes = [_P, C.c_int, _P, _P]
        L.ohodlr_near_nnz.argtypes = [_P]
        L.ohodlr_near_nnz.restype = _i64
        L.ohodlr_near.argtypes = [_P, _P, _P]
        L.ohodlr_near_level_nnz.argtypes = [_P, C.c_int]
        L.ohodlr_near_level_nnz.restype = _i64
        L.ohodlr_near_level.argtypes = [_P, C.c_int, _P, _P]
        L.ohodlr_box_flags.argtypes = [_P, C.c_int, _P]
        L.ohodlr_aca_dense.argtypes = [_P, _i64, _i64, C.c_double, C.c_int, _P, _P, _P, _P]
        L.ohodlr_aca_dense.restype = C.c_int
        L.ohodlr_compress.argtypes = [_P, C.POINTER(_Kernel), C.c_double, C.c_int, _i64, _i64]
        L.ohodlr_compress.restype = C.c_int
        L.ohodlr_ranks.argtypes = [_P, C.c_int, _P]
        L.ohodlr_factor_elems.argtypes = [_P, C.c_int, C.c_int]
        L.ohodlr_factor_elems.restype = _i64
        L.ohodlr_factors.argtypes = [_P, C.c_int, _P, _P]
        L.ohodlr_set_factors.argtypes = [_P, C.c_int, _P, _P, _P]
        L.ohodlr_set_factors.restype = C.c_int
        L.ohodlr_matvec.argtypes = [_P, C.POINTER(_Kernel), _P, C.c_int, _P, _i64, _i64]
        L.ohodlr_matvec.restype = C.c_int
        L.ohodlr_direct.argtypes = [_P, _i64, C.c_int, C.POINTER(_Kernel), _P, C.c_int,
                                    _P, _i64, _P]
        L.ohodlr_kernel_eval.argtypes = [C.POINTER(_Kernel), _P, _P, C.c_int]
        L.ohodlr_kernel_eval.restype = C.c_double
        L.ohodlr_kernel_block.argtypes = [C.POINTER(_Kernel), _P, _i64, _P, _i64, C.c_int, _P]
        L.ohodlr_num_threads.restype = C.c_int
        L.ohodlr_set_threads.argtypes = [C.c_int]
        L.ohodlr_set_threads.restype = None
        _lib = L
    return _lib


def kernel(kind: str | int, h: float = 1.0, scale: float = 1.0, diag: float = 0.0) -> _Kernel:
    k = KERNELS[kind] if isinstance(kind, str) else int(kind)
    return _Kernel(k, float(h), float(scale), float(diag))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return lib().ohodlr_num_threads()


def set_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops."""
    lib().ohodlr_set_threads(int(n))


def kernel_block(k: _Kernel, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    out = np.empty((X.shape[0], Y.shape[0]), dtype=np.float64)
    lib().ohodlr_kernel_block(C.byref(k), _ptr(X), X.shape[0], _ptr(Y), Y.shape[0],
                              X.shape[1], _ptr(out))
    return out


def direct(points: np.ndarray, k: _Kernel, q: np.ndarray, rows=None) -> np.ndarray:
    """b = K q by the plain definition (optionally only some rows)."""
    P = np.ascontiguousarray(points, dtype=np.float64)
    N, d = P.shape
    q2 = np.asfortranarray(q.reshape(N, -1), dtype=np.float64)
    nrhs = q2.shape[1]
    if rows is None:
        b = np.empty((N, nrhs), dtype=np.float64, order="F")
        lib().ohodlr_direct(_ptr(P), N, d, C.byref(k), _ptr(q2), nrhs, None, 0, _ptr(b))
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        b = np.empty((len(r), nrhs), dtype=np.float64, order="F")
        lib().ohodlr_direct(_ptr(P), N, d, C.byref(k), _ptr(q2), nrhs, _ptr(r), len(r), _ptr(b))
    return b.reshape((-1,) if q.ndim == 1 else b.shape)


def aca_dense(M: np.ndarray, tol: float, max_rank: int = 0):
    M = np.ascontiguousarray(M, dtype=np.float64)
    m, n = M.shape
    kk = min(m, n)
    U = np.zeros(m * kk)
    V = np.zeros(n * kk)
    pr = np.zeros(kk, dtype=np.int64)
    pc = np.zeros(kk, dtype=np.int64)
    r = lib().ohodlr_aca_dense(_ptr(M), m, n, tol, max_rank, _ptr(U), _ptr(V), _ptr(pr), _ptr(pc))
    if r < 0:
        raise MemoryError("oracle ACA ran out of memory")
    Um = U[: m * r].reshape(r, m).T.copy()      # m x r
    Vm = V[: n * r].reshape(r, n).copy()        # r x n
    return Um, Vm, pr[:r].copy(), pc[:r].copy()


class OracleHODLR:
    """Tree, lists, ACA factors and matvec of the HODLRdD method (FP64, CPU)."""

    def __init__(self, points, leaf: int, level_rule: int = 0, domain=None, adm_dim: int = 0):
        P = np.ascontiguousarray(points, dtype=np.float64)
        self.points = P
        self.N, self.d = P.shape
        st = C.c_int(0)
        lo = np.zeros(8)
        if domain is None:
            h = lib().ohodlr_create_adm(_ptr(P), self.N, self.d, 0, _ptr(lo), 1.0, leaf,
                                        level_rule, adm_dim, C.byref(st))
        else:
            lo[: self.d] = np.asarray(domain[0], dtype=np.float64)
            h = lib().ohodlr_create_adm(_ptr(P), self.N, self.d, 1, _ptr(lo), float(domain[1]),
                                        leaf, level_rule, adm_dim, C.byref(st))
        if not h:
            raise ValueError(f"oracle tree build failed (status {st.value})")
        self.h = h
        self.kappa = lib().ohodlr_kappa(h)
        self.lmax = lib().ohodlr_lmax(h)

    def __del__(self):
        if getattr(self, "h", None):
            lib().ohodlr_destroy(self.h)
            self.h = None

    def domain(self):
        lo = np.zeros(8)
        side = C.c_double(0)
        lib().ohodlr_domain(self.h, _ptr(lo), C.byref(side))
        return lo[: self.d].copy(), side.value

    def perm(self):
        p = np.empty(self.N, dtype=np.int64)
        lib().ohodlr_perm(self.h, _ptr(p))
        return p

    def keys(self):
        k = np.empty(self.N, dtype=np.uint64)
        lib().ohodlr_keys(self.h, _ptr(k))
        return k

    def quantized(self):
        q = np.empty((self.N, self.d), dtype=np.int64)
        lib().ohodlr_quantized(self.h, _ptr(q))
        return q

    def boxes(self, level: int):
        nb = lib().ohodlr_nboxes(self.h, level)
        start = np.empty(nb + 1, dtype=np.int64)
        key = np.empty(nb, dtype=np.uint64)
        coord = np.empty((nb, self.d), dtype=np.int32)
        lib().ohodlr_boxes(self.h, level, _ptr(start), _ptr(key), _ptr(coord))
        return start, key, coord

    def il(self, level: int):
        nnz = lib().ohodlr_il_nnz(self.h, level)
        nb = lib().ohodlr_nboxes(self.h, level)
        ptr = np.empty(nb + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        lib().ohodlr_il(self.h, level, _ptr(ptr), _ptr(col))
        return ptr, col[:nnz]

    def near(self):
        nnz = lib().ohodlr_near_nnz(self.h)
        nb = lib().ohodlr_nboxes(self.h, self.kappa)
        ptr = np.empty(nb + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        lib().ohodlr_near(self.h, _ptr(ptr), _ptr(col))
        return ptr, col[:nnz]

    def near_level(self, level: int):
        """Dense near-field pairs of one level (CSR over the level's boxes)."""
        nnz = lib().ohodlr_near_level_nnz(self.h, level)
        nb = lib().ohodlr_nboxes(self.h, level)
        ptr = np.empty(nb + 1, dtype=np.int64)
        col = np.empty(max(nnz, 1), dtype=np.int32)
        lib().ohodlr_near_level(self.h, level, _ptr(ptr), _ptr(col))
        return ptr, col[:nnz]

    def box_flags(self, level: int):
        """Per box: bit 0 active (parent subdivided), bit 1 leaf."""
        nb = lib().ohodlr_nboxes(self.h, level)
        f = np.empty(max(nb, 1), dtype=np.uint8)
        lib().ohodlr_box_flags(self.h, level, _ptr(f))
        return f[:nb]

    def compress(self, k: _Kernel, tol: float, max_rank: int = 0, rows=None):
        r0, r1 = (0, self.N) if rows is None else rows
        st = lib().ohodlr_compress(self.h, C.byref(k), tol, max_rank, r0, r1)
        if st != 0:
            raise RuntimeError(f"oracle compress failed (status {st})")

    def ranks(self, level: int):
        nnz = lib().ohodlr_il_nnz(self.h, level)
        r = np.empty(max(nnz, 1), dtype=np.int32)
        lib().ohodlr_ranks(self.h, level, _ptr(r))
        return r[:nnz]

    def factors(self, level: int):
        nu = lib().ohodlr_factor_elems(self.h, level, 0)
        nv = lib().ohodlr_factor_elems(self.h, level, 1)
        U = np.empty(max(nu, 1))
        V = np.empty(max(nv, 1))
        lib().ohodlr_factors(self.h, level, _ptr(U), _ptr(V))
        return self.ranks(level), U[:nu], V[:nv]

    def set_factors(self, level: int, ranks, U, V):
        ranks = np.ascontiguousarray(ranks, dtype=np.int32)
        U = np.ascontiguousarray(U, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        st = lib().ohodlr_set_factors(self.h, level, _ptr(ranks), _ptr(U), _ptr(V))
        if st != 0:
            raise ValueError("bad factors")

    def matvec(self, k: _Kernel, q: np.ndarray, rows=None) -> np.ndarray:
        N = self.N
        q2 = np.asfortranarray(q.reshape(N, -1), dtype=np.float64)
        nrhs = q2.shape[1]
        b = np.empty((N, nrhs), dtype=np.float64, order="F")
        r0, r1 = (0, N) if rows is None else rows
        st = lib().ohodlr_matvec(self.h, C.byref(k), _ptr(q2), nrhs, _ptr(b), r0, r1)
        if st != 0:
            raise RuntimeError("oracle matvec: factors missing")
        return b.reshape((-1,) if q.ndim == 1 else b.shape)
