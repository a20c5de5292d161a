"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every entry point its header declares, and the ctypes structures match."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hodlr.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hodlr_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hodlr_build", "hodlr_matvec", "hodlr_destroy", "hodlr_last_error",
              "hodlr_export_tree", "hodlr_export_il", "hodlr_import_factors"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2209_05819_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    L = C.CDLL(P.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing


def test_struct_layouts_match_header():
    import paper_2209_05819_amd as P
    # sizes implied by the C declarations on x86-64
    assert C.sizeof(P.Kernel) == 32
    assert C.sizeof(P.Opts) == 4 * 2 + 8 * 8 + 8 + 4 * 4 + 8 + 8
    assert P.Info.build_ms.offset + 32 == P.Info.mfma_proj_jobs.offset
    assert P.Info.mfma_proj_elems.offset + 8 == C.sizeof(P.Info)
    assert C.sizeof(P.SolveOpts) == 8 * 2 + 4 * 4
    assert C.sizeof(P.SolveInfo) == 4 * 3 + 4 + 8 + 8 * 64
    assert C.sizeof(P.ServerOpts) == 8 + 4 + 4 + 8 + 8
    assert C.sizeof(P.Request) == 4 * 3 + 4 + 8 * 2 + 8 * 3 + 8
    assert C.sizeof(P.ServerStats) == 8 * 7 + 8 * 2 + 4 + 4
    assert C.sizeof(P.Tuning) == 4 + 4 * 8 + 4 + 8 * 8 + 8 * 2 + 8 + 8


def test_default_opts_and_errors_without_gpu():
    import paper_2209_05819_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    o = P.default_opts()
    assert o.symmetric == 1 and o.storage == P.FP64 and o.level_rule == 1 and o.adm_dim == 0
    assert o.skeleton == 0
    L = P.lib()
    # argument errors are reported before any device work
    st = L.hodlr_build(None, 10, 3, None, 8, 1e-6, None, None, None)
    assert st == 1 and b"null" in L.hodlr_last_error()
    import numpy as np
    pts = np.zeros((4, 9))
    k = P.make_kernel("inv_r")
    out = C.c_void_p()
    st = L.hodlr_build(pts.ctypes.data_as(C.c_void_p), 4, 9, C.byref(k), 8, 1e-6, None, None,
                       C.byref(out))
    assert st == 1 and b"d must be" in L.hodlr_last_error()
    so = P.default_solve_opts()
    assert so.tol == 1e-10 and so.restart == 50 and so.lo_compute == P.FP32
    st = L.hodlr_solve(None, None, 1.0, 1.0, None, 0, 1, None, 0, None, None, None)
    assert st == 1 and b"null" in L.hodlr_last_error()
    st = L.hodlr_matvec(None, None, 0, 1, 0, None, 0, 0, None)
    assert st == 1
    # route and server options are checked before any device work too
    assert L.hodlr_set_route(None, 1) == 1 and b"null" in L.hodlr_last_error()
    srv = C.c_void_p()
    for field, bad in (("multiset", 2), ("max_concurrent", 0), ("max_batch_cols", 1025),
                       ("max_points", 0)):
        o = P.ServerOpts()
        L.hodlr_server_default_opts(C.byref(o))
        assert o.multiset == 0 and o.max_concurrent == 8
        setattr(o, field, bad)
        assert L.hodlr_server_create(C.byref(o), C.byref(srv)) == 1
        assert field.encode() in L.hodlr_last_error()
    assert srv.value is None


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_2209_05819_amd as P
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(P, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        P.lib()


def test_mfma_extent_guard_without_gpu():
    """The matrix-core passes address BF16 factors through buffer resources of a
    2^31-byte range and move idle lanes past it by adding 2^31 to their
    offset; the host check must reject every factor whose offsets could reach
    2^31 (so that sum cannot wrap to a real address) and accept the rest."""
    import paper_2209_05819_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("library not built")
    lim = 1 << 31

    def ld(n):
        return (n + 7) // 8 * 8

    rng = __import__("numpy").random.default_rng(7)
    # synthetic factor tables: ranks up to the compressor's limit, lengths up
    # to a level-1 box of N = 2^26
    ranks = rng.integers(0, 1025, 400)
    lens = (2.0 ** rng.uniform(3, 25, 400)).astype(int)
    for r, n in zip(ranks.tolist(), lens.tolist()):
        for nrhs in (1, 16, 17, 32):
            st, ext = P.hodlr_mfma_extent(r, n, nrhs)
            # at least the factor's own last byte and the last x row's bytes
            assert ext >= 2 * r * ld(n) and ext >= 2 * n * (16 if nrhs <= 16 else 32)
            assert (st == 0) == (ext < lim)
            assert st in (0, 6)
    # monotone in the rank and the length, so one boundary per length
    for n in (4096, 1 << 20, (1 << 20) + 3):
        prev = 0
        flips = 0
        last_ok = True
        for r in range(0, 1100, 7):
            st, ext = P.hodlr_mfma_extent(r, n, 32)
            assert ext >= prev
            prev = ext
            if (st == 0) != last_ok:
                flips += 1
                last_ok = st == 0
        assert flips <= 1
    # the workloads' factors are far inside the range; a rank-1024 factor of
    # 2^20 rows is not
    assert P.hodlr_mfma_extent(1024, 65536, 32)[0] == 0
    assert P.hodlr_mfma_extent(1024, 1 << 20, 32)[0] == 6
    # an x slice of 2^25 rows with 32 right-hand sides alone exceeds it
    assert P.hodlr_mfma_extent(0, 1 << 25, 32)[0] == 6
    assert P.hodlr_mfma_extent(-1, 10, 1)[0] == 1
    assert P.hodlr_mfma_extent(1, 10, 33)[0] == 1
