"""Adaptive 2^d tree (level_rule 2) on the GPU (needs an MI355X).

- tree, box flags, interaction lists and the dense pairs of every level:
  bit-exact with the oracle;
- apply with the oracle's own ACA factors imported: the GPU product equals
  the oracle's to FP64 rounding (leaves on several levels, dense pairs
  between a leaf and a larger box), for one and several right-hand sides,
  FP64 and BF16 factors;
- full pipeline (GPU ACA): within the tolerance of the direct sum.
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_bf16 import C_BOUND, _abs_product
from test_gpu_parity import _gpu_matvec, _rel, _symmetrize

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_05819_amd as P
    P.lib()
    return P


TREE_CASES = [
    # d, N, leaf, adm, seed
    (1, 3000, 12, 0, 61),
    (2, 6000, 32, 0, 62),
    (2, 5000, 20, -1, 63),
    (3, 20000, 64, 0, 64),
    (3, 12000, 40, 1, 65),
    (4, 8000, 60, 0, 66),
]


@pytest.mark.parametrize("d,N,leaf,adm,seed", TREE_CASES)
def test_adaptive_tree_and_lists_bit_exact(P, orc, d, N, leaf, adm, seed):
    _say(f"[adaptive tree] d={d} N={N} leaf={leaf} adm={adm}")
    pts = W.gaussian_mixture(N, d, seed)
    o = orc.OracleHODLR(pts, leaf, 2, adm_dim=adm)
    H = P.HODLR(pts, P.make_kernel("inv_r"), leaf, 1e-6, level_rule=2, adm_dim=adm,
                skip_aca=True)
    assert H.info().kappa == o.kappa
    perm, keys = P.hodlr_export_tree(H.h, N)
    assert np.array_equal(perm, o.perm()) and np.array_equal(keys, o.keys())
    leaf_levels = 0
    for l in range(o.kappa + 1):
        s0, k0, c0 = o.boxes(l)
        nb = len(s0) - 1
        s1, k1, c1 = P.hodlr_export_boxes(H.h, l, nb, d)
        assert np.array_equal(s0, s1) and np.array_equal(k0, k1) and np.array_equal(c0, c1)
        f0 = o.box_flags(l)
        assert np.array_equal(f0, P.hodlr_export_box_flags(H.h, l, nb)), f"flags level {l}"
        leaf_levels += int(np.any(f0 & 2))
        if l >= 1:
            p0, col0 = o.il(l)
            p1, col1 = P.hodlr_export_il(H.h, l, nb)
            assert np.array_equal(p0, p1) and np.array_equal(col0, col1), f"il level {l}"
        p0, col0 = o.near_level(l)
        p1, col1 = P.hodlr_export_near_level(H.h, l, nb)
        assert np.array_equal(p0, p1) and np.array_equal(col0, col1), f"near level {l}"
    assert leaf_levels >= 2
    # the dense point pairs reported by the library equal the oracle's lists
    pairs = 0
    for l in range(o.kappa + 1):
        s0, _, _ = o.boxes(l)
        ptr, col = o.near_level(l)
        m = np.diff(s0)
        for A in range(len(m)):
            pairs += int(m[A] * m[col[ptr[A]:ptr[A + 1]]].sum())
    assert H.info().near_pairs == pairs


def _import(P, o, H, sym):
    for l in range(1, o.kappa + 1):
        if sym:
            r, U, V = _symmetrize(o, l)
            o.set_factors(l, r, U, V)
        r, U, V = o.factors(l)
        P.hodlr_import_factors(H.h, l, r, U, V)


APPLY_CASES = [
    # d, N, leaf, kernel, tol, seed
    (3, 12000, 48, "inv_r", 1e-10, 71),
    (3, 10000, 32, "gauss", 1e-6, 72),
    (2, 8000, 40, "log", 1e-8, 73),
    (1, 4000, 16, "inv_r", 1e-10, 74),
]


@pytest.mark.parametrize("sym", [False, True])
@pytest.mark.parametrize("d,N,leaf,kern,tol,seed", APPLY_CASES)
def test_adaptive_apply_with_oracle_factors(P, orc, d, N, leaf, kern, tol, seed, sym):
    _say(f"[adaptive apply] d={d} N={N} {kern} sym={sym}")
    pts = W.gaussian_mixture(N, d, seed)
    diag = 1.001 if kern == "gauss" else 0.0
    ko = orc.kernel(kern, h=0.5, diag=diag)
    o = orc.OracleHODLR(pts, leaf, 2)
    o.compress(ko, tol)
    H = P.HODLR(pts, P.make_kernel(kern, h=0.5, diag=diag), leaf, tol, level_rule=2,
                skip_aca=True, symmetric=sym)
    _import(P, o, H, sym)
    q = W.rhs_normal(N, 3, 9)
    b_or = o.matvec(ko, q)
    for nr in (1, 3):
        qq = q[:, 0] if nr == 1 else q
        bo = b_or[:, 0] if nr == 1 else b_or
        bg = _gpu_matvec(P, H, qq)
        assert _rel(bg, bo) <= 1e-13
        assert np.max(np.abs(bg - bo)) <= 1e-12 * np.max(np.abs(bo))


@pytest.mark.parametrize("nrhs", [1, 16, 20])
def test_adaptive_bf16_apply_with_oracle_factors(P, orc, nrhs):
    """BF16 factors (matrix-core product for several right-hand sides), within
    the derived bound 4.25 u z of the oracle's product."""
    _say(f"[adaptive bf16] nrhs={nrhs}")
    N, d, leaf = 12000, 3, 48
    pts = W.gaussian_mixture(N, d, 75)
    ko = orc.kernel("gauss", h=0.5, diag=1.001)
    o = orc.OracleHODLR(pts, leaf, 2)
    o.compress(ko, 1e-6)
    H = P.HODLR(pts, P.make_kernel("gauss", h=0.5, diag=1.001), leaf, 1e-6, level_rule=2,
                skip_aca=True, storage=P.BF16)
    _import(P, o, H, True)
    q = W.rhs_normal(N, nrhs, 19)
    qq = q[:, 0] if nrhs == 1 else q
    bo = o.matvec(ko, qq)
    z = _abs_product(o, ko, qq)
    bg = _gpu_matvec(P, H, qq, x_dtype="f32", compute=P.FP32)
    assert np.all(np.abs(bg - bo) <= C_BOUND * z)


PIPE_CASES = [
    # d, N, leaf, kernel, h, diag, tol, seed
    (3, 30000, 64, "gauss", 0.5, 1.001, 1e-6, 81),
    (3, 20000, 64, "inv_r", 1.0, 0.0, 1e-10, 82),
    (2, 12000, 64, "log", 1.0, 0.0, 1e-8, 83),
]


@pytest.mark.parametrize("d,N,leaf,kern,h,diag,tol,seed", PIPE_CASES)
def test_adaptive_pipeline_against_direct_sum(P, orc, d, N, leaf, kern, h, diag, tol, seed):
    _say(f"[adaptive pipeline] d={d} N={N} {kern}")
    pts = W.gaussian_mixture(N, d, seed)
    ko = orc.kernel(kern, h=h, diag=diag)
    H = P.HODLR(pts, P.make_kernel(kern, h=h, diag=diag), leaf, tol, level_rule=2)
    q = W.rhs_normal(N, 2, 31)
    rows = np.sort(W.rng(seed).choice(N, 2000, replace=False))
    bd = orc.direct(pts, ko, q, rows=rows)
    bg = _gpu_matvec(P, H, q)[rows]
    err = _rel(bg, bd)
    _say(f"  rel err vs direct {err:.3e}")
    assert err <= tol
    # fewer dense pairs than the closed-form depth on the same clustered cloud
    C = P.HODLR(pts, P.make_kernel(kern, h=h, diag=diag), leaf, tol, level_rule=1,
                skip_aca=True)
    assert H.info().near_pairs < C.info().near_pairs
