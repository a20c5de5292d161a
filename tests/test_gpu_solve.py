"""GMRES with FP64 iterative refinement around the product (needs an MI355X).

The representations are built from the oracle's own FP64 ACA factors
(imported), so the operator the solver inverts is the oracle's HODLRdD
operator; each solution is checked by the oracle's own product:
|F - (alpha U + beta K~ U)| / |F| must meet the solver's tolerance (up to
the FP64 rounding of one product).  A tiny case with a full-accuracy
compression is also checked against a dense LU solve of the kernel matrix.
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W
from test_gpu_parity import _pts, _symmetrize

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


def _handles(P, orc, pts, kern, h, diag, leaf, tol, storages):
    ko = orc.kernel(kern, h=h, diag=diag)
    o = orc.OracleHODLR(pts, leaf, 1)
    o.compress(ko, tol)
    for l in range(1, o.kappa + 1):
        r, U, V = _symmetrize(o, l)
        o.set_factors(l, r, U, V)
    hs = []
    for st in storages:
        H = P.HODLR(pts, P.make_kernel(kern, h=h, diag=diag), leaf, tol, level_rule=1,
                    skip_aca=True, storage=st)
        for l in range(1, o.kappa + 1):
            r, U, V = o.factors(l)
            P.hodlr_import_factors(H.h, l, r, U, V)
        hs.append(H)
    return o, ko, hs


def _dev(a):
    import torch
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.tensor(a, device="cuda")
    return torch.tensor(np.ascontiguousarray(a.T), device="cuda").t()


def _host(t):
    return t.t().contiguous().cpu().numpy().T if t.dim() == 2 else t.cpu().numpy()


SOLVE_CASES = [
    # d, N, kernel, h, diag, alpha, beta, lo storage, nrhs
    (3, 6000, "gauss", 0.5, 1.0, 1.0, 1.0 / 6000, "fp64", 1),
    (3, 6000, "gauss", 0.5, 1.0, 1.0, 1.0 / 6000, "bf16", 4),
    (2, 5000, "log", 1.0, 0.0, 1.0, 1.0 / 5000, "fp32", 3),
    (3, 8000, "inv_r", 1.0, 0.0, 1.0, 1.0 / 8000, "bf16", 16),
]


@pytest.mark.parametrize("d,N,kern,h,diag,alpha,beta,lo,nrhs", SOLVE_CASES)
def test_solve_residual_by_oracle(P, orc, d, N, kern, h, diag, alpha, beta, lo, nrhs):
    _say(f"[solve] d={d} N={N} {kern} lo={lo} nrhs={nrhs}")
    import torch
    pts = _pts(d, N, 500 + d, "uniform")
    st = {"fp64": P.FP64, "fp32": P.FP32, "bf16": P.BF16}[lo]
    o, ko, (Hhi, Hlo) = _handles(P, orc, pts, kern, h, diag, 48, 1e-10, [P.FP64, st])
    f = W.rhs_normal(N, nrhs, 77)
    f = f[:, 0] if nrhs == 1 else f
    F = _dev(f)
    U = torch.zeros_like(F) if nrhs == 1 else torch.zeros((nrhs, N), dtype=torch.float64,
                                                         device="cuda").t()
    opts = P.default_solve_opts()
    opts.tol = 1e-10
    opts.inner_tol = 1e-6 if lo == "fp64" else 1e-3
    info = P.hodlr_solve(Hhi.h, Hlo.h, alpha, beta, F, U, opts)
    torch.cuda.synchronize()
    u = _host(U)
    res = f - (alpha * u + beta * o.matvec(ko, u))
    rel = np.linalg.norm(res, axis=0) / np.linalg.norm(f, axis=0)
    _say(f"  outer {info.outer_iters} inner {info.inner_iters} reported {info.rel_residual:.2e} "
         f"oracle residual {np.max(rel):.2e}")
    assert info.converged == 1
    assert info.rel_residual <= 1e-10
    assert np.max(rel) <= 2e-10
    if lo != "fp64":
        assert info.outer_iters >= 2   # the low-precision inner solve needs refinement


def test_solve_matches_dense_solution(P, orc):
    """N = 600 in 2D with a near-exact compression: the solution of
    (I + K/N) u = f equals the dense LU solution."""
    import torch
    pts = W.uniform_points(600, 2, 9)
    o, ko, (H,) = _handles(P, orc, pts, "gauss", 0.5, 1.0, 40, 1e-15, [P.FP64])
    f = W.rhs_normal(600, 1, 10)[:, 0]
    K = orc.kernel_block(ko, pts, pts)
    np.fill_diagonal(K, 1.0)
    A = np.eye(600) + K / 600
    u_ref = np.linalg.solve(A, f)
    U = torch.zeros(600, dtype=torch.float64, device="cuda")
    opts = P.default_solve_opts()
    opts.tol = 1e-13
    opts.inner_tol = 1e-10
    opts.lo_compute = P.FP64
    info = P.hodlr_solve(H.h, H.h, 1.0, 1.0 / 600, _dev(f), U, opts)
    u = _host(U)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    _say(f"[solve] dense check err {err:.2e} outer {info.outer_iters} inner {info.inner_iters}")
    assert info.converged == 1 and err <= 1e-11


def test_solve_argument_errors(P, orc):
    import torch
    pts = W.uniform_points(3000, 3, 3)
    H64 = P.HODLR(pts, P.make_kernel("inv_r"), 64, 1e-8)
    H32 = P.HODLR(pts, P.make_kernel("inv_r"), 64, 1e-8, storage=P.FP32)
    H16 = P.HODLR(pts, P.make_kernel("inv_r"), 64, 1e-8, storage=P.BF16)
    Hx = P.HODLR(W.uniform_points(2000, 3, 4), P.make_kernel("inv_r"), 64, 1e-8)
    F = torch.ones(3000, dtype=torch.float64, device="cuda")
    U = torch.zeros_like(F)
    with pytest.raises(RuntimeError, match="EINVAL"):
        P.hodlr_solve(H16.h, H64.h, 1.0, 1.0, F, U)          # hi applied in FP64: not BF16
    with pytest.raises(RuntimeError, match="EINVAL"):
        P.hodlr_solve(H64.h, Hx.h, 1.0, 1.0, F, U)           # different point sets
    bad = P.default_solve_opts()
    bad.restart = 0
    with pytest.raises(RuntimeError, match="EINVAL"):
        P.hodlr_solve(H64.h, H64.h, 1.0, 1.0, F, U, bad)
    # not converging within max_outer is reported, not an error
    few = P.default_solve_opts()
    few.max_outer = 1
    few.restart = 2
    info = P.hodlr_solve(H64.h, H32.h, 1.0, 1e-4, F, U, few)
    assert info.converged == 0 and info.outer_iters == 1


def test_solve_ignores_output_contents_and_rejects_nonfinite(P, orc):
    """U is an output: NaN in it before the call must not matter (the solution
    still equals the dense LU solution); NaN in F, or in U when it is the
    initial guess, is an error instead of a reported convergence."""
    import torch
    pts = W.uniform_points(600, 2, 9)
    o, ko, (H,) = _handles(P, orc, pts, "gauss", 0.5, 1.0, 40, 1e-15, [P.FP64])
    f = W.rhs_normal(600, 1, 10)[:, 0]
    K = orc.kernel_block(ko, pts, pts)
    np.fill_diagonal(K, 1.0)
    u_ref = np.linalg.solve(np.eye(600) + K / 600, f)
    opts = P.default_solve_opts()
    opts.tol = 1e-13
    opts.inner_tol = 1e-10
    opts.lo_compute = P.FP64
    U = torch.full((600,), float("nan"), dtype=torch.float64, device="cuda")
    info = P.hodlr_solve(H.h, H.h, 1.0, 1.0 / 600, _dev(f), U, opts)
    u = _host(U)
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    _say(f"[solve] NaN-filled output: err {err:.2e} converged {info.converged}")
    assert info.converged == 1 and err <= 1e-11
    fbad = f.copy()
    fbad[17] = np.nan
    with pytest.raises(RuntimeError, match="ENONFINITE"):
        P.hodlr_solve(H.h, H.h, 1.0, 1.0 / 600, _dev(fbad), torch.zeros_like(U), opts)
    guess = P.default_solve_opts()
    guess.use_initial_guess = 1
    U.fill_(float("nan"))
    with pytest.raises(RuntimeError, match="ENONFINITE"):
        P.hodlr_solve(H.h, H.h, 1.0, 1.0 / 600, _dev(f), U, guess)
