"""The product entry point that allocates nothing (hodlr_matvec_noalloc: the
static scratch array as workspace, the near field on the caller's stream),
checked against hodlr_matvec on the same handle (needs an MI355X): the
element-wise bar of the product's other parity tests (relative 1e-13 of the
largest entry for FP64, 1e-6 for FP32 arithmetic), on two calls in a row,
the second with a smaller input, and refused when the workspace exceeds the
scratch array."""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W

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


def _dev(torch, N, nrhs, seed, dtype):
    x = W.rhs_normal(N, nrhs, seed)
    if nrhs == 1:
        return torch.tensor(x[:, 0], dtype=dtype, device="cuda")
    return torch.tensor(np.ascontiguousarray(x.T), dtype=dtype, device="cuda").t()


def _same(a, b, rel):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    return np.max(np.abs(a - b)) <= rel * np.max(np.abs(b))


@pytest.mark.parametrize("storage,comp", [("fp64", "fp64"), ("fp32", "fp32"), ("bf16", "fp32")])
def test_noalloc_equals_matvec_on_two_calls(P, storage, comp):
    import torch
    st = {"fp64": P.FP64, "fp32": P.FP32, "bf16": P.BF16}[storage]
    cp = P.FP64 if comp == "fp64" else P.FP32
    dt = torch.float64 if comp == "fp64" else torch.float32
    rel = 1e-13 if comp == "fp64" else 1e-6
    # first call: 2D, 10000 points, several columns; second: a smaller 3D set,
    # one column
    big = P.HODLR(W.uniform_points(10000, 2, 31), P.make_kernel("log"), 64, 1e-8, storage=st)
    small = P.HODLR(W.uniform_points(3000, 3, 32), P.make_kernel("inv_r"), 64, 1e-8, storage=st)
    for H, N, nrhs, seed in ((big, 10000, 3 if storage != "bf16" else 20, 1), (small, 3000, 1, 2)):
        _say(f"[noalloc] {storage} N={N} nrhs={nrhs}")
        X = _dev(torch, N, nrhs, seed, dt)
        Yref = torch.empty_like(X)
        Y = torch.full_like(X, float("nan"))
        P.hodlr_matvec(H.h, X, Yref, cp)
        P.hodlr_matvec_noalloc(H.h, X, Y, cp)
        torch.cuda.synchronize()
        assert torch.isfinite(Y).all()
        assert _same(Y, Yref, rel)


def test_noalloc_refuses_a_workspace_beyond_the_scratch(P):
    import torch
    N = 300000
    H = P.HODLR(W.uniform_points(N, 3, 33), P.make_kernel("inv_r"), 64, 1e-4)
    X = torch.ones((8, N), dtype=torch.float64, device="cuda").t()
    Y = torch.empty_like(X)
    with pytest.raises(P.HodlrError, match="EINVAL.*scratch"):
        P.hodlr_matvec_noalloc(H.h, X, Y, P.FP64)
