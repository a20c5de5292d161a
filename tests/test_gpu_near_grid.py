"""The near field beside the low-rank stages in both of its launch regimes
(needs an MI355X).

The on-the-fly near kernel runs on the handle's second stream.  While the
near field is light next to the streamed factor bytes (at most 0.05 dense
pairs per column and factor byte) it takes one workgroup per CU, each
looping over many leaf chunks; otherwise one workgroup per chunk.  Each case
first checks from hodlr_get_info which regime it is in, then compares the
product with the direct sum on sampled rows, and checks that two products of
the same input agree bit for bit (the fork, the join and the item loop leave
no order to chance).
"""
import sys

import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W

pytestmark = pytest.mark.gpu

PAIRS_PER_BYTE = 0.05   # the library's switch between the two grids


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


CASES = [
    # N, leaf, storage, light (capped grid) expected
    (32768, 64, "fp64", True),
    # FP32 factors are truncated (fewer bytes per dense pair): light from
    # 2^17 points on, heavy at 2^15
    (131072, 64, "fp32", True),
    (32768, 64, "fp32", False),
    (32768, 512, "fp64", False),
]


@pytest.mark.parametrize("N,leaf,stor,light", CASES)
def test_near_grid_regimes_against_direct_sum(P, orc, N, leaf, stor, light):
    import torch
    _say(f"[near grid] N={N} leaf={leaf} {stor} light={light}")
    storage, esize = (P.FP64, 8) if stor == "fp64" else (P.FP32, 4)
    tol = 1e-10
    pts = W.uniform_points(N, 3, 401)
    H = P.HODLR(pts, P.make_kernel("inv_r"), leaf, tol, storage=storage)
    info = H.info()
    fe = sum(info.class_factor_elems[c] for c in range(8)) + info.split_factor_elems
    ratio = info.near_pairs / (fe * esize)
    _say(f"  near pairs {info.near_pairs}, streamed factor bytes {fe * esize}, ratio {ratio:.4f}")
    assert (ratio <= PAIRS_PER_BYTE) == light
    q = W.rhs_normal(N, 1, 402)[:, 0]
    dt = torch.float64 if stor == "fp64" else torch.float32
    X = torch.tensor(q, dtype=dt, device="cuda")
    comp = P.FP64 if stor == "fp64" else P.FP32
    Y1 = H.matvec(X, compute_prec=comp)
    Y2 = H.matvec(X, compute_prec=comp)
    torch.cuda.synchronize()
    assert torch.equal(Y1, Y2)
    rows = np.sort(W.rng(403).choice(N, 1000, replace=False))
    bd = orc.direct(pts, orc.kernel("inv_r"), q, rows=rows)
    err = float(np.linalg.norm(Y1.cpu().numpy().astype(np.float64)[rows] - bd) /
                np.linalg.norm(bd))
    _say(f"  rel err vs direct {err:.3e}")
    assert err <= (tol if stor == "fp64" else 1e-5)
