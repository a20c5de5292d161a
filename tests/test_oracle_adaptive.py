"""Adaptive 2^d tree (level_rule 2; sec. 5.2 names an adaptive tree as an
option to the balanced one): pins of the oracle's adaptive tree and lists.

A box is subdivided only while it holds more than `leaf` points.  The pins
recompute every fact from the quantized coordinates by brute force: which
boxes exist, which are active and which are leaves, that the leaves
partition the points, that every ordered pair of points is covered by
exactly one low-rank or dense block, that a perfectly balanced cloud gives
the uniform tree's lists, and that the product stays within the tolerance of
the direct sum.
"""
import numpy as np
import pytest

from paper_2209_05819_amd import workloads as W


def _box_counts(o, level):
    """{box coordinates at `level`: number of points}, from the quantized
    coordinates alone."""
    q = o.quantized() >> (o.lmax - level)
    keys, cnt = np.unique(q, axis=0, return_counts=True)
    return {tuple(int(v) for v in k): int(c) for k, c in zip(keys, cnt)}


def _cover(o):
    N = o.N
    cov = np.zeros((N, N), dtype=np.int32)
    for l in range(0, o.kappa + 1):
        start, _, _ = o.boxes(l)
        if l >= 1:
            ptr, col = o.il(l)
            for A in range(len(start) - 1):
                for B in col[ptr[A]:ptr[A + 1]]:
                    cov[start[A]:start[A + 1], start[B]:start[B + 1]] += 1
        ptr, col = o.near_level(l)
        for A in range(len(start) - 1):
            for B in col[ptr[A]:ptr[A + 1]]:
                cov[start[A]:start[A + 1], start[B]:start[B + 1]] += 1
    return cov


@pytest.mark.parametrize("d,N,leaf,seed", [(2, 3000, 16, 31), (3, 4000, 20, 32), (1, 1500, 8, 33)])
def test_adaptive_flags_from_counts(orc, d, N, leaf, seed):
    P = W.gaussian_mixture(N, d, seed)
    o = orc.OracleHODLR(P, leaf, 2)
    # depth: the first level whose fullest box holds at most `leaf` points
    kap = next(l for l in range(0, o.lmax + 1) if max(_box_counts(o, l).values()) <= leaf)
    assert o.kappa == kap
    leaf_of_point = np.full(N, -1)
    for l in range(0, o.kappa + 1):
        cnt = _box_counts(o, l)
        par = _box_counts(o, l - 1) if l > 0 else None
        start, _, coord = o.boxes(l)
        flags = o.box_flags(l)
        assert len(start) - 1 == len(cnt)
        for A in range(len(start) - 1):
            c = tuple(int(v) for v in coord[A])
            assert start[A + 1] - start[A] == cnt[c]
            act = l == 0 or par[tuple(v >> 1 for v in c)] > leaf
            is_leaf = act and (cnt[c] <= leaf or l == o.kappa)
            assert bool(flags[A] & 1) == act, (l, A)
            assert bool(flags[A] & 2) == is_leaf, (l, A)
            if is_leaf:
                assert np.all(leaf_of_point[start[A]:start[A + 1]] == -1)
                leaf_of_point[start[A]:start[A + 1]] = l
    # the leaves (on several levels) partition the points
    assert np.all(leaf_of_point >= 0)
    assert len(np.unique(leaf_of_point)) > 1


@pytest.mark.parametrize("d,N,leaf,adm,seed", [
    (1, 900, 6, 0, 41), (2, 1400, 10, 0, 42), (2, 1200, 8, -1, 43), (2, 1200, 8, 1, 44),
    (3, 1200, 12, 0, 45), (3, 1000, 10, 2, 46),
])
def test_adaptive_lists_cover_every_pair_exactly_once(orc, d, N, leaf, adm, seed):
    P = W.gaussian_mixture(N, d, seed)
    o = orc.OracleHODLR(P, leaf, 2, adm_dim=adm)
    levels_with_leaves = {l for l in range(o.kappa + 1) if np.any(o.box_flags(l) & 2)}
    assert len(levels_with_leaves) >= 2
    cov = _cover(o)
    assert cov.min() == 1 and cov.max() == 1


def test_adaptive_lists_no_inactive_boxes(orc):
    P = W.gaussian_mixture(3000, 3, 47)
    o = orc.OracleHODLR(P, 16, 2)
    for l in range(1, o.kappa + 1):
        flags = o.box_flags(l)
        ptr, col = o.il(l)
        nptr, ncol = o.near_level(l)
        for A in range(len(flags)):
            row = np.concatenate([col[ptr[A]:ptr[A + 1]], ncol[nptr[A]:nptr[A + 1]]])
            if not flags[A] & 1:
                assert len(row) == 0
            assert np.all(flags[row] & 1)
            # a dense pair needs a leaf on one side
            for B in ncol[nptr[A]:nptr[A + 1]]:
                assert (flags[A] & 2) or (flags[B] & 2)


@pytest.mark.parametrize("d", [2, 3])
def test_adaptive_equals_uniform_on_balanced_cloud(orc, d):
    """Every finest cell holds the same number of points: the adaptive tree
    subdivides everything down to the same level and its lists are those of
    the uniform tree."""
    cells, per = (8, 3) if d == 2 else (4, 2)
    g = (np.arange(cells) + 0.5) / cells
    mesh = np.meshgrid(*([g] * d), indexing="ij")
    base = np.stack([m.reshape(-1) for m in mesh], axis=1)
    jit = W.rng(5).uniform(-0.2, 0.2, size=(per, base.shape[0], d)) / cells
    P = np.concatenate([base + j for j in jit])
    dom = (np.zeros(d), 1.0)
    a = orc.OracleHODLR(P, per, 2, domain=dom)
    u = orc.OracleHODLR(P, per, 0, domain=dom)
    assert a.kappa == u.kappa
    for l in range(0, a.kappa + 1):
        assert np.all(a.box_flags(l) & 1)
        assert np.all(((a.box_flags(l) & 2) != 0) == (l == a.kappa))
        if l >= 1:
            for x, y in zip(a.il(l), u.il(l)):
                assert np.array_equal(x, y)
        for x, y in zip(a.near_level(l), u.near_level(l)):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("kern,tol", [("inv_r", 1e-10), ("gauss", 1e-8)])
def test_adaptive_matvec_within_tolerance(orc, kern, tol):
    P = W.gaussian_mixture(2500, 3, 48)
    ko = orc.kernel(kern, h=0.5, diag=1.0 if kern == "gauss" else 0.0)
    o = orc.OracleHODLR(P, 24, 2)
    o.compress(ko, tol)
    q = W.rhs_normal(2500, 2, 49)
    b = o.matvec(ko, q)
    bd = orc.direct(P, ko, q)
    err = np.linalg.norm(b - bd) / np.linalg.norm(bd)
    assert err <= tol


def test_adaptive_fewer_near_pairs_than_balanced_depth(orc):
    """On clustered points the closed-form depth leaves crowded leaves; the
    adaptive tree keeps every leaf at most `leaf` points and evaluates fewer
    dense pairs."""
    P = W.gaussian_mixture(4000, 3, 50)

    def pairs(o):
        t = 0
        for l in range(o.kappa + 1):
            start, _, _ = o.boxes(l)
            ptr, col = o.near_level(l)
            m = np.diff(start)
            for A in range(len(m)):
                t += int(m[A] * m[col[ptr[A]:ptr[A + 1]]].sum())
        return t

    a = orc.OracleHODLR(P, 16, 2)
    c = orc.OracleHODLR(P, 16, 1)
    assert pairs(a) < pairs(c) / 2
