"""Pins of the oracle's Galerkin coarse operator of an aggregation (a
multigrid hookup: Section VI-E builds smoothed-aggregation multigrid on these
aggregates): against the dense product P^T A P with the tentative prolongator
P[i][agg i] = 1/sqrt(|agg i|), the identity and one-aggregate special cases,
the constant-vector identity A_c s = P^T (A 1) with s_a = sqrt(|a|), and the
exact rounding of the final scaling on integer-valued matrices."""
import math

import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs


def _dense(rp, c, val, diag):
    n = rp.size - 1
    A = np.diag(np.asarray(diag, np.float64))
    src = np.repeat(np.arange(n), np.diff(rp))
    A[src, c] = val
    return A


def _prolongator(agg, n_agg):
    n = agg.size
    size = np.bincount(agg, minlength=n_agg).astype(np.float64)
    P = np.zeros((n, n_agg))
    P[np.arange(n), agg] = 1.0 / np.sqrt(size[agg])
    return P, size


def _coarse_dense(crow, ccol, cval, cdiag):
    na = crow.size - 1
    Ac = np.diag(cdiag)
    src = np.repeat(np.arange(na), np.diff(crow))
    Ac[src, ccol] = cval
    return Ac


CASES = [
    ("grid27", lambda: graphs.grid3d_27pt(7, 6, 5)),
    ("grid2d", lambda: graphs.grid2d_5pt(13, 11)),
    ("chunglu", lambda: graphs.chung_lu(700, 6.0, 2.1, 90, seed=4)),
    ("er", lambda: graphs.erdos_renyi(300, 0.03, seed=8)),
    ("union", lambda: graphs.disjoint_union([graphs.grid2d_5pt(6, 6), graphs.complete(7),
                                             graphs.edgeless(4), graphs.path(9)])),
]


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_equals_dense_ptap(name):
    rp, c = dict(CASES)[name]()
    val, diag = graphs.matrix_values(rp, c, 3, shift=0.5)
    agg, na = oracle.aggregate(rp, c, 1)
    crow, ccol, cval, cdiag = oracle.galerkin(rp, c, val, diag, agg, na)
    P, _ = _prolongator(agg, na)
    want = P.T @ _dense(rp, c, val, diag) @ P
    got = _coarse_dense(crow, ccol, cval, cdiag)
    scale = np.abs(want).max()
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13 * scale)
    # the quotient graph holds every off-diagonal coupling
    off = want - np.diag(np.diag(want))
    pattern = _coarse_dense(crow, ccol, np.ones_like(cval), np.zeros(na)) != 0
    assert not np.any((np.abs(off) > 1e-12 * scale) & ~pattern)


def test_identity_aggregation_returns_the_matrix():
    rp, c = graphs.grid3d_27pt(5, 5, 4)
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 1)
    crow, ccol, cval, cdiag = oracle.galerkin(rp, c, val, diag, np.arange(n, dtype=np.int32), n)
    assert np.array_equal(crow, rp) and np.array_equal(ccol, c)
    assert np.array_equal(cval, val) and np.array_equal(cdiag, diag)


def test_one_aggregate_is_the_mean_of_all_entries():
    rp, c = graphs.chung_lu(300, 5.0, 2.1, 40, seed=2)
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 5)
    crow, ccol, cval, cdiag = oracle.galerkin(rp, c, val, diag, np.zeros(n, np.int32), 1)
    assert crow.tolist() == [0, 0] and cval.size == 0
    exact = math.fsum(list(diag) + list(val)) / n
    assert abs(cdiag[0] - exact) <= 1e-12 * abs(exact) * (n + val.size)


@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_constant_vector_identity(name):
    rp, c = dict(CASES)[name]()
    val, diag = graphs.matrix_values(rp, c, 6)
    agg, na = oracle.aggregate(rp, c, 2)
    crow, ccol, cval, cdiag = oracle.galerkin(rp, c, val, diag, agg, na)
    P, size = _prolongator(agg, na)
    A = _dense(rp, c, val, diag)
    lhs = _coarse_dense(crow, ccol, cval, cdiag) @ np.sqrt(size)
    rhs = P.T @ (A @ np.ones(rp.size - 1))
    assert np.allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * np.abs(rhs).max())
    # a symmetric A gives a symmetric A_c
    Ac = _coarse_dense(crow, ccol, cval, cdiag)
    assert np.allclose(Ac, Ac.T, rtol=1e-12, atol=1e-13 * np.abs(Ac).max())


def test_scaling_rounds_once_on_exact_sums():
    # integer values: every sum is exact, so each coarse value is the one
    # correctly rounded quotient S / sqrt(n_a * n_b)
    rp, c = graphs.grid3d_27pt(8, 7, 6)
    n = rp.size - 1
    rng = np.random.default_rng(3)
    src = np.repeat(np.arange(n), np.diff(rp))
    w = rng.integers(-9, 10, size=(n, n))
    w = w + w.T
    val = w[src, c].astype(np.float64)
    diag = rng.integers(50, 100, size=n).astype(np.float64)
    agg, na = oracle.aggregate(rp, c, 0)
    crow, ccol, cval, cdiag = oracle.galerkin(rp, c, val, diag, agg, na)
    size = np.bincount(agg, minlength=na)
    S = np.zeros((na, na))
    np.add.at(S, (agg[src], agg[c]), val)
    S[np.arange(na), np.arange(na)] += np.bincount(agg, weights=diag, minlength=na)
    rows = np.repeat(np.arange(na), np.diff(crow))
    want = S[rows, ccol] / np.sqrt(size[rows].astype(np.float64) * size[ccol].astype(np.float64))
    assert np.array_equal(cval, want)
    assert np.array_equal(cdiag, np.diag(S) / size.astype(np.float64))


def test_empty_graph():
    crow, ccol, cval, cdiag = oracle.galerkin(np.zeros(1, np.int64), np.zeros(0, np.int32),
                                              np.zeros(0), np.zeros(0), np.zeros(0, np.int32), 0)
    assert cval.size == 0 and cdiag.size == 0
