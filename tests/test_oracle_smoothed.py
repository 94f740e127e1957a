"""Pins of the oracle's smoothed aggregation (oracle.smoothed): the damped-
Jacobi prolongator P = (I - omega D^-1 A) P_tent and the coarse operator
P^T A P, against a dense product written out with numpy (another order of
operations), exact rational arithmetic where every value is a dyadic
fraction, the tentative prolongator at omega = 0, the constant vector of a
Laplacian and symmetry."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2204_02934_amd import graphs


def _dense(rp, c, val, diag):
    n = rp.size - 1
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = diag[i]
        for e in range(rp[i], rp[i + 1]):
            A[i, c[e]] = val[e]
    return A


def _to_dense(ptr, col, v, rows, cols):
    D = np.zeros((rows, cols))
    for r in range(rows):
        for p in range(ptr[r], ptr[r + 1]):
            D[r, col[p]] = v[p]
    return D


def _tentative(agg, n_agg):
    n = agg.size
    size = np.bincount(agg, minlength=n_agg)
    Pt = np.zeros((n, n_agg))
    Pt[np.arange(n), agg] = 1.0 / np.sqrt(size[agg])
    return Pt


def _patterns(rp, c, agg, n_agg):
    """Expected structures, from the neighbourhood sets (no arithmetic)."""
    n = rp.size - 1
    nb = [set([i]) | set(c[rp[i]:rp[i + 1]].tolist()) for i in range(n)]
    prow = [sorted({int(agg[j]) for j in nb[i]}) for i in range(n)]
    aprow = [sorted(set().union(*[set(prow[j]) for j in nb[i]])) for i in range(n)]
    crow = [set() for _ in range(n_agg)]
    for i in range(n):
        for a in prow[i]:
            crow[a] |= set(aprow[i])
    return prow, [sorted(s) for s in crow]


CASES = {
    "grid2d_8x7": lambda: graphs.grid2d_5pt(8, 7),
    "grid27_5x5x4": lambda: graphs.grid3d_27pt(5, 5, 4),
    "chunglu_300": lambda: graphs.chung_lu(300, 6.0, 2.1, 60, seed=2),
    "er_120": lambda: graphs.erdos_renyi(120, 0.05, seed=4),
    "union": lambda: graphs.disjoint_union([graphs.grid2d_5pt(5, 4), graphs.path(9),
                                            graphs.star(12, 3)]),
}


@pytest.mark.parametrize("omega", [2.0 / 3.0, 0.5, 1.25])
@pytest.mark.parametrize("name", sorted(CASES))
def test_equals_dense_product(name, omega):
    rp, c = CASES[name]()
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 3, shift=0.2)
    agg, na = oracle.aggregate(rp, c, 0)
    prow, pcol, pval, crow, ccol, cval = oracle.smoothed(rp, c, val, diag, agg, na, omega)
    A = _dense(rp, c, val, diag)
    P = (np.eye(n) - omega * np.diag(1.0 / diag) @ A) @ _tentative(agg, na)
    Ac = P.T @ A @ P
    got_p = _to_dense(prow, pcol, pval, n, na)
    got_c = _to_dense(crow, ccol, cval, na, na)
    assert np.allclose(got_p, P, rtol=1e-13, atol=1e-14 * np.abs(P).max())
    assert np.allclose(got_c, Ac, rtol=1e-12, atol=1e-13 * np.abs(Ac).max())
    # structures: closed neighbourhoods' aggregates, and their unions
    want_p, want_c = _patterns(rp, c, agg, na)
    assert [pcol[prow[i]:prow[i + 1]].tolist() for i in range(n)] == want_p
    assert [ccol[crow[a]:crow[a + 1]].tolist() for a in range(na)] == want_c


@pytest.mark.parametrize("name", sorted(CASES))
def test_omega_zero_gives_the_tentative_prolongator(name):
    rp, c = CASES[name]()
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 5, shift=0.5)
    agg, na = oracle.aggregate(rp, c, 0)
    prow, pcol, pval, crow, ccol, cval = oracle.smoothed(rp, c, val, diag, agg, na, 0.0)
    size = np.bincount(agg, minlength=na)
    for i in range(n):
        for p in range(prow[i], prow[i + 1]):
            want = 1.0 / np.sqrt(float(size[agg[i]])) if pcol[p] == agg[i] else 0.0
            assert pval[p] == want, (i, pcol[p])
    # then P^T A P is the Galerkin operator of the tentative prolongator
    gr, gc, gv, gd = oracle.galerkin(rp, c, val, diag, agg, na)
    G = _to_dense(gr, gc, gv, na, na) + np.diag(gd)
    assert np.allclose(_to_dense(crow, ccol, cval, na, na), G, rtol=1e-13,
                       atol=1e-14 * np.abs(G).max())


def _exact(rp, c, val, diag, agg, na, omega):
    """P and P^T A P in rational arithmetic (every scaling a power of two)."""
    n = rp.size - 1
    F = Fraction
    size = np.bincount(agg, minlength=na)
    inv_sqrt = {}
    for s in set(size.tolist()):
        r = int(round(s ** 0.5))
        assert r * r == s and (r & (r - 1)) == 0, "sizes must be powers of four"
        inv_sqrt[s] = F(1, r)
    A = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        A[i][i] = F(diag[i])
        for e in range(rp[i], rp[i + 1]):
            A[i][int(c[e])] = F(val[e])
    Pt = [[F(0)] * na for _ in range(n)]
    for i in range(n):
        Pt[i][agg[i]] = inv_sqrt[int(size[agg[i]])]
    w = F(omega)
    P = [[Pt[i][a] - w / A[i][i] * sum(A[i][j] * Pt[j][a] for j in range(n))
          for a in range(na)] for i in range(n)]
    AP = [[sum(A[i][j] * P[j][b] for j in range(n)) for b in range(na)] for i in range(n)]
    Ac = [[sum(P[i][a] * AP[i][b] for i in range(n)) for b in range(na)] for a in range(na)]
    return P, Ac


@pytest.mark.parametrize("case", ["path8", "grid4x4", "grid4x4_1"])
def test_exact_on_dyadic_values(case):
    # integer matrix, aggregates of 4 (or 1) vertices, omega / d_i a power of
    # two: every intermediate value is a short dyadic fraction, so every sum
    # is exact and the result must equal rational arithmetic bit for bit
    if case == "path8":
        rp, c = graphs.path(8)
        agg = np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32)
        diag_v, omega = 4.0, 0.5
    else:
        rp, c = graphs.grid2d_5pt(4, 4)
        ij = [(k % 4, k // 4) for k in range(16)]
        agg = np.array([(i // 2) + 2 * (j // 2) for i, j in ij], np.int32)
        diag_v, omega = 8.0, 0.75
        if case == "grid4x4_1":
            agg = agg.copy()
            agg[agg == 3] = [3, 4, 5, 6]  # one aggregate split into singletons
    na = int(agg.max()) + 1
    val = -np.ones(int(rp[-1]))
    diag = np.full(rp.size - 1, diag_v)
    prow, pcol, pval, crow, ccol, cval = oracle.smoothed(rp, c, val, diag, agg, na, omega)
    P, Ac = _exact(rp, c, val, diag, agg, na, omega)
    for i in range(rp.size - 1):
        for p in range(prow[i], prow[i + 1]):
            assert pval[p] == float(P[i][pcol[p]]), (i, pcol[p])
    for a in range(na):
        for q in range(crow[a], crow[a + 1]):
            assert cval[q] == float(Ac[a][ccol[q]]), (a, ccol[q])


@pytest.mark.parametrize("name", ["grid2d_8x7", "grid27_5x5x4", "er_120"])
def test_constant_vector_of_a_laplacian(name):
    # zero row sums: (I - omega D^-1 A) 1 = 1, so P s = 1 with s_a = sqrt(n_a),
    # and P^T A P s = P^T A 1 = 0
    rp, c = CASES[name]()
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 1, shift=0.0)
    agg, na = oracle.aggregate(rp, c, 0)
    prow, pcol, pval, crow, ccol, cval = oracle.smoothed(rp, c, val, diag, agg, na, 2.0 / 3.0)
    s = np.sqrt(np.bincount(agg, minlength=na).astype(float))
    Ps = _to_dense(prow, pcol, pval, n, na) @ s
    assert np.allclose(Ps, 1.0, rtol=0, atol=1e-13)
    Acs = _to_dense(crow, ccol, cval, na, na) @ s
    assert np.abs(Acs).max() <= 1e-12 * np.abs(cval).max() * np.sqrt(n)


@pytest.mark.parametrize("name", sorted(CASES))
def test_symmetric_matrix_gives_symmetric_coarse_operator(name):
    rp, c = CASES[name]()
    val, diag = graphs.matrix_values(rp, c, 7, shift=0.3)
    agg, na = oracle.aggregate(rp, c, 0)
    _, _, _, crow, ccol, cval = oracle.smoothed(rp, c, val, diag, agg, na, 0.6)
    C = _to_dense(crow, ccol, cval, na, na)
    assert np.array_equal(C != 0, C.T != 0) or np.allclose(C, C.T, atol=1e-14)
    assert np.allclose(C, C.T, rtol=1e-13, atol=1e-14 * np.abs(C).max())
