"""Pins of the oracle's cluster multicolor Gauss-Seidel (Algorithm 4, Section
III-C): the colouring by brute force (Jones-Plassmann written out again from
its statement), the plan's structure, and the sweeps against the matrix form
of a Gauss-Seidel step in the plan's row order, (D + L) x' = b - U x with L
and U the parts of A before and after each row in that order, solved as a
dense triangular system, plus convergence to A^-1 b."""
import numpy as np
import pytest
from scipy.linalg import solve_triangular

import oracle
from bruteforce import adjacency, prio_hash, tuple_of
from paper_2204_02934_amd import graphs


def _jp(rp, c, seed=0):
    n = rp.size - 1
    adj = adjacency(rp, c)
    t = [tuple_of(prio_hash(seed, 0, v), v, n) for v in range(n)]
    color = [-1] * n
    while -1 in color:
        picked = [v for v in range(n) if color[v] == -1 and
                  all(t[v] < t[w] for w in adj[v] if color[w] == -1)]
        new = {}
        for v in picked:
            taken = {color[w] for w in adj[v] if color[w] >= 0}
            new[v] = min(set(range(len(adj[v]) + 1)) - taken)
        for v, k in new.items():
            color[v] = k
    return color


def test_coloring_matches_jones_plassmann_brute_force():
    rng = np.random.default_rng(21)
    for trial in range(40):
        n = int(rng.integers(1, 60))
        rp, c = graphs.erdos_renyi(n, float(rng.uniform(0.03, 0.4)), seed=2100 + trial)
        col, nc, _ = oracle.color_jp(rp, c, trial % 3)
        want = _jp(rp, c, trial % 3)
        assert list(col) == want
        assert nc == (max(want) + 1 if n else 0)


def test_coloring_is_proper_on_larger_graphs():
    for rp, c in [graphs.grid3d_27pt(12, 11, 10), graphs.chung_lu(3000, 10.0, 2.1, 400, seed=5)]:
        col, nc, _ = oracle.color_jp(rp, c, 0)
        src = np.repeat(np.arange(rp.size - 1), np.diff(rp))
        assert not np.any(col[src] == col[c])
        assert set(col.tolist()) == set(range(nc))


def _dense(rp, c, val, diag):
    n = rp.size - 1
    A = np.diag(diag)
    src = np.repeat(np.arange(n), np.diff(rp))
    A[src, c] = val
    return A


def _check_plan(rp, c, p, point):
    n = rp.size - 1
    rows = p["rows"]
    assert sorted(rows.tolist()) == list(range(n))
    coff, koff = p["cluster_off"], p["color_off"]
    assert coff[0] == 0 and coff[-1] == n and koff[0] == 0 and koff[-1] == p["n_clusters"]
    pos_cluster = np.empty(n, np.int64)
    for k in range(p["n_clusters"]):
        seg = rows[coff[k]:coff[k + 1]]
        assert len(seg) > 0 and np.all(np.diff(seg) > 0)  # rows of a cluster by id
        assert len(set(p["cluster"][seg].tolist())) == 1
        pos_cluster[seg] = k
    color_of_row = np.empty(n, np.int64)
    for col_ in range(p["n_colors"]):
        ks = range(koff[col_], koff[col_ + 1])
        ids = [int(p["cluster"][rows[coff[k]]]) for k in ks]
        assert ids == sorted(ids)  # clusters of a colour by id
        assert all(p["cluster_color"][a] == col_ for a in ids)
        for k in ks:
            color_of_row[rows[coff[k]:coff[k + 1]]] = col_
    # rows of different clusters with the same colour are never adjacent
    src = np.repeat(np.arange(n), np.diff(rp))
    same = (color_of_row[src] == color_of_row[c]) & (pos_cluster[src] != pos_cluster[c])
    assert not same.any()
    if point:
        assert np.array_equal(p["cluster"], np.arange(n))


@pytest.mark.parametrize("point", [False, True])
def test_plan_structure(point):
    for rp, c in [graphs.grid3d_27pt(9, 8, 7), graphs.chung_lu(1500, 8.0, 2.1, 200, seed=3),
                  graphs.path(40), graphs.edgeless(7)]:
        _check_plan(rp, c, oracle.cgs_plan(rp, c, 1, point=point), point)


def _gs_matrix_step(A, order, b, x, backward=False):
    # one Gauss-Seidel sweep in the given row order as a triangular solve
    P = np.asarray(order)
    Ap = A[np.ix_(P, P)]
    if backward:
        Ap = Ap[::-1, ::-1]
        P = P[::-1]
    L = np.tril(Ap)  # diagonal and the rows updated before
    U = np.triu(Ap, 1)
    xp = solve_triangular(L, b[P] - U @ x[P], lower=True)
    out = x.copy()
    out[P] = xp
    return out


@pytest.mark.parametrize("point", [False, True])
@pytest.mark.parametrize("symmetric", [False, True])
def test_sweeps_equal_the_matrix_form(point, symmetric):
    rng = np.random.default_rng(5)
    for rp, c in [graphs.grid3d_27pt(7, 6, 5), graphs.chung_lu(600, 6.0, 2.1, 80, seed=9),
                  graphs.grid2d_5pt(11, 9)]:
        n = rp.size - 1
        val, diag = graphs.matrix_values(rp, c, 2)
        A = _dense(rp, c, val, diag)
        p = oracle.cgs_plan(rp, c, 0, point=point)
        b = rng.standard_normal(n)
        x0 = rng.standard_normal(n)
        got = oracle.cgs_apply(rp, c, val, diag, p, b, x0, sweeps=2, symmetric=symmetric)
        want = x0.copy()
        for _ in range(2):
            want = _gs_matrix_step(A, p["rows"], b, want)
            if symmetric:
                want = _gs_matrix_step(A, p["rows"], b, want, backward=True)
        np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_sweeps_converge_to_the_solution():
    rp, c = graphs.grid3d_27pt(8, 8, 8)
    n = rp.size - 1
    val, diag = graphs.matrix_values(rp, c, 0, shift=3.0)  # well conditioned
    A = _dense(rp, c, val, diag)
    b = np.random.default_rng(2).standard_normal(n)
    p = oracle.cgs_plan(rp, c, 0)
    x = oracle.cgs_apply(rp, c, val, diag, p, b, np.zeros(n), sweeps=200, symmetric=True)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-9)


def test_edgeless_is_one_jacobi_step():
    rp, c = graphs.edgeless(6)
    val, diag = graphs.matrix_values(rp, c, 0)
    p = oracle.cgs_plan(rp, c, 0, point=True)
    b = np.arange(1.0, 7.0)
    x = oracle.cgs_apply(rp, c, val, diag, p, b, np.zeros(6), sweeps=1)
    assert p["n_colors"] == 1 and np.array_equal(x, b / diag)
