"""Seeded synthetic graph generators (symmetric CSR, no self-loops, no duplicates).

This module builds inputs only; it holds none of the MIS-2 or aggregation
arithmetic, so both the HIP library's tests and the CPU oracle can draw the
same bytes from it.  Every graph comes back as (row_ptr int64[n+1],
col int32[nnz]) with ascending columns in every row.

Workload shapes follow the paper's test matrices (Section VI, Table II):
structured Laplace stencils on natural-order grids (Galeri's Laplace3D is a
7-point 100^3 grid, its Elasticity3D a 27-point grid with 3 unknowns per
point), and stand-ins for the irregular SuiteSparse matrices.
"""
import numpy as np


def _offsets(dim, kind):
    if dim == 2 and kind == 5:
        offs = [(0, -1), (-1, 0), (1, 0), (0, 1)]  # (di, dj) sorted by dj then di
        return [(di, dj, 0) for di, dj in offs]
    if dim == 3 and kind == 7:
        return [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if dim == 3 and kind == 27:
        return [(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)
                if (di, dj, dk) != (0, 0, 0)]
    raise ValueError("unsupported stencil")


def _stencil(nx, ny, nz, offs):
    """Natural ordering id = i + nx*j + nx*ny*k.  Offsets are listed in
    increasing (dk, dj, di) order, which is increasing neighbour id, so the
    row-major compression below yields sorted rows without a sort."""
    n = nx * ny * nz
    if n == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32)
    idx = np.arange(n, dtype=np.int64)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    nb = np.empty((n, len(offs)), np.int64)
    ok = np.empty((n, len(offs)), bool)
    for t, (di, dj, dk) in enumerate(offs):
        ii, jj, kk = i + di, j + dj, k + dk
        ok[:, t] = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
        nb[:, t] = idx + di + nx * dj + nx * ny * dk
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(ok.sum(axis=1), out=row_ptr[1:])
    col = nb[ok].astype(np.int32)
    return row_ptr, col


def grid2d_5pt(nx, ny):
    """2D 5-point Laplacian graph, id = i + nx*j."""
    return _stencil(nx, ny, 1, _offsets(2, 5))


def grid3d_7pt(nx, ny, nz):
    """3D 7-point Laplacian graph (Galeri Laplace3D shape), id = i + nx*j + nx*ny*k."""
    return _stencil(nx, ny, nz, _offsets(3, 7))


def grid3d_27pt(nx, ny, nz):
    """3D 27-point Laplacian graph: every vertex of the 3x3x3 box around a point."""
    return _stencil(nx, ny, nz, _offsets(3, 27))


def elasticity3d(nx, ny, nz, dof=3):
    """Graph of a 27-point stencil with `dof` unknowns per grid point (the shape
    of Galeri's Elasticity3D): unknown id = dof*point + d, coupled to every
    unknown of every point in the 3x3x3 box around its point, itself excluded."""
    npt = nx * ny * nz
    if npt == 0:
        return np.zeros(1, np.int64), np.zeros(0, np.int32)
    offs = [(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)]
    idx = np.arange(npt, dtype=np.int64)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    nb = np.empty((npt, 27), np.int64)
    ok = np.empty((npt, 27), bool)
    for t, (di, dj, dk) in enumerate(offs):
        ii, jj, kk = i + di, j + dj, k + dk
        ok[:, t] = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
        nb[:, t] = idx + di + nx * dj + nx * ny * dk
    # unknown (p, d) couples to (q, e) for every valid box point q and every e,
    # in increasing order of q*dof + e, minus itself
    cols = (nb[:, None, :, None] * dof + np.arange(dof)[None, None, None, :])
    cols = np.broadcast_to(cols, (npt, dof, 27, dof))
    mask = np.broadcast_to(ok[:, None, :, None], (npt, dof, 27, dof)).copy()
    mask[:, np.arange(dof), 13, np.arange(dof)] = False  # offset 13 is (0,0,0)
    row_ptr = np.zeros(npt * dof + 1, np.int64)
    np.cumsum(mask.reshape(npt * dof, -1).sum(axis=1), out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    return row_ptr, col


def from_edges(n, u, v):
    """Symmetric, deduplicated CSR from an undirected edge list; self-pairs
    dropped.  Rows come out with ascending columns."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = np.concatenate([u, v])
    b = np.concatenate([v, u])
    key = np.unique(a * np.int64(max(n, 1)) + b)
    r = key // max(n, 1)
    c = key % max(n, 1)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return row_ptr, c.astype(np.int32)


def permute(row_ptr, col, perm):
    """Relabel vertex v as perm[v]; returns sorted CSR."""
    n = row_ptr.size - 1
    deg = np.diff(row_ptr)
    r = np.repeat(np.arange(n, dtype=np.int64), deg)
    return from_edges(n, perm[r], perm[col.astype(np.int64)])


def chung_lu(n, mean_deg=16.0, gamma=2.1, cap=20000, seed=1, permute_ids=True):
    """Chung-Lu power-law graph.  Weights w_i = c (i+1)^(-1/(gamma-1)), capped at
    `cap`, with c chosen (iteratively, re-capping) so that mean(w) = mean_deg;
    m = n*mean_deg/2 endpoint pairs are drawn i.i.d. with P(i) ~ w_i by inverse
    CDF from numpy's PCG64 (default_rng(seed)); self-pairs dropped, symmetrised,
    deduplicated; then a seeded random relabelling so hubs are not at low ids."""
    if n <= 1:
        return np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    cap = min(cap, n - 1)
    base = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (gamma - 1.0))
    c = mean_deg / base.mean()
    for _ in range(100):
        w = np.minimum(c * base, cap)
        mw = w.mean()
        if abs(mw - mean_deg) < 1e-9 * mean_deg:
            break
        c *= mean_deg / mw
    w = np.minimum(c * base, cap)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    rng = np.random.default_rng(seed)
    m = int(round(n * mean_deg / 2.0))
    # Inverse-CDF draws of the two endpoint columns.  Each column's uniforms
    # are sorted before the search (a cache-friendly search) and the second
    # column is then shuffled; a sorted i.i.d. column paired with an
    # independent shuffled i.i.d. column has the law of i.i.d. pairs.
    u = np.searchsorted(cdf, np.sort(rng.random(m)), side="right").astype(np.int64)
    v = np.searchsorted(cdf, np.sort(rng.random(m)), side="right").astype(np.int64)
    v = v[rng.permutation(m)]
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    if permute_ids:
        perm = rng.permutation(n).astype(np.int64)
        u, v = perm[u], perm[v]
    return from_edges(n, u, v)


def dropped_7pt(side, p_drop=0.1, seed=0):
    """3D 7-point side^3 subdomain with every undirected edge dropped
    independently with probability p_drop (both directions together)."""
    row_ptr, col = grid3d_7pt(side, side, side)
    n = row_ptr.size - 1
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    c = col.astype(np.int64)
    up = r < c
    ru, cu = r[up], c[up]
    rng = np.random.default_rng(seed)
    keep = rng.random(ru.size) >= p_drop
    return from_edges(n, ru[keep], cu[keep])


def batch_subdomains(num=512, lo=8, hi=48, p_drop=0.1, seed=2):
    """`num` dropped-edge 7-point subdomains with side ~ U{lo..hi} drawn from
    default_rng(seed); graph g uses seed (seed, g) for its edge drops."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=num)
    out = []
    for g, s in enumerate(sides):
        ss = np.random.SeedSequence([seed, g])
        out.append(dropped_7pt(int(s), p_drop, seed=ss))
    return out


def erdos_renyi(n, p, seed=0):
    """G(n, p) random graph (small test sizes)."""
    rng = np.random.default_rng(seed)
    if n < 2:
        return np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return from_edges(n, iu[keep], ju[keep])


def random_regular_ish(n, deg, seed=0):
    """Random graph with about n*deg/2 uniformly drawn edges (test sizes)."""
    rng = np.random.default_rng(seed)
    m = n * deg // 2
    return from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m))


def path(n):
    if n < 2:
        return np.zeros(n + 1, np.int64), np.zeros(0, np.int32)
    a = np.arange(n - 1)
    return from_edges(n, a, a + 1)


def cycle(n):
    a = np.arange(n)
    return from_edges(n, a, (a + 1) % n)


def complete(n):
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju)


def star(n, center=0):
    leaves = np.array([v for v in range(n) if v != center], np.int64)
    return from_edges(n, np.full(leaves.size, center), leaves)


def edgeless(n):
    return np.zeros(n + 1, np.int64), np.zeros(0, np.int32)



def serving_pool(count, seed=3, n_lo=1_000, n_hi=10_000_000):
    """Coarsening jobs of the serving workload: n log-uniform on [n_lo, n_hi];
    40% 2D 5-point (side round(sqrt n)), 40% 3D 27-point (side round(cbrt n)),
    20% Chung-Lu (n, mean degree 16, exponent 2.1, cap min(20000, n - 1)).
    Returns [(kind, (row_ptr, col))]."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        kind = rng.choice(3, p=[0.4, 0.4, 0.2])
        if kind == 0:
            s = max(2, int(round(n ** 0.5)))
            out.append(("2d5", grid2d_5pt(s, s)))
        elif kind == 1:
            s = max(2, int(round(n ** (1 / 3))))
            out.append(("3d27", grid3d_27pt(s, s, s)))
        else:
            out.append(("chunglu", chung_lu(n, 16.0, 2.1, min(20000, n - 1), seed=100 + i)))
    return out

def disjoint_union(graphs):
    """Block-diagonal union; vertex ids of graph g are offset by the sizes of
    graphs 0..g-1."""
    rps, cols = [np.zeros(1, np.int64)], []
    off_v, off_e = 0, 0
    for rp, c in graphs:
        n = rp.size - 1
        rps.append(rp[1:] + off_e)
        cols.append(c.astype(np.int64) + off_v)
        off_v += n
        off_e += int(rp[-1])
    return np.concatenate(rps), (np.concatenate(cols) if cols else np.zeros(0)).astype(np.int32)


def matrix_values(row_ptr, col, seed=0, shift=0.1):
    """Seeded values for a CSR pattern, to make a symmetric, strictly
    diagonally dominant M-matrix (the kind of system the Gauss-Seidel of
    Algorithm 4 is run on): off-diagonal entry (i, j) = -w with w uniform in
    [0.5, 1.5) drawn from the unordered pair {i, j}, and diagonal entry i =
    shift + the sum of its row's w.  Returns (val float64[nnz], diag
    float64[n])."""
    n = row_ptr.size - 1
    r = np.repeat(np.arange(n, dtype=np.uint64), np.diff(row_ptr).astype(np.int64))
    c = col.astype(np.uint64)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    with np.errstate(over="ignore"):
        z = lo * np.uint64(0x9E3779B97F4A7C15) ^ hi ^ (np.uint64(seed) << np.uint64(32))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    w = 0.5 + (z >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    diag = shift + np.bincount(r.astype(np.int64), weights=w, minlength=n)
    return -w, diag
