"""ctypes wrapper around oracle.c, the plain CPU reference implementation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the HIP library; the library itself
never imports it.  The arithmetic lives in oracle.c; this file only marshals
numpy arrays and runs the multilevel loop (a plain Python loop over
aggregate + quotient, Sections I-II of the paper: coarsen recursively until
the graph is below a size threshold).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def build_oracle(force=True, parallel=False):
    """Compile oracle.c with gcc into oracle/liboracle.so (sequential, the
    default) or, with parallel, into oracle/liboracle_omp.so with the pure-map
    phase loops of Algorithm 1 under OpenMP (same results; used only to time
    the oracle on every host core)."""
    global _lib
    out = _LIB_OMP if parallel else _LIB
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    extra = ["-DORACLE_OMP", "-fopenmp"] if parallel else []
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-Wall", "-Wextra", "-fPIC",
                           "-shared"] + extra + [_SRC, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    if not parallel:
        _lib = None
    return out


class use_library:
    """Context manager: the oracle functions below call the build at `path`
    (e.g. the OpenMP build) instead of the default one while it is active."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        os.environ["MIS2_ORACLE_LIB"], self.env = self.path, os.environ.get("MIS2_ORACLE_LIB")
        _lib = None
        _get()
        return self

    def __exit__(self, *exc):
        global _lib
        if self.env is None:
            os.environ.pop("MIS2_ORACLE_LIB", None)
        else:
            os.environ["MIS2_ORACLE_LIB"] = self.env
        _lib = self.saved
        return False


def _get():
    """The oracle library, loaded once.  MIS2_ORACLE_LIB names another build
    of oracle.c to load instead (the mutation tests plant mistakes in copies
    and check that the pins catch them)."""
    global _lib
    if _lib is None:
        path = os.environ.get("MIS2_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB):
                build_oracle()
        lib = ctypes.CDLL(path)
        lib.oracle_xorshift64star.restype = ctypes.c_uint64
        lib.oracle_xorshift64star.argtypes = [ctypes.c_uint64]
        lib.oracle_hash.restype = ctypes.c_uint64
        lib.oracle_hash.argtypes = [ctypes.c_uint64] * 3
        lib.oracle_id_bits.restype = ctypes.c_int
        lib.oracle_id_bits.argtypes = [ctypes.c_int64]
        lib.oracle_pack.restype = ctypes.c_uint32
        lib.oracle_pack.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int]
        lib.oracle_mis2_ex.restype = ctypes.c_int
        lib.oracle_mis2_ex.argtypes = [
            ctypes.c_int64, _i64p, _i32p, _u8p, ctypes.c_uint64, _u64p, ctypes.c_int32,
            _u8p, _i32p, _i64p, ctypes.c_int32, _u32p, _u32p, _u32p, ctypes.c_int32]
        lib.oracle_aggregate_ex.restype = ctypes.c_int
        lib.oracle_aggregate_ex.argtypes = [
            ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64, _i32p, _i64p, _i64p, _u8p,
            _i64p, _i64p, ctypes.c_int32]
        lib.oracle_xorshift64.restype = ctypes.c_uint64
        lib.oracle_xorshift64.argtypes = [ctypes.c_uint64]
        lib.oracle_mis2_ablation.restype = ctypes.c_int
        lib.oracle_mis2_ablation.argtypes = [
            ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64, ctypes.c_int, _u8p, _i32p, _i64p,
            ctypes.c_int32]
        _f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_color_jp.restype = ctypes.c_int
        lib.oracle_color_jp.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64, _i32p,
                                        _i32p, _i32p]
        lib.oracle_cgs_plan.restype = ctypes.c_int
        lib.oracle_cgs_plan.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64,
                                        ctypes.c_int, _i32p, _i32p, _i32p, _i64p, _i64p, _i64p,
                                        _i32p]
        lib.oracle_cgs_apply.restype = ctypes.c_int
        lib.oracle_cgs_apply.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _i32p,
                                         _i64p, _i64p, ctypes.c_int32, _f64p, _f64p,
                                         ctypes.c_int32, ctypes.c_int]
        lib.oracle_aggregate_basic.restype = ctypes.c_int
        lib.oracle_aggregate_basic.argtypes = [
            ctypes.c_int64, _i64p, _i32p, ctypes.c_uint64, _i32p, _i64p, _u8p, _i64p]
        lib.oracle_quotient.restype = ctypes.c_int64
        lib.oracle_quotient.argtypes = [
            ctypes.c_int64, _i64p, _i32p, _i32p, ctypes.c_int64, _i64p, _i32p, ctypes.c_int64]
        lib.oracle_galerkin.restype = ctypes.c_int
        lib.oracle_galerkin.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _i32p,
                                        ctypes.c_int64, _i64p, _i32p, _f64p, _f64p]
        lib.oracle_smoothed.restype = ctypes.c_int
        lib.oracle_smoothed.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p, _i32p,
                                        ctypes.c_int64, ctypes.c_double, _i64p, _i32p, _f64p,
                                        ctypes.c_int64, _i64p, _i32p, _f64p, ctypes.c_int64,
                                        _i64p, _i64p]
        _lib = lib
    return _lib


def _ptr(a, t):
    if a is None:
        return ctypes.cast(None, t)
    return a.ctypes.data_as(t)


def _csr(row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)  # a valid pointer for an edgeless graph
    return row_ptr, col


class OracleError(RuntimeError):
    pass


def xorshift64star(x):
    return int(_get().oracle_xorshift64star(x & 0xFFFFFFFFFFFFFFFF))


def hash_priority(seed, it, v):
    return int(_get().oracle_hash(seed, it, v))


def id_bits(n):
    return int(_get().oracle_id_bits(n))


def pack(prio, v, b):
    return int(_get().oracle_pack(prio & 0xFFFFFFFFFFFFFFFF, v, b))


TRACE_CAP = 4096


def mis2_ex(row_ptr, col, seed=0, active=None, prio=None, history=0):
    """Alg. 1 with everything exposed.  Returns a dict with status (u8[n]),
    n_iters, trace (int64[rounds, 4]) and, when history > 0, T/M/D snapshots
    of shape [min(rounds, history), n]."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    status = np.zeros(max(n, 1), np.uint8)
    it = ctypes.c_int32(0)
    trace = np.zeros((TRACE_CAP, 4), np.int64)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    pr = None
    rounds = 0
    if prio is not None:
        pr = np.ascontiguousarray(prio, dtype=np.uint64)
        rounds = pr.shape[0]
        pr = pr.reshape(-1)
    hist = None
    if history:
        hist = [np.zeros((history, max(n, 1)), np.uint32) for _ in range(3)]
    rc = _get().oracle_mis2_ex(
        n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), _ptr(act, _u8p), seed,
        _ptr(pr, _u64p), rounds, _ptr(status, _u8p), ctypes.byref(it),
        _ptr(trace, _i64p), TRACE_CAP,
        *(_ptr(h, _u32p) for h in (hist or [None] * 3)), history)
    if rc:
        raise OracleError("oracle_mis2_ex returned %d" % rc)
    r = it.value
    out = {"status": status[:n], "n_iters": r, "trace": trace[:min(r, TRACE_CAP)].copy()}
    if history:
        k = min(r, history)
        out["T"], out["M"], out["D"] = (h[:k, :n] for h in hist)
    return out


def mis2(row_ptr, col, seed=0):
    """Alg. 1: returns (status u8[n], n_iters)."""
    o = mis2_ex(row_ptr, col, seed)
    return o["status"], o["n_iters"]


def aggregate(row_ptr, col, seed=0, detail=False):
    """Alg. 3: returns (agg int32[n], n_agg) or, with detail, a dict that also
    holds per-phase counts, root marks and the two MIS-2 traces."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    agg = np.zeros(max(n, 1), np.int32)
    nagg = ctypes.c_int64(0)
    info = np.zeros(8, np.int64)
    roots = np.zeros(max(n, 1), np.uint8)
    t1 = np.zeros((TRACE_CAP, 4), np.int64)
    t2 = np.zeros((TRACE_CAP, 4), np.int64)
    rc = _get().oracle_aggregate_ex(
        n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), seed, _ptr(agg, _i32p),
        ctypes.byref(nagg), _ptr(info, _i64p), _ptr(roots, _u8p),
        _ptr(t1, _i64p), _ptr(t2, _i64p), TRACE_CAP)
    if rc:
        raise OracleError("oracle_aggregate_ex returned %d" % rc)
    if not detail:
        return agg[:n], int(nagg.value)
    return {"agg": agg[:n], "n_agg": int(nagg.value), "n1": int(info[0]),
            "n2": int(info[1]), "joined": int(info[2]), "iters1": int(info[3]),
            "iters2": int(info[4]), "m2": int(info[5]), "unagg1": int(info[6]),
            "roots": roots[:n], "trace1": t1[:min(int(info[3]), TRACE_CAP)].copy(),
            "trace2": t2[:min(int(info[4]), TRACE_CAP)].copy()}


PRIO_FIXED = 1     # priorities drawn once (Bell et al.)
PRIO_XORSHIFT = 2  # f = xorshift instead of xorshift* (Table I's "Xor Hash")


def xorshift64(x):
    return int(_get().oracle_xorshift64(x & 0xFFFFFFFFFFFFFFFF))


def mis2_ablation(row_ptr, col, seed=0, pflags=0):
    """Alg. 1 with the priorities of the Section V-A comparison: returns
    (status u8[n], n_iters, trace int64[rounds, 4])."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    status = np.zeros(max(n, 1), np.uint8)
    it = ctypes.c_int32(0)
    trace = np.zeros((TRACE_CAP, 4), np.int64)
    rc = _get().oracle_mis2_ablation(n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), seed, pflags,
                                     _ptr(status, _u8p), ctypes.byref(it), _ptr(trace, _i64p),
                                     TRACE_CAP)
    if rc:
        raise OracleError("oracle_mis2_ablation returned %d" % rc)
    r = it.value
    return status[:n], r, trace[:min(r, TRACE_CAP)].copy()


def aggregate_basic(row_ptr, col, seed=0, detail=False):
    """Alg. 2 (basic MIS-2 coarsening): returns (agg int32[n], n_agg) or,
    with detail, a dict that also holds the root marks and the number of
    vertices that joined a neighbour's aggregate."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    agg = np.zeros(max(n, 1), np.int32)
    nagg = ctypes.c_int64(0)
    roots = np.zeros(max(n, 1), np.uint8)
    joined = ctypes.c_int64(0)
    rc = _get().oracle_aggregate_basic(
        n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), seed, _ptr(agg, _i32p),
        ctypes.byref(nagg), _ptr(roots, _u8p), ctypes.byref(joined))
    if rc:
        raise OracleError("oracle_aggregate_basic returned %d" % rc)
    if not detail:
        return agg[:n], int(nagg.value)
    return {"agg": agg[:n], "n_agg": int(nagg.value), "roots": roots[:n],
            "joined": int(joined.value)}


_f64p = ctypes.POINTER(ctypes.c_double)


def color_jp(row_ptr, col, seed=0):
    """Jones-Plassmann colouring with fixed hash priorities (the reading of
    Algorithm 4's colouring): returns (color int32[n], n_colors, rounds)."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    color = np.zeros(max(n, 1), np.int32)
    nc, r = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = _get().oracle_color_jp(n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), seed,
                                _ptr(color, _i32p), ctypes.byref(nc), ctypes.byref(r))
    if rc:
        raise OracleError("oracle_color_jp returned %d" % rc)
    return color[:n], nc.value, r.value


def cgs_plan(row_ptr, col, seed=0, point=False):
    """Algorithm 4's setup: dict with cluster (int32[n]), cluster_color,
    rows (sweep order), cluster_off, color_off, n_clusters, n_colors."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    cl = np.zeros(max(n, 1), np.int32)
    cc = np.zeros(max(n, 1), np.int32)
    rows = np.zeros(max(n, 1), np.int32)
    coff = np.zeros(n + 1, np.int64)
    koff = np.zeros(n + 1, np.int64)
    ncl, nco = ctypes.c_int64(0), ctypes.c_int32(0)
    rc = _get().oracle_cgs_plan(n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), seed, int(point),
                                _ptr(cl, _i32p), _ptr(cc, _i32p), _ptr(rows, _i32p),
                                _ptr(coff, _i64p), _ptr(koff, _i64p), ctypes.byref(ncl),
                                ctypes.byref(nco))
    if rc:
        raise OracleError("oracle_cgs_plan returned %d" % rc)
    k, c = ncl.value, nco.value
    return {"cluster": cl[:n], "cluster_color": cc[:k], "rows": rows[:n],
            "cluster_off": coff[:k + 1], "color_off": koff[:c + 1], "n_clusters": k,
            "n_colors": c}


def cgs_apply(row_ptr, col, val, diag, plan, b, x0, sweeps=1, symmetric=False):
    """sweeps applications of Algorithm 4 to a copy of x0 (float64)."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    val = np.ascontiguousarray(val, dtype=np.float64)
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    rows = np.ascontiguousarray(plan["rows"], dtype=np.int32)
    coff = np.ascontiguousarray(plan["cluster_off"], dtype=np.int64)
    koff = np.ascontiguousarray(plan["color_off"], dtype=np.int64)
    if val.size == 0:
        val = np.zeros(1)
    rc = _get().oracle_cgs_apply(n, _ptr(row_ptr, _i64p), _ptr(col, _i32p), _ptr(val, _f64p),
                                 _ptr(diag, _f64p), _ptr(rows, _i32p), _ptr(coff, _i64p),
                                 _ptr(koff, _i64p), plan["n_colors"], _ptr(b, _f64p),
                                 _ptr(x, _f64p), sweeps, int(symmetric))
    if rc:
        raise OracleError("oracle_cgs_apply returned %d" % rc)
    return x


def quotient(row_ptr, col, agg, n_agg):
    """Coarse (quotient) graph of an aggregation: returns (row_ptr, col)."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    if agg.size == 0:
        agg = np.zeros(1, np.int32)
    cap = int(row_ptr[-1]) if n > 0 else 0
    crow = np.zeros(n_agg + 1, np.int64)
    ccol = np.zeros(max(cap, 1), np.int32)
    m = _get().oracle_quotient(n, _ptr(row_ptr, _i64p), _ptr(col, _i32p),
                               _ptr(agg, _i32p), n_agg, _ptr(crow, _i64p),
                               _ptr(ccol, _i32p), cap)
    if m < 0:
        raise OracleError("oracle_quotient returned %d" % m)
    return crow, ccol[:m].copy()


def galerkin(row_ptr, col, val, diag, agg, n_agg, crow=None, ccol=None):
    """Galerkin coarse operator P^T A P of an aggregation with the tentative
    prolongator P[i][agg i] = 1/sqrt(|agg i|): returns (crow, ccol, cval,
    cdiag) with the off-diagonal part on the quotient graph (computed here
    unless given) and the coarse diagonal."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    if crow is None:
        crow, ccol = quotient(row_ptr, col, agg, n_agg)
    crow = np.ascontiguousarray(crow, dtype=np.int64)
    ccol = np.ascontiguousarray(ccol, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    cval = np.zeros(max(int(crow[-1]), 1), np.float64)
    cdiag = np.zeros(max(n_agg, 1), np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    if n_agg == 0:
        return crow, ccol, np.zeros(0), np.zeros(0)
    rc = _get().oracle_galerkin(n, _ptr(row_ptr, _i64p), _ptr(col if col.size else np.zeros(1, np.int32), _i32p),
                                _ptr(val if val.size else np.zeros(1), dp), _ptr(diag if diag.size else np.zeros(1), dp),
                                _ptr(agg if agg.size else np.zeros(1, np.int32), _i32p), n_agg,
                                _ptr(crow, _i64p), _ptr(ccol if ccol.size else np.zeros(1, np.int32), _i32p),
                                _ptr(cval, dp), _ptr(cdiag, dp))
    if rc != 0:
        raise OracleError("oracle_galerkin returned %d" % rc)
    return crow, ccol, cval[:int(crow[-1])].copy(), cdiag[:n_agg].copy()


def smoothed(row_ptr, col, val, diag, agg, n_agg, omega):
    """Smoothed aggregation with the damped-Jacobi prolongator
    P = (I - omega D^-1 A) P_tent (P_tent as in galerkin) and the coarse
    operator P^T A P (see oracle_smoothed for the order of operations).
    Returns (prow, pcol, pval, crow, ccol, cval): P as an n x n_agg CSR and
    the coarse operator as an n_agg x n_agg CSR, diagonal included, columns
    ascending."""
    row_ptr, col = _csr(row_ptr, col)
    n = row_ptr.size - 1
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    one_i32, one_f64 = np.zeros(1, np.int32), np.zeros(1)
    args = (n, _ptr(row_ptr, _i64p), _ptr(col if col.size else one_i32, _i32p),
            _ptr(val if val.size else one_f64, dp), _ptr(diag if diag.size else one_f64, dp),
            _ptr(agg if agg.size else one_i32, _i32p), n_agg, float(omega))
    pn, cn = ctypes.c_int64(0), ctypes.c_int64(0)
    lib = _get()
    rc = lib.oracle_smoothed(*args, None, None, None, 0, None, None, None, 0,
                             ctypes.byref(pn), ctypes.byref(cn))
    if rc != 0:
        raise OracleError("oracle_smoothed returned %d" % rc)
    prow, crow = np.zeros(n + 1, np.int64), np.zeros(n_agg + 1, np.int64)
    pcol, pval = np.zeros(max(pn.value, 1), np.int32), np.zeros(max(pn.value, 1))
    ccol, cval = np.zeros(max(cn.value, 1), np.int32), np.zeros(max(cn.value, 1))
    rc = lib.oracle_smoothed(*args, _ptr(prow, _i64p), _ptr(pcol, _i32p), _ptr(pval, dp),
                             pcol.size, _ptr(crow, _i64p), _ptr(ccol, _i32p), _ptr(cval, dp),
                             ccol.size, ctypes.byref(pn), ctypes.byref(cn))
    if rc != 0:
        raise OracleError("oracle_smoothed returned %d" % rc)
    return (prow, pcol[:pn.value].copy(), pval[:pn.value].copy(), crow,
            ccol[:cn.value].copy(), cval[:cn.value].copy())


def coarsen(row_ptr, col, seed=0, stop_below=1000, max_levels=64):
    """Multilevel coarsening: aggregate, then take the quotient graph, while
    the graph has at least stop_below vertices; stop early when a level does
    not shrink.  Reading: every level uses the same seed.  Returns a list of
    per-level dicts {n, nnz, agg, n_agg}; the coarse graph of level l is the
    input of level l + 1."""
    row_ptr, col = np.asarray(row_ptr, np.int64), np.asarray(col, np.int32)
    levels = []
    while row_ptr.size - 1 >= stop_below and len(levels) < max_levels:
        n = row_ptr.size - 1
        agg, n_agg = aggregate(row_ptr, col, seed)
        levels.append({"n": n, "nnz": int(row_ptr[-1]), "agg": agg, "n_agg": n_agg})
        if n_agg == n:
            break
        row_ptr, col = quotient(row_ptr, col, agg, n_agg)
    return levels
