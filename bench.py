"""Benchmark: deterministic MIS-2 + MIS-2 aggregation on one MI355X.

One step = one mis2_run and one mis2_aggregate call on the same device-resident
graph (default workload: 3D 27-point Laplacian graph on a 100^3 grid, 1M
vertices, 25.46M stored entries, int64 row offsets, int32 columns, seed 0).
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1|c2|c3|c4|c5]

c4 (batched multilevel coarsening of 512 subdomains, against a per-graph
loop) and c5 (serving with Poisson arrivals, p50/p99 latency) print their own
JSON line with the same keys.

value = graph nnz / step time (nnz/s).  roofline: the sweep kernel with the
largest share of GPU time, its algorithmic bytes per launch (exact, from an
untimed accounting run: 4 B per visited column index, 20 B (Refresh Column)
or 24 B (Decide Set) per worklist row, 4 B per row kept) over its mean launch
duration from HIP events recorded on the library's stream in a second timed
loop.  cpu_baseline: the CPU oracle on the host, one thread (median of 5
steps after a warm-up), with the host's CPU model and core counts and the
OpenMP build of the same oracle on every usable core beside it.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_2204_02934_amd import graphs
    if name == "c1":
        return "2D 5-point Laplacian graph 64x64 (n=4096), MIS-2 + MIS-2 aggregation", \
            graphs.grid2d_5pt(64, 64)
    if name == "c2":
        return "3D 27-point Laplacian graph 100^3 (n=1,000,000), MIS-2 + MIS-2 aggregation", \
            graphs.grid3d_27pt(100, 100, 100)
    if name == "c3":
        return "Chung-Lu power-law graph (n=4,000,000, mean degree 16, exponent 2.1, cap 20000), " \
               "MIS-2 + MIS-2 aggregation", graphs.chung_lu(4_000_000, 16.0, 2.1, 20000, seed=1)
    if name == "l100":
        return "3D 7-point Laplacian graph 100^3 (n=1,000,000; the paper's Laplace3D_100), " \
               "MIS-2 + MIS-2 aggregation", graphs.grid3d_7pt(100, 100, 100)
    raise SystemExit("unknown workload " + name)


# Fig. 2's ladder: each rung adds one optimization of Section V to the one
# before (flags of mis2_run_ablation that are still set = optimizations
# still taken away).
ABL_FIXED, ABL_XOR, ABL_NOWL, ABL_UNPACKED, ABL_ONE_LANE, ABL_SIMPLE = 1, 2, 4, 8, 16, 32
LADDER = [
    ("baseline (fixed priorities, every vertex every round, 3-field tuples, 1 lane)",
     ABL_FIXED | ABL_NOWL | ABL_UNPACKED | ABL_ONE_LANE),
    ("+ random priorities", ABL_NOWL | ABL_UNPACKED | ABL_ONE_LANE),
    ("+ worklists", ABL_UNPACKED | ABL_ONE_LANE),
    ("+ packed tuples (same simple kernels)", ABL_SIMPLE | ABL_ONE_LANE),
    ("production kernels, 1 lane per row", ABL_ONE_LANE),
    ("+ lanes per row by the degree rule (SIMD)", 0),
]


def run_ablation(args):
    """Fig. 2 and Table I on one graph: MIS-2 time per rung of the ladder
    (mis2_run_ablation, graph resident in HBM) with cumulative speedups, and
    the rounds taken with fixed, xorshift and xorshift* priorities."""
    import numpy as np
    import torch
    from paper_2204_02934_amd import api
    name, (rp_h, col_h) = workload(args.workload)
    name = name.split(", MIS-2")[0]
    n, nnz = rp_h.size - 1, int(rp_h[-1])
    dev = torch.device("cuda", 0)
    rp, col = api.as_device_csr(rp_h, col_h, dev)
    ctx = api.Context(0)
    rungs = []
    for label, flags in LADDER:
        for _ in range(args.warmup):
            ctx.mis2_ablation(rp, col, args.seed, flags, nnz=nnz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, nr, it = ctx.mis2_ablation(rp, col, args.seed, flags, nnz=nnz)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        rungs.append({"rung": label, "flags": flags, "ms": ms, "rounds": it, "mis2": nr})
        log("%-80s %8.3f ms  %2d rounds" % (label, ms, it))
    for r in rungs:
        r["speedup_vs_baseline"] = rungs[0]["ms"] / r["ms"]
    for a, b in zip(rungs, rungs[1:]):
        b["speedup_vs_previous"] = a["ms"] / b["ms"]
    rounds = {}
    for key, flags in (("fixed", ABL_FIXED), ("xor", ABL_XOR), ("xorstar", 0)):
        rounds[key] = ctx.mis2_ablation(rp, col, args.seed, flags, nnz=nnz)[2]
    return {
        "metric": "MIS-2 time per optimization rung (Fig. 2) and rounds per priority scheme "
                  "(Table I)",
        "value": rungs[0]["ms"] / rungs[-1]["ms"], "unit": "x (all four optimizations)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": rungs[-1]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": name, "n": n, "nnz": nnz, "seed": args.seed},
        "rungs": rungs, "table1_rounds": rounds,
    }


def galerkin_bytes(n, nnz, na, cnnz):
    """Bytes mis2_galerkin must move: the fine CSR, values, diagonal and labels
    once (8 + 4 + 8 + 8 + 4 B per row and entry as they apply), each entry's
    neighbour label (4 B), the member lists (4 + 8 B), the coarse rows (8 + 4 B)
    and the coarse values and diagonal written (8 B each)."""
    return (8 * n + 12 * nnz + 8 * n + 4 * n + 4 * nnz + 4 * n + 8 * na +
            8 * na + 4 * cnnz + 8 * cnnz + 8 * na)


def run_galerkin(args):
    """An aggregation multigrid hierarchy on the GPU: per level, Algorithm 3,
    the quotient graph and the Galerkin operator P^T A P (tentative
    prolongator), until fewer than 1000 rows remain."""
    import numpy as np
    import torch
    from paper_2204_02934_amd import api, graphs
    name, (rp_h, col_h) = workload(args.workload)
    name = name.split(", MIS-2")[0]
    dev = torch.device("cuda", 0)
    val_h, diag_h = graphs.matrix_values(rp_h, col_h, args.seed, shift=1.0)
    ctx = api.Context(0)

    def hierarchy():
        rp, col = api.as_device_csr(rp_h, col_h, dev)
        val, diag = torch.as_tensor(val_h, device=dev), torch.as_tensor(diag_h, device=dev)
        levels = []
        while rp.numel() - 1 >= 1000:
            n, nnz = rp.numel() - 1, int(rp[-1].item())
            t0 = time.perf_counter()
            agg, na = ctx.aggregate(rp, col, args.seed, nnz=nnz)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            crow, ccol = ctx.quotient(rp, col, agg, na, nnz=nnz)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            cval, cdiag = ctx.galerkin(rp, col, val, diag, agg, crow, ccol, nnz=nnz)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            levels.append({"n": n, "nnz": nnz, "n_agg": na, "coarse_nnz": int(ccol.numel()),
                           "aggregate_ms": 1e3 * (t1 - t0), "quotient_ms": 1e3 * (t2 - t1),
                           "galerkin_ms": 1e3 * (t3 - t2)})
            if na == n:
                break
            rp, col, val, diag = crow, ccol, cval, cdiag
        return levels

    for _ in range(max(args.warmup, 1)):
        hierarchy()
    runs = [hierarchy() for _ in range(args.steps)]
    best = min(runs, key=lambda lv: sum(l["aggregate_ms"] + l["quotient_ms"] + l["galerkin_ms"]
                                        for l in lv))
    total = [sum(l["aggregate_ms"] + l["quotient_ms"] + l["galerkin_ms"] for l in lv) for lv in runs]
    l0 = best[0]
    gb = galerkin_bytes(l0["n"], l0["nnz"], l0["n_agg"], l0["coarse_nnz"])
    # smoothed aggregation of level 0 (mis2_smoothed, omega = 2/3): wall time
    # of the call, which counts, sizes and fills P, A P and P^T A P
    rp, col = api.as_device_csr(rp_h, col_h, dev)
    val, diag = torch.as_tensor(val_h, device=dev), torch.as_tensor(diag_h, device=dev)
    nnz0 = int(rp_h[-1])
    agg, na = ctx.aggregate(rp, col, args.seed, nnz=nnz0)
    sm = []
    for k in range(max(args.warmup, 1) + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (prow, pcol, pval), (crow, ccol, cval) = ctx.smoothed(rp, col, val, diag, agg, na,
                                                              2.0 / 3.0, nnz=nnz0)
        torch.cuda.synchronize()
        if k >= max(args.warmup, 1):
            sm.append(1e3 * (time.perf_counter() - t0))
    p_nnz, c_nnz = int(pcol.numel()), int(ccol.numel())
    n0 = int(rp_h.size - 1)
    # compulsory traffic: A (col, val, row offsets, diagonal) and the labels
    # read once, P and A_c written once (the intermediate A P not counted)
    sb = 12 * nnz0 + 8 * (n0 + 1) + 8 * n0 + 4 * n0 + 12 * p_nnz + 8 * (n0 + 1) + \
        12 * c_nnz + 8 * (na + 1)
    sm_ms = float(np.median(sm))
    log("smoothed aggregation, level 0: %.3f ms (P %d entries, P^T A P %d entries)"
        % (sm_ms, p_nnz, c_nnz))
    for i, l in enumerate(best):
        log("level %d: n %d nnz %d -> %d aggregates, %d coarse entries; aggregate %.3f ms, "
            "quotient %.3f ms, Galerkin %.3f ms" % (i, l["n"], l["nnz"], l["n_agg"], l["coarse_nnz"],
                                                   l["aggregate_ms"], l["quotient_ms"], l["galerkin_ms"]))
    return {
        "metric": "aggregation multigrid setup: levels of Algorithm 3 + quotient + Galerkin P^T A P",
        "value": float(np.median(total)), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": float(np.median(total)),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "n": int(rp_h.size - 1), "nnz": int(rp_h[-1]), "seed": args.seed,
                   "levels": len(best), "stop_below": 1000,
                   "matrix": "symmetric M-matrix, off-diagonals -U[0.5,1.5), diagonal = row sum + 1"},
        "levels": best,
        "galerkin_level0": {"ms_wall": l0["galerkin_ms"], "bytes": gb,
                            "achieved_gbps_wall": gb / (l0["galerkin_ms"] * 1e-3) / 1e9,
                            "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                            "note": "wall time of the call: a range check, a counting sort of the "
                                    "members, the operator kernel and two read-backs"},
        "smoothed_level0": {"omega": 2.0 / 3.0, "ms_wall": sm_ms, "p_nnz": p_nnz,
                            "coarse_nnz": c_nnz, "bytes_compulsory": sb,
                            "achieved_gbps_wall": sb / (sm_ms * 1e-3) / 1e9,
                            "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                            "note": "median wall time of mis2_smoothed (structure and values of "
                                    "P, A P and P^T A P, with read-backs of the counts)"},
    }


def cgs_sweep_bytes(n, nnz, point):
    """Bytes one symmetric sweep (forward, then backward) must move: per
    direction the off-diagonal entries once (col 4 B + val 8 B), and per row
    its sweep-order index (4 B), CSR extent (8 B), b, diagonal, old x and new
    x (8 B each).  The upper figure also counts every x gather (8 B per
    entry) and, for clusters, every neighbour's sweep position (4 B)."""
    per_dir = 12 * nnz + (4 + 8 + 8 + 8 + 8 + 8) * n
    upper = per_dir + 8 * nnz + (0 if point else 4 * nnz)
    return 2 * per_dir, 2 * upper


def run_cgs(args):
    """Algorithm 4 on one graph: setup time (coarsening, colouring, ordering)
    and symmetric sweep time for cluster and point multicolor Gauss-Seidel,
    and the symmetric sweeps each needs, as a stationary iteration, to bring
    ||b - A x|| / ||b|| below 1e-8 (the paper measures GMRES iterations with
    these sweeps as preconditioner; GMRES is not part of this library)."""
    import numpy as np
    import torch
    from paper_2204_02934_amd import api, graphs
    name, (rp_h, col_h) = workload(args.workload)
    name = name.split(", MIS-2")[0]
    n, nnz = rp_h.size - 1, int(rp_h[-1])
    dev = torch.device("cuda", 0)
    rp, col = api.as_device_csr(rp_h, col_h, dev)
    val_h, diag_h = graphs.matrix_values(rp_h, col_h, args.seed, shift=1.0)
    val = torch.as_tensor(val_h, device=dev)
    diag = torch.as_tensor(diag_h, device=dev)
    b = torch.as_tensor(np.random.default_rng(args.seed).standard_normal(n), device=dev)
    # the residual check (outside the timed regions) as a sparse product
    A = torch.sparse_csr_tensor(rp, col[:nnz].long(), val, size=(n, n))

    def rel_residual(x):
        ax = diag * x + torch.mv(A, x)
        return float(torch.linalg.norm(b - ax) / torch.linalg.norm(b))

    ctx = api.Context(0)
    out = {}
    for kind, point in (("cluster", False), ("point", True)):
        ctx.cgs_setup(rp, col, args.seed, point=point, nnz=nnz)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            plan = ctx.cgs_setup(rp, col, args.seed, point=point, nnz=nnz)
        torch.cuda.synchronize()
        setup_ms = 1e3 * (time.perf_counter() - t0) / reps
        x = torch.zeros(n, dtype=torch.float64, device=dev)
        ctx.cgs_apply(rp, col, val, diag, plan, b, x, sweeps=2, symmetric=True, nnz=nnz)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.cgs_apply(rp, col, val, diag, plan, b, x, sweeps=args.steps, symmetric=True, nnz=nnz)
        torch.cuda.synchronize()
        sweep_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        x.zero_()
        sweeps, res = 0, 1.0
        while res > 1e-8 and sweeps < 4000:
            ctx.cgs_apply(rp, col, val, diag, plan, b, x, sweeps=10, symmetric=True, nnz=nnz)
            sweeps += 10
            res = rel_residual(x)
            if sweeps % 200 == 0:
                log("%s: %d sweeps, residual %.3e" % (kind, sweeps, res))
        sweep_bytes, upper = cgs_sweep_bytes(n, nnz, point)
        out[kind] = {"setup_ms": setup_ms, "sgs_sweep_ms": sweep_ms, "clusters": plan.n_clusters,
                     "colors": plan.n_colors, "sweeps_to_1e-8": sweeps, "final_residual": res,
                     "roofline": {"bound": "hbm", "achieved": sweep_bytes / (sweep_ms * 1e-3) / 1e9,
                                  "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                  "frac": sweep_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                  "bytes_per_sgs_sweep": sweep_bytes,
                                  "bytes_per_sgs_sweep_upper": upper,
                                  "achieved_upper": upper / (sweep_ms * 1e-3) / 1e9}}
        log("%s: setup %.3f ms, %d clusters, %d colours, SGS sweep %.3f ms, %d sweeps to 1e-8"
            % (kind, setup_ms, plan.n_clusters, plan.n_colors, sweep_ms, sweeps))
    c, p = out["cluster"], out["point"]
    return {
        "metric": "cluster multicolor SGS: time to 1e-8 relative residual (Algorithm 4)",
        "value": c["setup_ms"] + c["sgs_sweep_ms"] * c["sweeps_to_1e-8"], "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": 2, "ms_per_step": c["sgs_sweep_ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": name, "n": n, "nnz": nnz, "seed": args.seed,
                   "matrix": "symmetric M-matrix, off-diagonals -U[0.5,1.5), diagonal = row sum + 1"},
        "cluster": c, "point": p,
        "point_time_to_1e-8_ms": p["setup_ms"] + p["sgs_sweep_ms"] * p["sweeps_to_1e-8"],
    }


def kernel_sources_digest():
    """SHA-256 over the sources the MIS-2 sweeps and their launch plan are
    built from (the kernels, their header and the host round loop), so a
    stored hardware-counter measurement is used only for the code it measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2204_02934_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("abi.hip", "internal.h", "lanes.h", "mis2_kernels.hip")]
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, kernel, launches_per_step, plan):
    """HBM bytes per launch of `kernel` from profiles/traffic_<workload>.json
    (rocprofv3 FETCH_SIZE and WRITE_SIZE runs of this bench, one pair per
    explicit launch plan, scaled by the same counters on a plain device copy
    of known size; bytes per step over the launches per step counted here),
    or None when there is no such measurement for the current sources and
    the plan this run used."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("sources_sha256") != kernel_sources_digest():
        return None
    for m in t.get("measurements", []):
        tp = m.get("plan", {})
        if (tp.get("lanes"), tp.get("tail")) != (plan.get("lanes"), plan.get("tail")):
            continue
        k = m.get("kernels", {}).get(kernel)
        if k is None or "hbm_bytes_per_step" not in k:
            return None
        return k["hbm_bytes_per_step"] / launches_per_step
    return None


def sweep_bytes(rec, identity, written=0):
    """Algorithmic bytes of one sweep launch: column indices of the visited
    rows, per-row terms (row extents 8, worklist entry 4 unless the list is
    the identity, own value 4, written value 4, plus the compulsory first
    touch of the gathered value 4 (Refresh Column) or read of M_v and T_v
    (Decide Set)), and the compacted worklist written.  A Refresh Column
    that rewrites long rows without their OUT neighbours also writes those
    `written` column indices (and a length per rewritten row, not counted:
    at most one per 32 indices), and one that reads such rows reads a length
    per row as well."""
    per_row = 20 if rec["kind"] == 0 else 24
    if identity:
        per_row -= 4
    b = 4 * rec["edges"] + per_row * rec["rows"] + 4 * rec["rows_out"]
    if rec["kind"] == 0:
        b += 4 * written
        if rec.get("compact", 0) == 2:
            b += 4 * rec["rows"]
    return b


def compaction_writes(recs):
    """Column indices each compacting Refresh Column wrote into compacted
    rows (counted by the accounting pass)."""
    return [max(r.get("written", 0), 0) if r["kind"] == 0 else 0 for r in recs]


KERNELS = {0: "refresh_column", 1: "decide", 2: "mis2_rounds_persistent", 3: "mis2_tail",
           4: "refresh_column", 5: "decide"}


def sweep_table(recs):
    """Algorithmic bytes of every sweep of one call's accounting run, and the
    upper-bound gather bytes: {(phase, kind, round): (bytes, gather bytes)}."""
    out = {}
    for r in recs:
        if r["kind"] in (0, 1):
            w = max(r.get("written", 0), 0) if r["kind"] == 0 else 0
            out[(r["phase"], r["kind"], r["round"])] = (
                sweep_bytes(r, r["phase"] == 0 and r["round"] == 0, w), gather_bytes(r))
    return out


def launch_costs(table, recs):
    """(kernel, bytes, upper bytes, ms) of every launch of one profiled call:
    a launched sweep is priced with its round's bytes, a persistent launch
    (kind 2) with every sweep of its phase, the one-workgroup tail (kind 3)
    with the sweeps of its phase from its first round on, and a round issued
    after the end of the run (kinds 4, 5) with none."""
    whole = {r["phase"] for r in recs if r["kind"] == 2}
    tail = {r["phase"]: r["round"] for r in recs if r["kind"] == 3}
    out = []
    for r in recs:
        k, ph = r["kind"], r["phase"]
        if k in (0, 1):
            if ph in whole or (ph in tail and r["round"] >= tail[ph]):
                continue  # ran inside a persistent or tail launch
            b, g = table.get((ph, k, r["round"]), (0, 0))
            out.append((KERNELS[k], b, g, r["ms"]))
        elif k in (2, 3):
            first = 0 if k == 2 else r["round"]
            sw = [v for (p, _, rd), v in table.items() if p == ph and rd >= first]
            out.append((KERNELS[k], sum(v[0] for v in sw), sum(v[1] for v in sw), r["ms"]))
        elif k in (4, 5):
            out.append((KERNELS[k], 0, 0, r["ms"]))
    return out


def gather_bytes(rec):
    """Bytes one sweep would add if every neighbour-value gather went to HBM
    (4 per visited edge) instead of the compulsory first touch counted in
    sweep_bytes: the upper-bound variant of the algorithmic model."""
    return 4 * rec["edges"] if rec["kind"] in (0, 1) else 0


def host_cpu():
    """The host's CPU model, sockets, physical cores and logical CPUs (from
    /proc/cpuinfo) and the CPUs this process may run on."""
    model, sockets, cores, logical = None, set(), set(), 0
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                    sockets.add(v)
                elif k == "core id":
                    core = v
                    cores.add((phys, core))
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "sockets": len(sockets) or None,
            "physical_cores": len(cores) or None, "logical_cpus": logical or os.cpu_count(),
            "usable_cpus": usable}


def cpu_baseline(rp_h, col_h, seed, agg_call, nnz, agg_name, reps=5):
    """The oracle (oracle/oracle.c as it stands) timed on the host: one
    warm-up, then the median of `reps` full steps (MIS-2 + aggregation of the
    same graph), single-threaded; and the OpenMP build of the same source
    (its pure-map phase loops on every usable host CPU, OMP_NUM_THREADS when
    set) timed the same way."""
    import numpy as np
    import oracle

    def timed():
        ts = []
        for i in range(reps + 1):
            t0 = time.perf_counter()
            oracle.mis2(rp_h, col_h, seed)
            getattr(oracle, agg_call)(rp_h, col_h, seed)
            if i:
                ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    host = host_cpu()
    t1 = timed()
    log("cpu oracle, 1 thread: %.3f s/step" % t1)
    out = {"value": nnz / t1, "unit": "nnz/s", "cores": 1, "kind": "oracle",
           "sample": "median of %d full steps (MIS-2 + %s) of the same graph after 1 warm-up, "
                     "%.3f s each, one thread" % (reps, agg_name, t1),
           "host": host}
    threads = int(os.environ.get("OMP_NUM_THREADS") or host["usable_cpus"] or 1)
    try:
        path = oracle.build_oracle(force=False, parallel=True)
        os.environ["OMP_NUM_THREADS"] = str(threads)
        with oracle.use_library(path):
            tn = timed()
        out["all_cores"] = {"value": nnz / tn, "unit": "nnz/s", "cores": threads,
                            "s_per_step": tn,
                            "build": "oracle.c with -DORACLE_OMP -fopenmp (Algorithm 1's "
                                     "three phase loops in parallel; identical results)"}
        log("cpu oracle, %d threads: %.3f s/step" % (threads, tn))
    except Exception as e:  # no OpenMP toolchain: the single-thread figure stands alone
        out["all_cores"] = {"error": str(e)}
    return out


def c5_pool(count, seed=3, n_lo=1_000, n_hi=10_000_000):
    """Serving jobs (graphs.serving_pool): n log-uniform on [n_lo, n_hi];
    40% 2D 5-point, 40% 3D 27-point, 20% Chung-Lu."""
    from paper_2204_02934_amd import graphs
    return graphs.serving_pool(count, seed, n_lo, n_hi)


def run_c4(args):
    """Batched multilevel coarsening of 512 dropped-edge 7-point subdomains
    (mis2_aggregate_batched, one call) against the same library called per
    graph on one stream (mis2_coarsen in a loop)."""
    import numpy as np
    import torch
    from paper_2204_02934_amd import api, graphs
    gs = graphs.batch_subdomains(num=512, lo=8, hi=48, p_drop=0.1, seed=2)
    rp_h, col_h = graphs.disjoint_union(gs)
    voff = np.cumsum([0] + [g[0].size - 1 for g in gs]).astype(np.int64)
    n, nnz = rp_h.size - 1, int(rp_h[-1])
    log("c4: %d graphs, union n=%d nnz=%d" % (len(gs), n, nnz))
    dev = torch.device("cuda", 0)
    rp, col = api.as_device_csr(rp_h, col_h, dev)
    per = [api.as_device_csr(a, b, dev) for a, b in gs]
    per_nnz = [int(a[-1]) for a, _ in gs]
    ctx = api.Context(0)
    for _ in range(args.warmup):
        ctx.aggregate_batched(rp, col, voff, seed=args.seed, stop_below=1000, nnz=nnz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.aggregate_batched(rp, col, voff, seed=args.seed, stop_below=1000, nnz=nnz)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    # per-graph loop (one pass after one warm pass)
    for (a, b), z in zip(per, per_nnz):
        ctx.coarsen(a, b, seed=args.seed, stop_below=1000, nnz=z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (a, b), z in zip(per, per_nnz):
        ctx.coarsen(a, b, seed=args.seed, stop_below=1000, nnz=z)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    rule = api.Context(0, autotune=False)
    for _ in range(args.warmup):
        rule.aggregate_batched(rp, col, voff, seed=args.seed, stop_below=1000, nnz=nnz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rule.aggregate_batched(rp, col, voff, seed=args.seed, stop_below=1000, nnz=nnz)
    torch.cuda.synchronize()
    t_rule = (time.perf_counter() - t0) / args.steps
    log("c4: batched %.2f ms (degree rule %.2f ms), per-graph loop %.2f ms"
        % (1e3 * t_batch, 1e3 * t_rule, 1e3 * t_loop))
    return {
        "metric": "MIS-2+aggregation graph nnz/s and HBM GB/s fraction",
        "value": nnz / t_batch, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_batch, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "512 dropped-edge (p=0.1) 3D 7-point subdomains, side U{8..48}, "
                               "multilevel MIS-2 aggregation to < 1000 vertices, batched",
                   "n": n, "nnz": nnz, "graphs": len(gs), "seed": args.seed},
        "per_graph_loop_ms": 1e3 * t_loop,
        "per_graph_loop_nnz_per_s": nnz / t_loop,
        "batched_speedup": t_loop / t_batch,
        "degree_rule_ms": 1e3 * t_rule,
        "plan_last_level": ctx.last_plan(),
    }


def run_c5(args):
    """Serving: a seeded stream of coarsening jobs (each one of a pool of
    distinct graphs of the serving mix) through a mis2_server.  Saturation:
    the whole stream queued at once, graphs already in HBM (the value); the
    same with jobs handed over as host CSRs, copied to the GPU on a side
    stream while the running level computes (PCIe-inclusive); then Poisson
    arrivals at 0.5x and 0.8x of the saturation rate, graphs in HBM.  Latency
    = completion - arrival (host monotonic clock).  Beside it, the same jobs
    through mis2_coarsen one at a time on one stream (graphs in HBM): the
    plain per-graph launch."""
    import numpy as np
    import torch
    from paper_2204_02934_amd import api
    pool = c5_pool(args.c5_graphs)
    rng = np.random.default_rng(4)
    pick = rng.integers(0, len(pool), args.c5_jobs)
    dev = torch.device("cuda", 0)
    host = [(a, b, a.size - 1, int(a[-1])) for _, (a, b) in pool]
    dev_graphs = [api.as_device_csr(a, b, dev) for _, (a, b) in pool]
    jobs = [host[i] for i in pick]
    tot_nnz = sum(j[3] for j in jobs)
    vmax = max(j[2] for j in host)
    emax = max(j[3] for j in host)
    srv = api.Server(max_vertices=max(4 * vmax, 1 << 20), max_nnz=max(4 * emax, 1 << 22),
                     max_graphs=256, seed=args.seed, stop_below=1000)
    log("c5: %d jobs over %d distinct graphs, sum nnz %d, largest n %d"
        % (len(jobs), len(pool), tot_nnz, vmax))

    def run(rate, rng, upload=False):
        n_jobs = len(jobs)
        arrive = np.zeros(n_jobs) if rate is None else np.cumsum(rng.exponential(1.0 / rate,
                                                                                 n_jobs))
        done_at = {}
        t0 = time.perf_counter()
        nxt = 0
        while len(done_at) < n_jobs:
            now = time.perf_counter() - t0
            while nxt < n_jobs and arrive[nxt] <= now:
                i = pick[nxt]
                if upload:  # host CSR, copied in on the server's side stream
                    srv.submit(host[i][0], host[i][1], tag=nxt, nnz=host[i][3])
                else:       # already in HBM
                    srv.submit(dev_graphs[i][0], dev_graphs[i][1], tag=nxt, nnz=host[i][3])
                nxt += 1
            pending = srv.step()
            for r in srv.poll():
                done_at[r["tag"]] = time.perf_counter() - t0
            if pending == 0 and nxt < n_jobs:
                time.sleep(max(0.0, min(arrive[nxt] - (time.perf_counter() - t0), 0.05)))
        wall = time.perf_counter() - t0
        lat = np.array([done_at[i] - arrive[i] for i in range(n_jobs)])
        return wall, lat

    run(None, None)  # warm-up
    wall_sat, lat_sat = run(None, None)
    sat = len(jobs) / wall_sat
    log("c5: saturation %.2f jobs/s (%.3f s for the stream)" % (sat, wall_sat))
    # the same stream handed over as host CSRs: PCIe-inclusive
    wall_up, lat_up = run(None, None, upload=True)
    log("c5: saturation with host uploads %.2f jobs/s (%.3f s)" % (len(jobs) / wall_up, wall_up))
    res = {}
    for frac in (0.5, 0.8):
        wall, lat = run(frac * sat, np.random.default_rng(3))
        res["%.1fx" % frac] = {"qps": frac * sat, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                               "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                               "max_ms": 1e3 * float(lat.max()),
                               "nnz_per_s": tot_nnz / wall, "wall_s": wall}
        log("c5 %.1fx: %s" % (frac, json.dumps(res["%.1fx" % frac])))
    srv.close()
    # the plain per-graph launch: mis2_coarsen per job, one stream, graphs on the GPU
    ctx = api.Context(0)
    for i in sorted(set(pick.tolist())):  # warm pass over the distinct graphs
        ctx.coarsen(*dev_graphs[i], seed=args.seed, stop_below=1000, nnz=host[i][3])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in pick:
        ctx.coarsen(*dev_graphs[i], seed=args.seed, stop_below=1000, nnz=host[i][3])
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    log("c5: per-graph loop %.3f s (%.3g nnz/s)" % (t_loop, tot_nnz / t_loop))
    return {
        "metric": "MIS-2+aggregation graph nnz/s and HBM GB/s fraction",
        "value": tot_nnz / wall_sat, "unit": "nnz/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": 1e3 * wall_sat, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serving: %d multilevel coarsening jobs over %d distinct graphs, "
                               "n log-uniform [1e3, 1e7], 2D 5-pt / 3D 27-pt / Chung-Lu "
                               "40/40/20, whole stream queued, graphs in HBM"
                               % (len(jobs), len(pool)),
                   "jobs": len(jobs), "distinct_graphs": len(pool), "sum_nnz": tot_nnz,
                   "seed": args.seed},
        "saturation_jobs_per_s": sat,
        "saturation_p50_ms": 1e3 * float(np.percentile(lat_sat, 50)),
        "saturation_p99_ms": 1e3 * float(np.percentile(lat_sat, 99)),
        "host_upload": {"nnz_per_s": tot_nnz / wall_up, "jobs_per_s": len(jobs) / wall_up,
                        "p99_ms": 1e3 * float(np.percentile(lat_up, 99)),
                        "note": "jobs handed over as host CSRs (pageable), PCIe-inclusive"},
        "poisson": res,
        "per_graph_loop_s": t_loop,
        "per_graph_nnz_per_s": tot_nnz / t_loop,
        "served_vs_per_graph": t_loop / wall_sat,
    }


def run_launch_cost(args):
    """Dispatch cost of a small kernel on this GPU: back-to-back direct launches
    against the same launches replayed from a captured HIP graph (torch's
    graph capture), GPU time per launch from events, host time per direct
    launch from the host clock.  Sets the price of the host-driven round loop's
    launches against what graph replay would save."""
    import torch
    dev = torch.device("cuda", 0)
    x = torch.zeros(256, device=dev)
    n = 400
    for _ in range(50):
        x.add_(1.0)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    direct, host = [], []
    for _ in range(5):
        e0.record()
        t0 = time.perf_counter()
        for _ in range(n):
            x.add_(1.0)
        host.append((time.perf_counter() - t0) / n)
        e1.record()
        torch.cuda.synchronize()
        direct.append(e0.elapsed_time(e1) / n)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            x.add_(1.0)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(n):
            x.add_(1.0)
    before = float(x[0].item())
    graph = []
    for _ in range(5):
        e0.record()
        g.replay()
        e1.record()
        torch.cuda.synchronize()
        graph.append(e0.elapsed_time(e1) / n)
    after = float(x[0].item())
    assert after == before + 5 * n, (before, after)  # every replayed launch ran
    return {"metric": "small-kernel dispatch cost", "unit": "us per launch",
            "kernel": "add_ on 256 floats", "launches": n,
            "direct_gpu_us": 1e3 * min(direct), "graph_gpu_us": 1e3 * min(graph),
            "direct_host_us": 1e6 * min(host), "reps": 5}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run three device-to-device copies of MIB MiB (a known-size "
                         "kernel for scaling hardware byte counters)")
    ap.add_argument("--c5-jobs", type=int, default=200, help="serving: jobs in the stream")
    ap.add_argument("--c5-graphs", type=int, default=48,
                    help="serving: distinct graphs the jobs are drawn from")
    ap.add_argument("--ablation", action="store_true",
                    help="c1-c3, l100: the optimization ladder of Fig. 2 and the rounds of "
                         "Table I instead of the step")
    ap.add_argument("--galerkin", action="store_true",
                    help="an aggregation multigrid hierarchy (Algorithm 3, quotient graph, "
                         "Galerkin P^T A P per level) instead of the step")
    ap.add_argument("--cgs", action="store_true",
                    help="c1, c2, l100: cluster vs point multicolor Gauss-Seidel (Algorithm 4) "
                         "instead of the step")
    ap.add_argument("--launch-cost", action="store_true",
                    help="dispatch cost of a small kernel, direct against HIP graph replay, "
                         "instead of the step")
    ap.add_argument("--lanes", type=int, default=None,
                    help="c1-c3: lanes per row of the sweeps (-2 = staged, -1 = flat) instead "
                         "of the tuned plan")
    ap.add_argument("--tail", type=int, default=None, choices=(0, 1),
                    help="c1-c3: the one-workgroup tail off (0) or on (1) instead of the tuned "
                         "choice")
    ap.add_argument("--aggregation", choices=("alg3", "alg2"), default="alg3",
                    help="c1-c3: the aggregation of the step, MIS-2 based aggregation "
                         "(mis2_aggregate) or basic MIS-2 coarsening (mis2_aggregate_basic)")
    args = ap.parse_args()
    if args.gpus != 1:
        raise SystemExit("bench.py measures one GPU: the library has no multi-GPU path "
                         "(--gpus %d requested)" % args.gpus)
    if args.launch_cost:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps(run_launch_cost(args)), flush=True)
        return
    if args.galerkin:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps(run_galerkin(args)), flush=True)
        return
    if args.cgs:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps(run_cgs(args)), flush=True)
        return
    if args.ablation:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps(run_ablation(args)), flush=True)
        return
    if args.workload in ("c4", "c5"):
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        out = run_c4(args) if args.workload == "c4" else run_c5(args)
        print(json.dumps(out), flush=True)
        return

    import numpy as np
    import torch

    from paper_2204_02934_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    agg_call = "aggregate" if args.aggregation == "alg3" else "aggregate_basic"
    # an explicit launch plan (the tuner then stays out: profiler runs count
    # the same kernels in every step)
    plan_kw = {}
    if args.lanes is not None:
        plan_kw["lanes"] = args.lanes
    if args.tail is not None:
        plan_kw["tail"] = args.tail
    name, (rp_h, col_h) = workload(args.workload)
    if args.aggregation == "alg2":
        name = name.replace("MIS-2 + MIS-2 aggregation", "MIS-2 + basic MIS-2 coarsening")
    n, nnz = rp_h.size - 1, int(rp_h[-1])
    log("workload:", name, "n=%d nnz=%d" % (n, nnz))
    dev = torch.device("cuda", 0)
    rp, col = api.as_device_csr(rp_h, col_h, dev)

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copies: 3 x %d MiB" % args.calibrate_copy)

    ctx = api.Context(0, **plan_kw)
    ctx.ensure_workspace(n, 1, nnz)
    torch.cuda.synchronize()

    def step(c):
        c.mis2(rp, col, args.seed, nnz=nnz)
        getattr(c, agg_call)(rp, col, args.seed, nnz=nnz)

    for _ in range(args.warmup):
        step(ctx)
    torch.cuda.synchronize()
    log("warmup done")

    # value: plain timed loop
    t_mis = []
    t_agg = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        ctx.mis2(rp, col, args.seed, nnz=nnz)
        b = time.perf_counter()
        getattr(ctx, agg_call)(rp, col, args.seed, nnz=nnz)
        c = time.perf_counter()
        t_mis.append(b - a)
        t_agg.append(c - b)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    log("timed: %.3f ms/step (mis2 %.3f ms, aggregate %.3f ms)"
        % (ms_per_step, 1e3 * np.median(t_mis), 1e3 * np.median(t_agg)))

    # algorithmic bytes per launch (untimed accounting run; results are
    # deterministic, so every timed step visits the same rows)
    acc = api.Context(0, account=True, **plan_kw)
    acc.ensure_workspace(n, 1, nnz)
    acc.mis2(rp, col, args.seed, nnz=nnz)
    recs_mis = acc.last_sweeps()
    getattr(acc, agg_call)(rp, col, args.seed, nnz=nnz)
    recs_agg = acc.last_sweeps()
    accounted = recs_mis + recs_agg

    # launch durations: a second timed loop with HIP events around each
    # launch; each launch is priced with the accounting run's bytes of the
    # sweeps it ran (the round where the one-workgroup tail takes over may
    # differ from run to run, the bytes of a round do not)
    prof = api.Context(0, profile=True, **plan_kw)
    prof.ensure_workspace(n, 1, nnz)
    step(prof)
    torch.cuda.synchronize()
    tables = [sweep_table(recs_mis), sweep_table(recs_agg)]
    per_kind = {}
    tp0 = time.perf_counter()
    for _ in range(args.steps):
        prof.mis2(rp, col, args.seed, nnz=nnz)
        r1 = prof.last_sweeps()
        getattr(prof, agg_call)(rp, col, args.seed, nnz=nnz)
        r2 = prof.last_sweeps()
        for table, recs in zip(tables, (r1, r2)):
            for k, b, g, ms in launch_costs(table, recs):
                e = per_kind.setdefault(k, {"bytes": 0, "bytes_upper": 0, "ms": 0.0,
                                            "launches": 0})
                e["bytes"] += b
                e["bytes_upper"] += b + g
                e["ms"] += ms
                e["launches"] += 1
    torch.cuda.synchronize()
    ms_profiled = 1e3 * (time.perf_counter() - tp0) / args.steps
    for e in per_kind.values():  # per step
        for key in ("bytes", "bytes_upper", "ms", "launches"):
            e[key] /= args.steps
    dom = max(per_kind, key=lambda k: per_kind[k]["ms"])
    d = per_kind[dom]
    # GB/s = the kernel's bytes per step / its GPU time per step (every launch
    # of it, rounds issued after the end of a run included)
    achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
    sweep_ms = sum(v["ms"] for v in per_kind.values())
    sweep_bytes_total = sum(v["bytes"] for v in per_kind.values())
    log("per kind:", json.dumps(per_kind))

    # the plan the tuner chose for this graph, and the step with the fixed
    # degree rule (tuner off) for comparison
    plan = ctx.last_plan()
    tuning = ctx.last_tuning()
    rule_ms, rule_plan = None, {"lanes": None, "blocks": None}
    if not plan_kw:
        rule = api.Context(0, autotune=False)
        rule.ensure_workspace(n, 1, nnz)
        for _ in range(args.warmup):
            step(rule)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(rule)
        torch.cuda.synchronize()
        rule_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        rule_plan = rule.last_plan()
        log("plan %s (rule %s): %.3f ms/step with the tuned plan, %.3f ms with the rule"
            % (plan, rule_plan, ms_per_step, rule_ms))

    rounds_mis = 1 + max(r["round"] for r in recs_mis if r["kind"] in (0, 1)) if recs_mis else 0

    # device-copy ceiling on this machine: 256 MiB device-to-device copies
    cb = 256 << 20
    src = torch.ones(cb, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * cb * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9  # bytes read + written
    del src, dst
    log("device copy ceiling: %.0f GB/s" % copy_gbps)

    # CPU baseline: the oracle on the host, median of 5 full steps after 1
    # warm-up, single-threaded; beside it the OpenMP build of the same source
    # on every usable host core
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(rp_h, col_h, args.seed, agg_call, nnz,
                           "aggregation" if args.aggregation == "alg3" else "basic coarsening")

    out = {
        "metric": "MIS-2+aggregation graph nnz/s and HBM GB/s fraction",
        "value": nnz / (ms_per_step * 1e-3),
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": name, "n": n, "nnz": nnz, "seed": args.seed,
                   "step": "mis2_run + %s, graph resident in HBM" % (
                       "mis2_aggregate" if args.aggregation == "alg3" else "mis2_aggregate_basic"),
                   "index_types": "int64 row offsets, int32 columns"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": measured_traffic(args.workload + ("" if args.aggregation == "alg3"
                                                                  else "_alg2"), dom, d["launches"],
                                                 plan),
                     "copy_ceiling": copy_gbps, "frac_of_copy_ceiling": achieved / copy_gbps,
                     "kernel": dom, "launches_per_step": d["launches"],
                     "bytes_per_launch": d["bytes"] / d["launches"],
                     "bytes_per_launch_upper": d["bytes_upper"] / d["launches"],
                     "achieved_upper": d["bytes_upper"] / (d["ms"] * 1e-3) / 1e9,
                     "mean_launch_ms": d["ms"] / d["launches"]},
        "cpu_baseline": cpu,
        "mis2_ms": 1e3 * float(np.median(t_mis)),
        "aggregate_ms": 1e3 * float(np.median(t_agg)),
        "mis2_rounds": rounds_mis,
        "round_kernels_gpu_ms_per_step": sweep_ms,
        "round_kernels_bytes_per_step": sweep_bytes_total,
        "round_kernels_gbps": sweep_bytes_total / (sweep_ms * 1e-3) / 1e9,
        "step_algorithmic_gbps": sweep_bytes_total / (ms_per_step * 1e-3) / 1e9,
        "step_algorithmic_frac": sweep_bytes_total / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "kernels_per_step": {k: {"launches": v["launches"], "ms": v["ms"], "bytes": v["bytes"]}
                             for k, v in per_kind.items()},
        "plan": {"lanes": plan["lanes"], "blocks": plan["blocks"],
                 "tail": plan["tail"],
                 "source": ["rule or options", "tuned (cached)", "tuned"][plan["source"]],
                 "tuning": tuning, "rule_plan": {"lanes": rule_plan["lanes"],
                                                 "blocks": rule_plan["blocks"]},
                 "rule_ms_per_step": rule_ms},
        "ms_per_step_profiled": ms_profiled,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
