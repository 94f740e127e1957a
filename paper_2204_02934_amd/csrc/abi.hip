// abi.hip -- the C ABI declared in include/mis2.h: contexts, workspace, and the
// host side of Algorithm 1 (MIS-2) and Algorithm 3 (aggregation).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <mutex>

#include "internal.h"

using namespace mis2;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int fail(mis2_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(mis2_ctx *ctx, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), MIS2_EHIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_),   \
                        __FILE__, __LINE__);                                                \
    } while (0)

// Tuple parameters of a round, carrying the graphs of a batched run.
TupleParams tparams(const mis2_ctx *ctx, int64_t n, uint64_t seed, uint64_t iter) {
    TupleParams p = tuple_params(n, seed, iter);
    p.batch = ctx->batch;
    return p;
}

int check_graph_args(mis2_ctx *ctx, const mis2_graph *g) {
    if (!ctx) return MIS2_EINVAL;
    if (!g) return fail(ctx, MIS2_EINVAL, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return fail(ctx, MIS2_EINVAL, "negative graph size");
    if (g->n > (int64_t)0x7FFFFFFE)
        return fail(ctx, MIS2_EINVAL, "n = %lld exceeds 2^31 - 2", (long long)g->n);
    if (g->n > 0 && !g->row_ptr) return fail(ctx, MIS2_EINVAL, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col) return fail(ctx, MIS2_EINVAL, "col is NULL");
    return MIS2_OK;
}

// Lanes per row of the MIS-2 sweeps; 0 selects the flat (merge-path) sweeps.
int lanes_for(const mis2_ctx *ctx, const mis2_graph *g) {
    if (ctx->plan.lanes == -1) return 0;
    // the staged sweeps' 16-byte column loads need at least 4 entries
    if (ctx->plan.lanes == kStagedLanes) return g->nnz >= 4 ? kStagedLanes : 1;
    if (ctx->plan.lanes) return ctx->plan.lanes;
    // Section V-D: one thread per row below an average degree of 16, lanes
    // cooperating on a row above it; here the group grows with the degree.
    // Measured on gfx950 (MIS-2 time, 1 / 2 / 4 lanes): 5-point 1000^2
    // 0.25 / 0.27 / 0.32 ms, 7-point 100^3 0.29 / 0.31 / 0.37 ms, power-law
    // graphs of average degree 8 and 16 1.25 / 1.26 / 1.31 and 5.25 / 5.34 /
    // 5.52 ms (their rows past 32 entries go to the whole wavefront anyway),
    // 27-point 100^3 (average 25) 0.61 / 0.50 / 0.45 ms; 8 lanes never won
    // below an average of 64.
    const double avg = g->n > 0 ? (double)g->nnz / (double)g->n : 0.0;
    if (avg < 20) return 1;
    if (avg < 64) return 4;
    if (avg < 256) return 8;
    return 16;
}

// Workgroups of the segmented sweeps: a multiple of 8 (one run of logical
// blocks per XCD), about 320 vertices per workgroup, at most kMaxBlocks.
// Measured on gfx950 with the 27-point 100^3 graph: 2048 workgroups ran
// MIS-2 in 0.49 ms, 3072 in 0.46 ms, 4096 in 0.47 ms.
// One workgroup (4 wavefronts) per about 640 vertices, in whole multiples of
// the 256 compute units once there are that many: on a 10^6-row graph 1536
// workgroups, six per CU, all resident at once, so every round (most are
// short) is one wave of dispatch with no partial second one.  Smaller graphs
// take one workgroup per 320 vertices (a multiple of 8, one per XCD).
int blocks_for(const mis2_ctx *ctx, int64_t n) {
    if (ctx->plan.blocks) return ctx->plan.blocks;
    int64_t b = (n + 639) / 640;
    b = b >= 256 ? (b + 128) / 256 * 256 : std::min<int64_t>(256, ((n + 319) / 320 + 7) / 8 * 8);
    return (int)std::max<int64_t>(8, std::min<int64_t>(b, kMaxBlocks));
}

int maybe_validate(mis2_ctx *ctx, const mis2_graph *g, const Workspace &ws, hipStream_t s) {
    if (!ctx->validate || g->n == 0) return MIS2_OK;
    uint32_t *err = ws.scalars + kS_Err;
    HIP_TRY(ctx, launch_fill_u32(err, 0u, 1, s));
    HIP_TRY(ctx, launch_validate(g->n, g->nnz, g->row_ptr, g->col, err, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[0])
        return fail(ctx, MIS2_EGRAPH, "invalid CSR (check bits 0x%x)", ctx->pinned[0]);
    return MIS2_OK;
}

int get_workspace(mis2_ctx *ctx, const mis2_graph *g, int op, Workspace *ws) {
    const size_t need = workspace_bytes(g->n, op);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "workspace of %zu bytes needed, %zu set", need,
                    ctx->ws ? ctx->ws_bytes : (size_t)0);
    if (!carve(ctx->ws, ctx->ws_bytes, g->n, op, ws))
        return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
    // the compacted adjacency, when the workspace has room for it past the end
    if (ctx->ws_bytes >= need + compact_bytes(g->n, g->nnz)) {
        char *tail = (char *)ctx->ws + need;
        ws->colc = (int32_t *)tail;
        ws->lenc = (int32_t *)(tail + align_up(4 * (size_t)std::max<int64_t>(g->nnz, 1)));
    }
    return MIS2_OK;
}

hipEvent_t take_event(mis2_ctx *ctx) {
    if (ctx->events_used == ctx->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->events.push_back(e);
    }
    return ctx->events[ctx->events_used++];
}

struct Launch {
    int kind, phase, round, lanes;  // kind 3: the tail kernel, from round `round` on
    hipEvent_t e0, e1;
    bool persistent = false;  // a sweep inside a persistent launch (timed by device stamps)
    int compact = 0;          // mis2_sweep_record.compact
    int cstart = -1;          // tail: first compacting round (< 0: none)
};


// Segment geometry of a run: S wavefronts, seg vertices each.
struct Geometry {
    int blocks;
    int64_t S, seg;
};

Geometry geometry(const mis2_ctx *ctx, int64_t n, int lanes) {
    Geometry gm;
    gm.blocks = blocks_for(ctx, n);
    if (!ctx->plan.blocks && lanes == kStagedLanes) {
        // the staged sweeps' LDS slots limit the resident workgroups; one
        // wave of dispatch per round
        if (ctx->staged_blocks < 0) ctx->staged_blocks = sweep_resident_blocks(lanes, ctx->num_cus);
        const int cap = ctx->staged_blocks / 8 * 8;
        if (cap >= 8 && gm.blocks > cap) gm.blocks = cap;
    }
    if (!ctx->plan.blocks && ctx->plan.persistent) {
        // the persistent launch needs every workgroup resident at once
        const int cap = rounds_max_blocks(lanes, ctx->num_cus) / 8 * 8;
        if (cap >= 8 && gm.blocks > cap) gm.blocks = cap;
    }
    gm.S = (int64_t)gm.blocks * (kBlock / 64);
    gm.seg = std::max<int64_t>(1, (n + gm.S - 1) / gm.S);
    return gm;
}

// Per-round sizes as recorded by the sweeps in the round table (rows
// 0..rounds-1): queue_trace copies them to pinned memory on the stream; after
// the call's final synchronisation parse_trace turns them into ctx->trace and
// the round count (the first round with an empty worklist1 ends the run).
int queue_trace(mis2_ctx *ctx, const Workspace &ws, int phase, int rounds, hipStream_t s,
                bool written = false) {
    ctx->trace_rounds[phase] = rounds;
    if (rounds > 0 && !written)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned_rt + (size_t)phase * (kTraceCap + 2) * kRoundStride,
                                    ws.rt, (size_t)rounds * kRoundStride * sizeof(uint32_t),
                                    hipMemcpyDeviceToHost, s));
    return MIS2_OK;
}

int32_t parse_trace(mis2_ctx *ctx, int phase) {
    if (ctx->tail_used[phase]) {
        // rows written by the tail kernel, up to the one that ended the run
        const unsigned long long e = __atomic_load_n(ctx->alive_host + 2 + phase, __ATOMIC_ACQUIRE);
        if (e > 0 && e <= (unsigned long long)kTraceCap) ctx->trace_rounds[phase] = (int)e;
        ctx->tail_used[phase] = 0;
    }
    const int rounds = ctx->trace_rounds[phase];
    const uint32_t *rt = ctx->pinned_rt + (size_t)phase * (kTraceCap + 2) * kRoundStride;
    std::vector<int64_t> &tr = ctx->trace[phase];
    tr.clear();
    std::vector<float> &st = ctx->stamp_ms[phase];
    st.clear();
    auto stamp_at = [&](int row, int word) {
        const uint32_t *p = &rt[(size_t)row * kRoundStride + word];
        return (double)((uint64_t)p[0] | ((uint64_t)p[1] << 32));
    };
    for (int q = 0; q < rounds && ctx->stamps_valid[phase]; q++) {
        const double t0 = stamp_at(q, kRtStamp0), t1 = stamp_at(q, kRtStamp1),
                     t2 = stamp_at(q, kRtStamp2);
        st.push_back((float)((t1 - t0) / ctx->wall_khz));
        st.push_back((float)((t2 - t1) / ctx->wall_khz));
    }
    int r = 0;
    for (; r < rounds; r++) {
        const int64_t c1 = rt[(size_t)r * kRoundStride], c2 = rt[(size_t)r * kRoundStride + 1];
        if (c1 == 0) break;
        tr.push_back(c1);
        tr.push_back(c2);
    }
    return r;
}

constexpr int kFallBack = 1;

// Round 0 of an unmasked run on one graph of at least kGenMinN vertices
// computes its neighbours' tuples rather than gathering them (the tuples are
// a pure function of the id).  Measured on gfx950 (mis2_run +
// mis2_aggregate): Chung-Lu 4M 12.42 -> 11.63 ms; 7-point 100^3 0.617 ->
// 0.611 ms; 27-point 100^3, staged sweeps, 1.053 -> 1.073 ms (its T, 4 MB,
// stays in the L2s, so a gather costs less than the hash).
constexpr int64_t kGenMinN = (int64_t)1 << 21;

RoundsArgs round_args(const mis2_ctx *ctx, const mis2_graph *g, uint64_t seed,
                      const Workspace &ws, const Geometry &gm, bool masked,
                      unsigned long long *degs, int lanes);

// All rounds in one cooperative launch (k_rounds).  Returns kFallBack when
// the grid cannot be made co-resident, so the caller issues rounds instead.
int run_rounds_persistent(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, const Workspace &ws,
                          const Geometry &gm, bool masked, int phase, hipStream_t s,
                          int32_t *iters_out, std::vector<Launch> *launches, int lanes) {
    const int cap = rounds_max_blocks(lanes, ctx->num_cus);
    if (cap < gm.blocks) return kFallBack;  // geometry() sizes the default plan to fit
    unsigned long long *degs = ws.degs + (size_t)phase * kTraceCap * kDegStride;
    HIP_TRY(ctx, launch_fill_u32(ws.bar, 0u, kBarWords, s));
    RoundsArgs a = round_args(ctx, g, seed, ws, gm, masked, degs, lanes);
    a.alive_host = nullptr;  // the host waits for the whole launch
    a.colc = nullptr;        // the single launch does not compact
    a.lenc = nullptr;
    Launch lp{2, phase, -1, lanes, nullptr, nullptr};
    if (ctx->profile) {
        lp.e0 = take_event(ctx), lp.e1 = take_event(ctx);
        if (!lp.e0 || !lp.e1) return fail(ctx, MIS2_EHIP, "hipEventCreate failed");
        HIP_TRY(ctx, hipEventRecord(lp.e0, s));
    }
    HIP_TRY(ctx, launch_rounds(lanes, gm.blocks, g->row_ptr, g->col, ws.T, ws.M, a, s));
    if (ctx->profile) HIP_TRY(ctx, hipEventRecord(lp.e1, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned + 32, ws.bar + kMaxBlocks, 64 * sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[32 + 16])
        return fail(ctx, MIS2_EINTERNAL, "grid barrier timed out in the round kernel");
    const int rounds = (int)ctx->pinned[32 + 32];
    ctx->stamps_valid[phase] = 1;
    // the row of the round that ended the run is written too
    int rc = queue_trace(ctx, ws, phase, std::min(rounds + 1, kTraceCap), s);
    if (rc) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (parse_trace(ctx, phase) >= rounds && rounds + 2 >= kTraceCap)
        return fail(ctx, MIS2_EINTERNAL, "more than %d rounds", kTraceCap - 2);
    *iters_out = rounds;
    for (int r = 0; r < rounds; r++) {
        launches->push_back(Launch{0, phase, r, lanes, nullptr, nullptr, true});
        launches->push_back(Launch{1, phase, r, lanes, nullptr, nullptr, true});
    }
    launches->push_back(lp);
    return MIS2_OK;
}

// The round loop of Algorithm 1.  Round 0 starts from the identity
// worklists (whole graph, masked == false) or from the per-wave lists of the
// active vertices already in wl1[0] / cnt1[0] (induced subgraph; T and M
// already initialised).
//
// A round issued after the last one finds empty per-wavefront lists and
// does nothing.  Workgroup 0 of
// each Refresh Column stores (round, |worklist1|) in a host-pinned word as
// the round starts; the host polls that word and keeps only a round or two
// queued beyond the one running, so it stops issuing as soon as a round
// reports an empty worklist1 and never sleeps in the driver.  (Measured on
// gfx950 with ROCm 7.2: two direct launches cost the host 5 us, a two-kernel
// HIP graph launch 16 us and a stream query 11 us, so rounds are launched
// directly and the stream is queried only after a long wait.)  The per-round
// sizes the sweeps record in the round table give the round count afterwards.
constexpr double kProgressTimeoutS = 60.0;  // no round started for this long: give up
constexpr double kQueryAfterS = 1e-3;       // check the stream for errors after this long idle

RoundsArgs round_args(const mis2_ctx *ctx, const mis2_graph *g, uint64_t seed,
                      const Workspace &ws, const Geometry &gm, bool masked,
                      unsigned long long *degs, int lanes) {
    RoundsArgs a;
    memset(&a, 0, sizeof a);
    const TupleParams tp = tparams(ctx, g->n, seed, 0);
    a.batch = ctx->batch;
    for (int i = 0; i < 2; i++) {
        a.wl1[i] = ws.wl1[i];
        a.wl2[i] = ws.wl2[i];
        a.cnt1[i] = ws.cnt1[i];
        a.cnt2[i] = ws.cnt2[i];
    }
    a.rt = ws.rt;
    a.rt_host = nullptr;  // set by run_rounds for launched rounds
    a.ctr = ws.ctr;
    a.alive_host = ctx->alive_host;
    a.epoch = 0;  // run_rounds gives each run its own
    a.degs = ctx->account ? degs : nullptr;
    a.dsplit = ctx->account ? ws.dsplit : nullptr;
    a.bar = ws.bar;
    a.lflag = ws.lflag;
    a.n = g->n;
    a.nnz = g->nnz;
    a.seg = gm.seg;
    a.S = gm.S;
    a.seed = seed;
    a.pmask = tp.pmask;
    a.b = tp.b;
    a.masked = masked ? 1 : 0;
    a.max_rounds = kTraceCap;
    // rounds 0 and 1 compute their tuples in place of gathering them where T
    // outgrows the L2 of an XCD (4 MB); on smaller graphs the gathers hit and
    // the hash costs more
    a.gen0 = g->n >= kGenMinN ? 1 : 0;
    a.near = ws.near;
    // compacted Refresh Column rows (L-lane sweeps only; the flat sweeps
    // read the CSR as given)
    if (ws.colc && ws.lenc && lanes > 0 && ctx->plan.compact && g->nnz > 0) {
        a.colc = ws.colc;
        a.lenc = ws.lenc;
    }
    return a;
}

// long_rows: for an unmasked run, out: 1 if round 0 met rows longer than the
// cooperative threshold, 0 if not (or if the run ended before round 1
// started); for a masked run, in: the value of the unmasked run of the same
// graph.  Refresh Column compacts (launch modes 1 then 2) only when it is 1.
// The ablation kernels' configuration (null: the production kernels).
struct AblRun {
    bool unpacked = false;  // three-field tuples
    bool all = false;       // every vertex every round
    int pflags = 0;         // kAblFixed | kAblXorshift
    AblTuples T, M;
};

// The words a run of rounds starts from: size counters zero (a masked run
// keeps slot 0, which holds its active count), round table row 0 = n and
// the long-row flags clear (unmasked runs).  Callers launch them with the
// round-0 tuples (filled = true) or run_rounds does (filled = false).
FillSpans round_fills(const mis2_graph *g, const Workspace &ws, bool masked) {
    FillSpans f;
    f.add(ws.ctr + (masked ? kCtrSlot : 0), 0u,
          (int64_t)(masked ? kCtrRing - 1 : kCtrRing) * kCtrSlot);
    if (!masked) f.add(ws.rt, (uint32_t)g->n, 2);
    if (!masked) f.add(ws.lflag, 0u, (int64_t)kSplit * kCtrLine);
    // round 1's marks start clear (set after round 0)
    if (!masked && g->n >= kGenMinN && ws.near) f.add((uint32_t *)ws.near, 0u, (g->n + 3) / 4);
    return f;
}

// Staged plans on graphs without long rows switch to kLateLanes-lane kernels
// once the host sees |worklist2| * kLateShare < n.  Measured on gfx950 (27-point 100^3,
// mis2_run + mis2_aggregate, staged sweeps at 1024 workgroups with the tail):
// 1.055-1.061 ms staged throughout; switching at n/2 1.041, n/4 1.035, n/8
// 1.052 ms; 2 lanes at n/4 1.048 ms.  The staged kernels stage each row in
// LDS, which pays while rows are dense and costs 1-2 us per launch once they
// are sparse.
constexpr int kLateLanes = 4;
constexpr uint64_t kLateShare = 4;

int run_rounds(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, const Workspace &ws,
               const Geometry &gm, bool masked, int phase, hipStream_t s, int32_t *iters_out,
               std::vector<Launch> *launches, int *long_rows, const AblRun *abl = nullptr,
               bool filled = false) {
    const int lanes = abl ? 1 : lanes_for(ctx, g);
    unsigned long long *degs = ws.degs + (size_t)phase * kTraceCap * kDegStride;
    if (ctx->account) {
        HIP_TRY(ctx, launch_fill_u64(degs, 0ull, kDegStride * kTraceCap, s));
        HIP_TRY(ctx, launch_fill_u64(ws.dsplit, 0ull, 2 * (int64_t)kSplit * 16, s));
    }
    // size counters: every ring slot zero except slot 0 of a masked start,
    // which holds its active count; each Refresh Column clears the slot two
    // rounds ahead.
    if (!filled) HIP_TRY(ctx, launch_fill_spans(round_fills(g, ws, masked), s));
    if (ctx->plan.persistent && !abl) {
        if (!masked) *long_rows = 0;
        int rc = run_rounds_persistent(ctx, g, seed, ws, gm, masked, phase, s, iters_out, launches,
                                       lanes);
        if (rc != kFallBack) return rc;
    }
    RoundsArgs a = round_args(ctx, g, seed, ws, gm, masked, degs, lanes);
    // workgroup 0 of each Refresh Column writes its round's sizes straight
    // into the host-pinned round table of this phase
    a.rt_host = ctx->pinned_rt + (size_t)phase * (kTraceCap + 2) * kRoundStride;
    if (abl) {
        a.colc = nullptr;
        a.lenc = nullptr;
        a.degs = nullptr;
        a.dsplit = nullptr;
        a.abl = abl->pflags;
    }
    // compaction: unknown (-1) until round 1 reports what round 0 met
    int longs = masked ? (*long_rows > 0 ? 1 : 0) : -1;
    const int cfrom = masked ? 0 : kCompactFrom;
    int cstart = -1;  // first compacting round
    // a new epoch: words still arriving from the late rounds of the run
    // before this one carry the old one and are ignored
    ctx->epoch = ctx->epoch % kEpochMax + 1;
    a.epoch = ctx->epoch;
    __atomic_store_n(ctx->alive_host + 1, ~0ull, __ATOMIC_RELEASE);
    __atomic_store_n(ctx->alive_host, ~0ull, __ATOMIC_RELEASE);
    ctx->tail_used[phase] = 0;
    // the last rounds go to the one-workgroup tail once both worklists fit it
    const bool tail_ok = ctx->plan.tail > 0 && !abl && lanes != 0 && g->nnz > 0;
    int round = 0;  // rounds issued
    int late_lanes = 0;  // staged plans: lanes of the sparse rounds once switched
    auto last_progress = std::chrono::steady_clock::now();
    int last_seen = -2;
    for (;;) {
        const unsigned long long v = __atomic_load_n(ctx->alive_host, __ATOMIC_ACQUIRE);
        int seen = -1;  // round of the latest Refresh Column of this run that has started
        uint32_t live = 1;
        if (v != ~0ull && (uint32_t)(v >> 48) == a.epoch) {
            seen = (int)((v >> 32) & 0xFFFFu);
            live = (uint32_t)v & ~kLongRowsBit;
            if (longs < 0 && seen >= 1) longs = ((uint32_t)v & kLongRowsBit) ? 1 : 0;
        }
        if (live == 0u) break;  // worklist1 empty: the run has ended at round `seen`
        if (seen != last_seen) {
            last_seen = seen;
            last_progress = std::chrono::steady_clock::now();
        }
        // queue depth beyond the running round: two while rounds are big,
        // one near the end (fewer rounds issued past it); a round that could
        // compact waits until the host knows whether it should
        // Measured on gfx950 (mis2_run + mis2_aggregate): two rounds ahead
        // throughout against two, then one once |worklist1| < 4096: 5-point
        // 64^2 0.374 / 0.409 ms, 7-point 100^3 0.681 / 0.693 ms, C2 1.109 /
        // 1.122 ms; three ahead 0.382, 0.695, 1.114 ms.  The round issued
        // past the end costs less than the host gaps a shallow queue leaves
        // between the short late rounds.
        const int ahead = ctx->plan.ahead > 0 ? ctx->plan.ahead : 2;
        const bool can_compact = a.colc != nullptr && round >= cfrom;
        if (round - seen <= ahead && !(can_compact && longs < 0)) {
            if (round + 2 >= kTraceCap)
                return fail(ctx, MIS2_EINTERNAL, "more than %d rounds", kTraceCap - 2);
            if (tail_ok && round >= 1 && seen >= (masked ? 0 : 1) && live < (uint32_t)kTailCap &&
                !(a.colc && longs < 0)) {
                // worklist2 at round `seen` (word 1, written before word 0)
                const unsigned long long w2 = __atomic_load_n(ctx->alive_host + 1, __ATOMIC_ACQUIRE);
                if (w2 != ~0ull && (uint32_t)(w2 >> 48) == a.epoch &&
                    (int)((w2 >> 32) & 0xFFFFu) == seen && (uint32_t)w2 < (uint32_t)kTailCap) {
                    int cs = -1;  // first compacting round
                    if (a.colc && longs > 0) cs = cstart >= 0 ? cstart : std::max(round, cfrom);
                    Launch lt{3, phase, round, lanes, nullptr, nullptr};
                    lt.cstart = cs;
                    if (ctx->profile) {
                        lt.e0 = take_event(ctx), lt.e1 = take_event(ctx);
                        if (!lt.e0 || !lt.e1) return fail(ctx, MIS2_EHIP, "hipEventCreate failed");
                    }
                    __atomic_store_n(ctx->alive_host + 2 + phase, 0ull, __ATOMIC_RELEASE);
                    uint32_t *rt_host =
                        ctx->pinned_rt + (size_t)phase * (kTraceCap + 2) * kRoundStride;
                    HIP_TRY(ctx, launch_tail(g->row_ptr, g->col, ws.T, ws.M, a, round, cs,
                                             coop_threshold(lanes), rt_host,
                                             ctx->alive_host + 2 + phase, s, lt.e0, lt.e1));
                    launches->push_back(lt);
                    if (!masked) *long_rows = longs > 0 ? 1 : 0;
                    // the tail stamps its rounds' phases in the round table
                    ctx->stamps_valid[phase] = 1;
                    *iters_out = round;
                    // every row is in host memory already (the launched rounds
                    // and the tail write them)
                    int rc = queue_trace(ctx, ws, phase, round, s, true);
                    ctx->tail_used[phase] = 1;
                    return rc;
                }
            }
            int mode = 0;
            if (can_compact && longs > 0) {
                if (cstart < 0) cstart = round;
                mode = round == cstart ? 1 : 2;
            }
            // the staged sweeps hand the sparse rounds to 4-lane kernels
            // (same segments, same results), whose per-launch cost is lower
            // once few rows are left; only where no row is long, so that no
            // round compacts (the two kernels' compaction thresholds differ)
            if (lanes == kStagedLanes && !abl && !late_lanes && longs == 0) {
                const unsigned long long w2 = __atomic_load_n(ctx->alive_host + 1, __ATOMIC_ACQUIRE);
                if (w2 != ~0ull && (uint32_t)(w2 >> 48) == a.epoch &&
                    (uint64_t)(uint32_t)w2 * kLateShare < (uint64_t)g->n)
                    late_lanes = kLateLanes;
            }
            const int rl = late_lanes ? late_lanes : lanes;
            Launch lc{0, phase, round, rl, nullptr, nullptr, false, mode};
            Launch ld{1, phase, round, rl, nullptr, nullptr};
            if (ctx->profile) {
                lc.e0 = take_event(ctx), lc.e1 = take_event(ctx);
                ld.e0 = take_event(ctx), ld.e1 = take_event(ctx);
                if (!lc.e0 || !lc.e1 || !ld.e0 || !ld.e1)
                    return fail(ctx, MIS2_EHIP, "hipEventCreate failed");
            }
            if (abl) {
                HIP_TRY(ctx, launch_abl_round(0, abl->unpacked, abl->all, gm.blocks, g->row_ptr,
                                              g->col, abl->T, abl->M, a, round, s, lc.e0, lc.e1));
                HIP_TRY(ctx, launch_abl_round(1, abl->unpacked, abl->all, gm.blocks, g->row_ptr,
                                              g->col, abl->T, abl->M, a, round, s, ld.e0, ld.e1));
            } else {
                HIP_TRY(ctx, launch_col_round(rl, gm.blocks, g->row_ptr, g->col, ws.T, ws.M,
                                              a, round, mode, s, lc.e0, lc.e1));
                HIP_TRY(ctx, launch_dec_round(rl, gm.blocks, g->row_ptr, g->col, ws.T, ws.M,
                                              a, round, s, ld.e0, ld.e1));
                // round 1's Refresh Column computes its tuples once the IN
                // vertices have marked their neighbourhoods, and its Decide
                // Set reads the marks of their neighbours
                if (round == 0 && a.gen0 && !masked && !a.batch.voff) {
                    HIP_TRY(ctx, launch_push_in(g->n, g->row_ptr, g->col, ws.T, ws.M, s));
                    if (ws.near)
                        HIP_TRY(ctx,
                                launch_push_near(g->n, g->row_ptr, g->col, ws.M, ws.near, s));
                }
            }
            launches->push_back(lc);
            launches->push_back(ld);
            round++;
            continue;
        }
        // the GPU is behind: wait for the next round to start
        const double idle =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - last_progress).count();
        if (idle > kQueryAfterS) {
            const hipError_t q = hipStreamQuery(s);
            if (q != hipSuccess && q != hipErrorNotReady) HIP_TRY(ctx, q);
        }
        if (idle > kProgressTimeoutS)
            return fail(ctx, MIS2_EHIP, "no MIS-2 round started for %.0f s", idle);
    }
    if (!masked) *long_rows = longs > 0 ? 1 : 0;
    ctx->stamps_valid[phase] = 0;
    *iters_out = round;  // rounds issued; parse_trace gives the count after the sync
    return queue_trace(ctx, ws, phase, round, s, true);
}

// Fill ctx->sweeps from the launches of the finished call.
int collect_sweeps(mis2_ctx *ctx, const std::vector<Launch> &launches, const Workspace &ws,
                   hipStream_t s) {
    ctx->sweeps.clear();
    std::vector<unsigned long long> degs;
    if (ctx->account) {
        degs.resize((size_t)2 * kTraceCap * kDegStride);
        HIP_TRY(ctx, hipMemcpyAsync(degs.data(), ws.degs, degs.size() * sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
    }
    for (const Launch &l : launches) {
        const std::vector<int64_t> &tr = ctx->trace[l.phase];
        const int rounds = (int)(tr.size() / 2);
        if (l.kind == 2) {
            // one persistent launch covering every round of this phase
            mis2_sweep_record rec;
            memset(&rec, 0, sizeof rec);
            rec.kind = 2;
            rec.phase = l.phase;
            rec.round = -1;
            rec.lanes = l.lanes == kStagedLanes ? MIS2_LANES_STAGED : l.lanes;
            rec.rows = 0;
            rec.edges = ctx->account ? 0 : -1;
            for (int r = 0; r < rounds; r++) {
                rec.rows += tr[2 * r] + tr[2 * r + 1];
                if (ctx->account)
                    rec.edges += (int64_t)degs[((size_t)l.phase * kTraceCap + r) * kDegStride] +
                                 (int64_t)degs[((size_t)l.phase * kTraceCap + r) * kDegStride + 1];
            }
            rec.rows_out = rounds;
            rec.compact = l.compact;
            rec.written = ctx->account ? 0 : -1;
            rec.ms = -1.0f;
            if (ctx->profile && l.e0 && l.e1) {
                float ms = 0.f;
                HIP_TRY(ctx, hipEventElapsedTime(&ms, l.e0, l.e1));
                rec.ms = ms;
            }
            ctx->sweeps.push_back(rec);
            continue;
        }
        if (l.kind == 3) {
            // the tail kernel: one record per sweep it ran (untimed), then its own
            mis2_sweep_record sum;
            memset(&sum, 0, sizeof sum);
            sum.kind = 3;
            sum.phase = l.phase;
            sum.round = l.round;
            sum.lanes = l.lanes == kStagedLanes ? MIS2_LANES_STAGED : l.lanes;
            sum.edges = ctx->account ? 0 : -1;
            sum.written = ctx->account ? 0 : -1;
            sum.rows_out = std::max(0, rounds - l.round);
            for (int r = l.round; r < rounds; r++) {
                for (int kind = 0; kind < 2; kind++) {
                    mis2_sweep_record rec;
                    memset(&rec, 0, sizeof rec);
                    rec.kind = kind;
                    rec.phase = l.phase;
                    rec.round = r;
                    rec.lanes = sum.lanes;
                    const int list = kind == 0 ? 1 : 0;
                    rec.rows = tr[2 * r + list];
                    rec.rows_out = r + 1 < rounds ? tr[2 * (r + 1) + list] : 0;
                    const size_t di = ((size_t)l.phase * kTraceCap + r) * kDegStride;
                    rec.edges = ctx->account ? (int64_t)degs[di + list] : -1;
                    rec.written = ctx->account && kind == 0 ? (int64_t)degs[di + 2] : -1;
                    rec.compact = kind == 0 && l.cstart >= 0 && r >= l.cstart
                                      ? (r == l.cstart ? 1 : 2) : 0;
                    rec.ms = -1.0f;
                    const std::vector<float> &st = ctx->stamp_ms[l.phase];
                    if (ctx->profile && (size_t)(2 * r + kind) < st.size()) rec.ms = st[2 * r + kind];
                    ctx->sweeps.push_back(rec);
                    sum.rows += rec.rows;
                    if (ctx->account) sum.edges += rec.edges;
                    if (ctx->account && kind == 0) sum.written += rec.written;
                }
            }
            sum.ms = -1.0f;
            if (ctx->profile && l.e0 && l.e1) {
                float ms = 0.f;
                HIP_TRY(ctx, hipEventElapsedTime(&ms, l.e0, l.e1));
                sum.ms = ms;
            }
            ctx->sweeps.push_back(sum);
            continue;
        }
        if (l.round >= rounds) {
            // issued after the run had finished: found empty worklists
            mis2_sweep_record rec;
            memset(&rec, 0, sizeof rec);
            rec.kind = l.kind == 0 ? 4 : 5;
            rec.phase = l.phase;
            rec.round = l.round;
            rec.lanes = l.lanes == kStagedLanes ? MIS2_LANES_STAGED : l.lanes;
            rec.edges = ctx->account ? 0 : -1;
            rec.written = ctx->account ? 0 : -1;
            rec.ms = -1.0f;
            if (ctx->profile && l.e0 && l.e1) {
                float ms = 0.f;
                HIP_TRY(ctx, hipEventElapsedTime(&ms, l.e0, l.e1));
                rec.ms = ms;
            }
            ctx->sweeps.push_back(rec);
            continue;
        }
        mis2_sweep_record rec;
        memset(&rec, 0, sizeof rec);
        rec.kind = l.kind;
        rec.phase = l.phase;
        rec.round = l.round;
        rec.lanes = l.lanes == kStagedLanes ? MIS2_LANES_STAGED : l.lanes;
        const int list = l.kind == 0 ? 1 : 0;
        rec.rows = tr[2 * l.round + list];
        rec.rows_out = l.round + 1 < rounds ? tr[2 * (l.round + 1) + list] : 0;
        const size_t di = ((size_t)l.phase * kTraceCap + l.round) * kDegStride;
        rec.edges = ctx->account ? (int64_t)degs[di + list] : -1;
        rec.written = ctx->account && l.kind == 0 ? (int64_t)degs[di + 2] : -1;
        rec.compact = l.compact;
        rec.ms = -1.0f;
        if (ctx->profile && l.e0 && l.e1) {
            float ms = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, l.e0, l.e1));
            rec.ms = ms;
        } else if (ctx->profile && l.persistent) {
            const std::vector<float> &st = ctx->stamp_ms[l.phase];
            const size_t k = (size_t)l.round * 2 + (size_t)l.kind;
            if (k < st.size()) rec.ms = st[k];
        }
        ctx->sweeps.push_back(rec);
    }
    return MIS2_OK;
}

// ---------------------------------------------------------------------------
// Plan tuner.  Launch plans (lanes per row, grid) never change results, only
// time, and the best one depends on the graph: the degree rule of Section V-D
// (lanes_for) is right for some graphs and not others.  A graph is
// classified by its size and degree histogram (one small kernel, read back
// once per graph and context); the first time a class is seen on a device,
// a few candidate plans each run the graph's MIS-2 twice and the fastest is
// kept for the class, process-wide, so every context on the device uses it.
// ---------------------------------------------------------------------------
constexpr int64_t kTuneMinN = 16384;   // smaller graphs keep the degree rule
constexpr double kTuneMargin = 0.01;    // a candidate replaces the best when 1% faster
constexpr size_t kSeenCap = 32;        // graphs remembered per context

struct TuneEntry {
    GraphClass cls;
    Plan plan;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tuned[64];    // per device

int size_bucket(int64_t n) {
    // floor(2 log2 n) from the integer log and the top bits
    int lg = 0;
    while ((n >> (lg + 1)) > 0) lg++;
    const bool upper = lg >= 1 ? ((n >> (lg - 1)) & 1) != 0 : false;  // n >= 1.5 * 2^lg
    return 2 * lg + (upper ? 1 : 0);
}

int host_deg_bin(uint64_t d) {
    if (d == 0) return 0;
    if (d <= 2) return 1;
    if (d <= 4) return 2;
    if (d <= 8) return 3;
    if (d <= 16) return 4;
    if (d <= 32) return 5;
    if (d <= 128) return 6;
    if (d <= 1024) return 7;
    return 8;
}

// The class of g (cached per context by row_ptr, n and nnz).
int classify(mis2_ctx *ctx, const mis2_graph *g, const Workspace &ws, hipStream_t s,
             GraphClass *out) {
    for (size_t i = ctx->seen.size(); i-- > 0;) {
        const auto &e = ctx->seen[i];
        if (e.row_ptr == g->row_ptr && e.n == g->n && e.nnz == g->nnz) {
            *out = e.cls;
            return MIS2_OK;
        }
    }
    // partial rows go to the accounting sums' buffer (idle here; an
    // accounting run clears it before use), then to pinned host memory
    HIP_TRY(ctx, launch_degree_hist(g->n, g->row_ptr, ws.degs, s));
    static_assert((size_t)kHistBlocks * kHistWords * 8 <= 2 * (size_t)kCtrList * 4,
                  "histogram read-back fits the pinned counter buffer");
    unsigned long long *h = (unsigned long long *)ctx->pinned_ctr;
    HIP_TRY(ctx, hipMemcpyAsync(h, ws.degs, (size_t)kHistBlocks * kHistWords * 8,
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    unsigned long long cnt[kDegBins] = {}, mx = 0;
    for (int b = 0; b < kHistBlocks; b++) {
        for (int k = 0; k < kDegBins; k++) cnt[k] += h[(size_t)b * kHistWords + k];
        mx = std::max(mx, h[(size_t)b * kHistWords + kDegBins]);
    }
    GraphClass c;
    c.size_bucket = size_bucket(g->n);
    for (int k = 0; k < kDegBins; k++)
        c.share[k] = (uint8_t)((cnt[k] * 16 + (unsigned long long)g->n / 2) / (unsigned long long)g->n);
    c.max_bin = host_deg_bin(mx);
    if (ctx->seen.size() >= kSeenCap) ctx->seen.erase(ctx->seen.begin());
    ctx->seen.push_back({g->row_ptr, g->n, g->nnz, c});
    *out = c;
    return MIS2_OK;
}

// Host wall time of one MIS-2 run of g (round 0 tuples, the rounds, a final
// synchronisation) with the context's current plan.
int time_mis2(mis2_ctx *ctx, const mis2_graph *g, const Workspace &ws, hipStream_t s,
              double *sec) {
    std::vector<Launch> launches;
    const Geometry gm = geometry(ctx, g->n, lanes_for(ctx, g));
    int32_t iters = 0;
    int long_rows = 0;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    const auto t0 = std::chrono::steady_clock::now();
    HIP_TRY(ctx, launch_init_tuples(tparams(ctx, g->n, 0, 0), g->n, ws.T,
                                    round_fills(g, ws, false), s));
    int rc = run_rounds(ctx, g, 0, ws, gm, false, 0, s, &iters, &launches, &long_rows, nullptr,
                        true);
    if (rc) return rc;
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MIS2_OK;
}

int tune(mis2_ctx *ctx, const mis2_graph *g, const Workspace &ws, hipStream_t s, Plan *best) {
    std::vector<Plan> cand;
    for (int L : {1, 2, 4, 8}) {
        Plan p = ctx->plan;
        p.lanes = L;
        cand.push_back(p);
    }
    if (g->nnz >= 4) {
        Plan p = ctx->plan;
        p.lanes = kStagedLanes;
        cand.push_back(p);
    }
    const bool tune_tail = ctx->plan.tail < 0;
    for (Plan &p : cand)
        if (tune_tail) p.tail = 0;
    const int saved_profile = ctx->profile, saved_account = ctx->account;
    const Plan saved_plan = ctx->plan;
    ctx->profile = 0;
    ctx->account = 0;
    ctx->tuning.clear();
    double best_t = 0;
    int rc = MIS2_OK;
    for (size_t ci = 0; ci < cand.size() + (tune_tail ? 1 : 0); ci++) {
        Plan p;
        if (ci < cand.size()) {
            p = cand[ci];
        } else {
            p = *best;  // the fastest so far, with its last rounds in the tail
            p.tail = 1;
        }
        ctx->plan = p;
        double t = 1e30;
        for (int rep = 0; rep < 2 && rc == MIS2_OK; rep++) {
            double x = 0;
            rc = time_mis2(ctx, g, ws, s, &x);
            t = std::min(t, x);
        }
        if (rc) break;
        const Geometry gm = geometry(ctx, g->n, lanes_for(ctx, g));
        ctx->tuning.push_back({p.lanes == kStagedLanes ? MIS2_LANES_STAGED : p.lanes, gm.blocks,
                               p.tail > 0 ? 1 : 0, (float)(t * 1e3)});
        // a later candidate must be clearly faster: timing noise alone does
        // not flip the choice between plans that run alike.  The tail
        // candidate needs only to be no slower: it is timed on one MIS-2,
        // and an aggregation runs two, each ending in the tail (27-point
        // 100^3, mis2_run + mis2_aggregate: 1.05 ms with it, 1.07 without)
        const bool tail_cand = ci >= cand.size();
        if (ctx->tuning.size() == 1 || t < best_t * (1.0 - (tail_cand ? 0.0 : kTuneMargin))) {
            best_t = t;
            *best = p;
        }
    }
    ctx->plan = saved_plan;
    ctx->profile = saved_profile;
    ctx->account = saved_account;
    return rc;
}

// Sets the plan of this call: the tuned plan of g's class when the context's
// plan is automatic (tuning the class first if it is new), else the
// context's own.  *saved receives the plan to restore after the call.
int apply_plan(mis2_ctx *ctx, const mis2_graph *g, const Workspace &ws, hipStream_t s,
               Plan *saved) {
    *saved = ctx->plan;
    ctx->last_source = 0;
    const bool automatic = ctx->plan.lanes == 0 && ctx->plan.blocks == 0 && !ctx->plan.persistent;
    if (!ctx->autotune || !automatic || g->n < kTuneMinN || ctx->device < 0 || ctx->device >= 64)
        return MIS2_OK;
    GraphClass c;
    int rc = classify(ctx, g, ws, s, &c);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const TuneEntry &e : g_tuned[ctx->device]) {
            if (e.cls == c) {
                ctx->plan = e.plan;
                ctx->last_source = 1;
                return MIS2_OK;
            }
        }
    }
    if (ctx->autotune == 2) return MIS2_OK;  // lookup only: the degree rule
    Plan best = ctx->plan;
    if ((rc = tune(ctx, g, ws, s, &best))) return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[ctx->device].push_back({c, best});
    }
    ctx->plan = best;
    ctx->last_source = 2;
    return MIS2_OK;
}

// Restores the context's plan at the end of a call and records the one used.
struct PlanScope {
    mis2_ctx *ctx;
    const mis2_graph *g;
    Plan saved;
    bool armed = false;
    ~PlanScope() {
        if (!armed) return;
        const int L = lanes_for(ctx, g);
        ctx->last_lanes = L == kStagedLanes ? MIS2_LANES_STAGED : L;
        ctx->last_blocks = geometry(ctx, g->n, L).blocks;
        ctx->last_tail = ctx->plan.tail > 0 ? 1 : 0;
        ctx->plan = saved;
    }
};

}  // namespace

namespace mis2 {

// The ablation flags that take the ablation kernels (the others run the
// production kernels).
constexpr int kAblFamily = MIS2_ABL_FIXED_PRIORITY | MIS2_ABL_XORSHIFT | MIS2_ABL_NO_WORKLISTS |
                           MIS2_ABL_UNPACKED | MIS2_ABL_SIMPLE;

size_t ablation_bytes(int64_t n, int flags) {
    size_t b = workspace_bytes(n, MIS2_OP_MIS2);
    if (flags & MIS2_ABL_UNPACKED) b += 4 * align_up(4 * (size_t)std::max<int64_t>(n, 0));
    return b;
}

size_t compact_bytes(int64_t n, int64_t nnz) {
    return align_up(4 * (size_t)std::max<int64_t>(nnz, 1)) + align_up(4 * (size_t)std::max<int64_t>(n, 0));
}

size_t workspace_bytes(int64_t n, int op) {
    if (n < 0) return 0;
    const size_t un = (size_t)n;
    size_t b = 0;
    b += align_up(4 * un) * 2;                          // T, M
    b += align_up(un);                                  // near (round 1 of large graphs)
    b += align_up(4 * un) * 4;                          // wl1[2], wl2[2]
    b += align_up(4 * (size_t)kMaxWaves) * 4;           // cnt1[2], cnt2[2]
    b += align_up(4 * (size_t)(kTraceCap + 2) * kRoundStride);  // round table
    b += align_up(4 * (size_t)kCtrRing * kCtrSlot);     // size counters
    b += align_up(4 * kScalars);                        // scalars
    b += align_up(8 * 2 * kDegStride * (size_t)kTraceCap);  // degs
    b += align_up(8 * 2 * (size_t)kSplit * 16);         // their partial sums
    b += align_up(4 * (size_t)(compact_blocks(n) + 1)); // blocksum
    b += align_up(4 * (size_t)kBarWords);               // barrier state
    b += align_up(4 * (size_t)kSplit * kCtrLine);       // long-row flags
    if (op != MIS2_OP_MIS2) {
        b += align_up(4 * un) * 3;                      // label, list, aggsize
        b += align_up(un);                              // flag
    }
    if (op == MIS2_OP_COARSEN) {
        b += align_up(4 * un) * 2;                      // quotient counts, members
        b += align_up(8 * (un + 1));                    // member offsets
        b += align_up(8 * (size_t)scan_parts(n));       // scan partials
        b += align_up(4 * un) + align_up(4);            // large coarse rows and their count
        b += align_up(4 * (size_t)kGiantSlots * giant_words(n));  // giant rows' bitmaps
        b += align_up(4 * (size_t)kGiantMeta);
        b += align_up(un);                              // row classes
    }
    return b;
}

bool carve(void *base, size_t bytes, int64_t n, int op, Workspace *ws) {
    if (workspace_bytes(n, op) > bytes || ((uintptr_t)base % kAlign) != 0) return false;
    char *p = (char *)base;
    const size_t un = (size_t)n;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    ws->T = (uint32_t *)take(4 * un);
    ws->M = (uint32_t *)take(4 * un);
    ws->near = (uint8_t *)take(un);
    ws->wl1[0] = (int32_t *)take(4 * un);
    ws->wl1[1] = (int32_t *)take(4 * un);
    ws->wl2[0] = (int32_t *)take(4 * un);
    ws->wl2[1] = (int32_t *)take(4 * un);
    ws->cnt1[0] = (uint32_t *)take(4 * (size_t)kMaxWaves);
    ws->cnt1[1] = (uint32_t *)take(4 * (size_t)kMaxWaves);
    ws->cnt2[0] = (uint32_t *)take(4 * (size_t)kMaxWaves);
    ws->cnt2[1] = (uint32_t *)take(4 * (size_t)kMaxWaves);
    ws->rt = (uint32_t *)take(4 * (size_t)(kTraceCap + 2) * kRoundStride);
    ws->ctr = (uint32_t *)take(4 * (size_t)kCtrRing * kCtrSlot);
    ws->scalars = (uint32_t *)take(4 * kScalars);
    ws->degs = (unsigned long long *)take(8 * 2 * kDegStride * (size_t)kTraceCap);
    ws->dsplit = (unsigned long long *)take(8 * 2 * (size_t)kSplit * 16);
    ws->blocksum = (uint32_t *)take(4 * (size_t)(compact_blocks(n) + 1));
    ws->bar = (uint32_t *)take(4 * (size_t)kBarWords);
    ws->lflag = (uint32_t *)take(4 * (size_t)kSplit * kCtrLine);
    if (op != MIS2_OP_MIS2) {
        ws->label = (int32_t *)take(4 * un);
        ws->list = (int32_t *)take(4 * un);
        ws->aggsize = (int32_t *)take(4 * un);
        ws->flag = (uint8_t *)take(un);
    }
    if (op == MIS2_OP_COARSEN) {
        ws->q.cnt = (uint32_t *)take(4 * un);
        ws->q.members = (int32_t *)take(4 * un);
        ws->q.moff = (int64_t *)take(8 * (un + 1));
        ws->q.part = (unsigned long long *)take(8 * (size_t)scan_parts(n));
        ws->q.big = (int32_t *)take(4 * un);
        ws->q.big_count = (uint32_t *)take(4);
        ws->q.gbits = (uint32_t *)take(4 * (size_t)kGiantSlots * giant_words(n));
        ws->q.gmeta = (uint32_t *)take(4 * (size_t)kGiantMeta);
        ws->q.cls = (uint8_t *)take(un);
    }
    return true;
}

}  // namespace mis2

namespace {

// Workspace of mis2_run_noalloc: a device global array, so that the call
// allocates nothing.  Every GPU the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address on each GPU is taken once, with that GPU
// current, when the first context on it is created, and only that address
// is handed to kernels and copies.
constexpr size_t kScratchBytes = (size_t)48 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};  // device address of `scratch` per device

// Called with `device` current.  Returns the HIP error of the address query.
hipError_t take_scratch_address(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return hipSuccess;  // the call reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = ptr;
    return e;
}

void *scratch_address(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

int mis2_create(mis2_ctx **out, int device) {
    if (!out) return MIS2_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return MIS2_EINVAL;
    mis2_ctx *ctx = new mis2_ctx();
    ctx->device = device;
    ctx->seen.reserve(kSeenCap + 1);
    ctx->tuning.reserve(8);
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return MIS2_EHIP;
    }
    if (take_scratch_address(device) != hipSuccess) {
        delete ctx;
        return MIS2_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cus = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        ctx->wall_khz = (double)khz;
    // coherent: kernels write scalars into it directly
    if (hipHostMalloc((void **)&ctx->pinned, (64 + 2 * kTraceCap) * sizeof(uint32_t),
                      hipHostMallocCoherent) != hipSuccess) {
        delete ctx;
        return MIS2_EHIP;
    }
    if (hipHostMalloc((void **)&ctx->pinned_ctr, 2 * (size_t)kCtrList * sizeof(uint32_t),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(ctx->pinned);
        delete ctx;
        return MIS2_EHIP;
    }
    // coherent, so the host sees the GPU's stores while kernels still run
    if (hipHostMalloc((void **)&ctx->alive_host, 64, hipHostMallocCoherent) != hipSuccess) {
        (void)hipHostFree(ctx->pinned);
        (void)hipHostFree(ctx->pinned_ctr);
        delete ctx;
        return MIS2_EHIP;
    }
    // coherent: the round kernels write their rows into it directly
    if (hipHostMalloc((void **)&ctx->pinned_rt,
                      2 * (size_t)(kTraceCap + 2) * kRoundStride * sizeof(uint32_t),
                      hipHostMallocCoherent) != hipSuccess) {
        (void)hipHostFree(ctx->pinned);
        (void)hipHostFree(ctx->pinned_ctr);
        (void)hipHostFree(ctx->alive_host);
        delete ctx;
        return MIS2_EHIP;
    }
    *out = ctx;
    return MIS2_OK;
}

void mis2_destroy(mis2_ctx *ctx) {
    if (!ctx) return;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->pinned_ctr) (void)hipHostFree(ctx->pinned_ctr);
    if (ctx->alive_host) (void)hipHostFree(ctx->alive_host);
    if (ctx->pinned_rt) (void)hipHostFree(ctx->pinned_rt);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    delete ctx;
}

const char *mis2_last_error(const mis2_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

int mis2_set_option(mis2_ctx *ctx, int option, int64_t value) {
    if (!ctx) return MIS2_EINVAL;
    switch (option) {
        case MIS2_OPT_VALIDATE:
            ctx->validate = value != 0;
            return MIS2_OK;
        case MIS2_OPT_LANES_PER_ROW:
            if (value != 0 && value != -1 && value != MIS2_LANES_STAGED &&
                (value < 1 || value > 64 || (value & (value - 1))))
                return fail(ctx, MIS2_EINVAL,
                            "lanes per row must be 0, -1, -2 or a power of two <= 64");
            ctx->plan.lanes = value == MIS2_LANES_STAGED ? kStagedLanes : (int)value;
            return MIS2_OK;
        case MIS2_OPT_GRID_BLOCKS:
            if (value < 0 || value > kMaxBlocks)
                return fail(ctx, MIS2_EINVAL, "grid blocks must be in [0, %d]", kMaxBlocks);
            ctx->plan.blocks = (int)value;
            return MIS2_OK;
        case MIS2_OPT_PROFILE:
            ctx->profile = value != 0;
            return MIS2_OK;
        case MIS2_OPT_PERSISTENT:
            ctx->plan.persistent = value != 0;
            return MIS2_OK;
        case MIS2_OPT_ACCOUNT:
            ctx->account = value != 0;
            return MIS2_OK;
        case MIS2_OPT_COMPACT:
            ctx->plan.compact = value != 0;
            return MIS2_OK;
        case MIS2_OPT_AUTOTUNE:
            if (value < 0 || value > 2) return fail(ctx, MIS2_EINVAL, "autotune must be 0, 1 or 2");
            ctx->autotune = (int)value;
            return MIS2_OK;
        case MIS2_OPT_TAIL:
            if (value < -1 || value > 1) return fail(ctx, MIS2_EINVAL, "tail must be -1, 0 or 1");
            ctx->plan.tail = (int)value;
            return MIS2_OK;
        case MIS2_OPT_QUEUE_DEPTH:
            if (value < 0 || value > 8)
                return fail(ctx, MIS2_EINVAL, "queue depth must be in [0, 8]");
            ctx->plan.ahead = (int)value;
            return MIS2_OK;
        default:
            return fail(ctx, MIS2_EINVAL, "unknown option %d", option);
    }
}

int mis2_workspace_bytes(int64_t n, int op, size_t *bytes) {
    if (!bytes || n < 0 || op < MIS2_OP_MIS2 || op > MIS2_OP_COARSEN) return MIS2_EINVAL;
    *bytes = workspace_bytes(n, op);
    return MIS2_OK;
}

int mis2_workspace_bytes_csr(int64_t n, int64_t nnz, int op, size_t *bytes) {
    if (!bytes || n < 0 || nnz < 0 || op < MIS2_OP_MIS2 || op > MIS2_OP_COARSEN)
        return MIS2_EINVAL;
    *bytes = workspace_bytes(n, op) + compact_bytes(n, nnz);
    return MIS2_OK;
}

int mis2_set_workspace(mis2_ctx *ctx, void *dev_ptr, size_t bytes) {
    if (!ctx) return MIS2_EINVAL;
    if (dev_ptr && ((uintptr_t)dev_ptr % kAlign) != 0)
        return fail(ctx, MIS2_EINVAL, "workspace must be %zu-byte aligned", kAlign);
    ctx->ws = dev_ptr;
    ctx->ws_bytes = dev_ptr ? bytes : 0;
    return MIS2_OK;
}

int mis2_run(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, uint8_t *status, int64_t *n_roots,
             int32_t *n_iters, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (g->n > 0 && !status) return fail(ctx, MIS2_EINVAL, "status is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->trace[0].clear();
    ctx->trace[1].clear();
    ctx->sweeps.clear();
    if (g->n == 0) {
        if (n_roots) *n_roots = 0;
        if (n_iters) *n_iters = 0;
        return MIS2_OK;
    }
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_MIS2, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    PlanScope ps{ctx, g, ctx->plan};
    if ((rc = apply_plan(ctx, g, ws, s, &ps.saved))) return rc;
    ps.armed = true;

    ctx->events_used = 0;
    std::vector<Launch> launches;
    const Geometry gm = geometry(ctx, g->n, lanes_for(ctx, g));
    HIP_TRY(ctx, launch_init_tuples(tparams(ctx, g->n, seed, 0), g->n, ws.T,
                                    round_fills(g, ws, false), s));
    int32_t iters = 0;
    int long_rows = 0;
    if ((rc = run_rounds(ctx, g, seed, ws, gm, false, 0, s, &iters, &launches, &long_rows,
                         nullptr, true)))
        return rc;
    // the root count goes straight to the coherent host buffer (no copy)
    HIP_TRY(ctx, launch_status(g->n, ws.T, status, ws.blocksum, ctx->pinned, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    iters = parse_trace(ctx, 0);
    if (n_roots) *n_roots = __atomic_load_n(ctx->pinned, __ATOMIC_ACQUIRE);
    if (n_iters) *n_iters = iters;
    return collect_sweeps(ctx, launches, ws, s);
}

int mis2_run_noalloc_max_n(int64_t *max_n) {
    if (!max_n) return MIS2_EINVAL;
    int64_t lo = 0, hi = (int64_t)0x7FFFFFFE;
    while (lo < hi) {  // largest n whose MIS-2 workspace fits the scratch array
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (workspace_bytes(mid, MIS2_OP_MIS2) <= kScratchBytes) lo = mid; else hi = mid - 1;
    }
    *max_n = lo;
    return MIS2_OK;
}

int mis2_run_noalloc(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, uint8_t *status,
                     int64_t *n_roots, int32_t *n_iters, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (ctx->profile)
        return fail(ctx, MIS2_EINVAL, "mis2_run_noalloc: profiling creates events; switch "
                                      "MIS2_OPT_PROFILE off");
    const size_t need = workspace_bytes(g->n, MIS2_OP_MIS2);
    if (need > kScratchBytes) {
        int64_t max_n = 0;
        (void)mis2_run_noalloc_max_n(&max_n);
        return fail(ctx, MIS2_ENOSPACE,
                    "mis2_run_noalloc: n = %lld needs %zu bytes of workspace; the static scratch "
                    "holds %zu (n <= %lld)", (long long)g->n, need, kScratchBytes,
                    (long long)max_n);
    }
    void *ptr = scratch_address(ctx->device);
    if (!ptr)
        return fail(ctx, MIS2_EHIP, "mis2_run_noalloc: no scratch address for device %d",
                    ctx->device);
    // mis2_run with the scratch as the workspace; it writes every word it
    // later reads (counters, round table and flags are filled by its first
    // launch), so nothing from an earlier call leaks into this one
    void *const saved = ctx->ws;
    const size_t saved_bytes = ctx->ws_bytes;
    ctx->ws = ptr;
    ctx->ws_bytes = kScratchBytes;
    rc = mis2_run(ctx, g, seed, status, n_roots, n_iters, stream);
    ctx->ws = saved;
    ctx->ws_bytes = saved_bytes;
    return rc;
}

int mis2_ablation_workspace_bytes(int64_t n, int flags, size_t *bytes) {
    if (!bytes || n < 0 || (flags & ~MIS2_ABL_ALL_FLAGS)) return MIS2_EINVAL;
    *bytes = ablation_bytes(n, flags);
    return MIS2_OK;
}

int mis2_run_ablation(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int flags,
                      uint8_t *status, int64_t *n_roots, int32_t *n_iters, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (flags & ~MIS2_ABL_ALL_FLAGS) return fail(ctx, MIS2_EINVAL, "unknown ablation flags 0x%x", flags);
    if (!(flags & kAblFamily)) {
        // the production kernels, with one lane per row on request
        const int keep_lanes = ctx->plan.lanes;
        if (flags & MIS2_ABL_ONE_LANE) ctx->plan.lanes = 1;
        rc = mis2_run(ctx, g, seed, status, n_roots, n_iters, stream);
        ctx->plan.lanes = keep_lanes;
        return rc;
    }
    if (g->n > 0 && !status) return fail(ctx, MIS2_EINVAL, "status is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->trace[0].clear();
    ctx->trace[1].clear();
    ctx->sweeps.clear();
    if (g->n == 0) {
        if (n_roots) *n_roots = 0;
        if (n_iters) *n_iters = 0;
        return MIS2_OK;
    }
    const size_t need = ablation_bytes(g->n, flags);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "ablation workspace of %zu bytes needed, %zu set", need,
                    ctx->ws ? ctx->ws_bytes : (size_t)0);
    Workspace ws;
    if (!carve(ctx->ws, ctx->ws_bytes, g->n, MIS2_OP_MIS2, &ws))
        return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    AblRun abl;
    abl.unpacked = (flags & MIS2_ABL_UNPACKED) != 0;
    abl.all = (flags & MIS2_ABL_NO_WORKLISTS) != 0;
    abl.pflags = ((flags & MIS2_ABL_FIXED_PRIORITY) ? kAblFixed : 0) |
                 ((flags & MIS2_ABL_XORSHIFT) ? kAblXorshift : 0);
    abl.T.s = ws.T;
    abl.M.s = ws.M;
    if (abl.unpacked) {
        // three more arrays per tuple set, past the MIS-2 workspace
        char *tail = (char *)ctx->ws + workspace_bytes(g->n, MIS2_OP_MIS2);
        uint32_t *x[4];
        for (int k = 0; k < 4; k++) x[k] = (uint32_t *)(tail + (size_t)k * align_up(4 * (size_t)g->n));
        abl.T.p = x[0];
        abl.T.i = x[1];
        abl.M.p = x[2];
        abl.M.i = x[3];
    }
    ctx->events_used = 0;
    std::vector<Launch> launches;
    Geometry gm = geometry(ctx, g->n, 1);
    const int simple_flags = MIS2_ABL_FIXED_PRIORITY | MIS2_ABL_XORSHIFT | MIS2_ABL_NO_WORKLISTS |
                             MIS2_ABL_UNPACKED | MIS2_ABL_SIMPLE;
    if ((flags & simple_flags) && !ctx->plan.blocks) {
        // the simple kernels (one lane per row, a plain loop) hide latency with
        // threads: one workgroup per 320 vertices, a multiple of 8
        gm.blocks = (int)std::max<int64_t>(8, std::min<int64_t>(((g->n + 319) / 320 + 7) / 8 * 8,
                                                                kMaxBlocks));
        gm.S = (int64_t)gm.blocks * (kBlock / 64);
        gm.seg = std::max<int64_t>(1, (g->n + gm.S - 1) / gm.S);
    }
    RoundsArgs ia = round_args(ctx, g, seed, ws, gm, false, nullptr, 1);
    ia.abl = abl.pflags;
    HIP_TRY(ctx, launch_abl_init(abl.unpacked, abl.T, ia, s));
    int32_t iters = 0;
    int long_rows = 0;
    if ((rc = run_rounds(ctx, g, seed, ws, gm, false, 0, s, &iters, &launches, &long_rows, &abl)))
        return rc;
    // IN is 0 in the packed tuple and in the status field alike
    // the root count goes straight to the coherent host buffer (no copy)
    HIP_TRY(ctx, launch_status(g->n, ws.T, status, ws.blocksum, ctx->pinned, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    iters = parse_trace(ctx, 0);
    if (n_roots) *n_roots = __atomic_load_n(ctx->pinned, __ATOMIC_ACQUIRE);
    if (n_iters) *n_iters = iters;
    return collect_sweeps(ctx, launches, ws, s);
}

int mis2_last_trace(const mis2_ctx *ctx, int phase, int64_t *sizes, int32_t cap, int32_t *rounds) {
    if (!ctx || phase < 0 || phase > 1 || cap < 0 || (cap > 0 && !sizes)) return MIS2_EINVAL;
    const std::vector<int64_t> &tr = ctx->trace[phase];
    const int32_t r = (int32_t)(tr.size() / 2);
    for (int32_t i = 0; i < std::min(r, cap); i++) {
        sizes[2 * i] = tr[2 * i];
        sizes[2 * i + 1] = tr[2 * i + 1];
    }
    if (rounds) *rounds = r;
    return MIS2_OK;
}

int mis2_last_sweeps(const mis2_ctx *ctx, mis2_sweep_record *out, int32_t cap, int32_t *count) {
    if (!ctx || cap < 0 || (cap > 0 && !out)) return MIS2_EINVAL;
    const int32_t k = (int32_t)ctx->sweeps.size();
    for (int32_t i = 0; i < std::min(k, cap); i++) out[i] = ctx->sweeps[i];
    if (count) *count = k;
    return MIS2_OK;
}

int mis2_last_plan(const mis2_ctx *ctx, int32_t *lanes, int32_t *blocks, int32_t *tail,
                   int32_t *source) {
    if (!ctx) return MIS2_EINVAL;
    if (lanes) *lanes = ctx->last_lanes;
    if (blocks) *blocks = ctx->last_blocks;
    if (tail) *tail = ctx->last_tail;
    if (source) *source = ctx->last_source;
    return MIS2_OK;
}

int mis2_last_tuning(const mis2_ctx *ctx, mis2_tune_record *out, int32_t cap, int32_t *count) {
    if (!ctx || cap < 0 || (cap > 0 && !out)) return MIS2_EINVAL;
    const int32_t k = (int32_t)ctx->tuning.size();
    for (int32_t i = 0; i < std::min(k, cap); i++) out[i] = ctx->tuning[i];
    if (count) *count = k;
    return MIS2_OK;
}

}  // extern "C"

namespace {

// Algorithm 3 on a validated graph with n > 0 and a carved workspace.  In a
// batched run (ctx->batch set) P1 / P2 (device, [G + 1] each) receive the
// per-graph root bounds of phases 1 and 2 (see batch.hip) and agg_id holds
// union-wide aggregate ids.
// The first step of Algorithms 2 and 3: the MIS-2 of G, its roots listed in
// increasing id (ws.list, count in scalar kS_Count1, cleared scalars
// otherwise) and each root's closed neighbourhood labelled with the root's
// rank (ws.label, -1 elsewhere; ws.aggsize of each root); roots[v] = 1 for
// a root when roots is not null.
int phase1_labels(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, const Workspace &ws,
                  const Geometry &gm, hipStream_t s, uint8_t *roots, int32_t *iters,
                  std::vector<Launch> *launches, int *long_rows) {
    int rc;
    const int64_t n = g->n;
    uint32_t *sc = ws.scalars;
    HIP_TRY(ctx, launch_init_tuples(tparams(ctx, n, seed, 0), n, ws.T, round_fills(g, ws, false),
                                    s));
    if ((rc = run_rounds(ctx, g, seed, ws, gm, false, 0, s, iters, launches, long_rows, nullptr,
                         true)))
        return rc;
    // the roots, numbered by increasing id: the fills and per-tile root
    // counts in one launch, then the ordered scatter
    {
        FillSpans f;
        f.add(sc, 0u, kScalars);
        f.add((uint32_t *)ws.label, 0xFFFFFFFFu, n);  // -1
        HIP_TRY(ctx, count_in_with_fills(ws.T, n, f, roots, ws.blocksum, s));
    }
    HIP_TRY(ctx, scatter_counted_u32_eq(ws.T, kIn, n, ws.list, sc + kS_Count1, ws.blocksum, s));
    HIP_TRY(ctx, launch_label_roots(n, g->row_ptr, g->col, ws.list, sc + kS_Count1, nullptr, false,
                                    ws.label, ws.aggsize, roots, 1, s));
    return MIS2_OK;
}

// Algorithm 2: phase1_labels, then every vertex still unlabelled joins the
// smallest aggregate id among its neighbours' labels.
int aggregate_basic_impl(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                         int64_t *n_agg, uint8_t *roots, const Workspace &ws, hipStream_t s) {
    int rc;
    const int64_t n = g->n;
    uint32_t *sc = ws.scalars;
    PlanScope ps{ctx, g, ctx->plan};
    if ((rc = apply_plan(ctx, g, ws, s, &ps.saved))) return rc;
    ps.armed = true;
    ctx->events_used = 0;
    std::vector<Launch> launches;
    const int lanes = lanes_for(ctx, g);
    const Geometry gm = geometry(ctx, n, lanes);
    int32_t it = 0;
    int long_rows = 0;
    if ((rc = phase1_labels(ctx, g, seed, ws, gm, s, roots, &it, &launches, &long_rows))) return rc;
    SegIO left_io{};
    left_io.wl_out = ws.wl2[0];
    left_io.cnt_out = ws.cnt2[0];
    left_io.n = n;
    left_io.seg = gm.seg;
    left_io.S = gm.S;
    HIP_TRY(ctx, launch_list_unlabelled(gm.blocks, n, ws.label, agg_id, left_io, s));
    SegIO join_io{};
    join_io.wl_in = ws.wl2[0];
    join_io.cnt_in = ws.cnt2[0];
    join_io.n = n;
    join_io.seg = gm.seg;
    join_io.S = gm.S;
    HIP_TRY(ctx, launch_join_min(lanes > 0 ? group_lanes(lanes) : 4, gm.blocks, g->row_ptr, g->col, ws.label,
                                 join_io, agg_id, sc + kS_Err, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, sc, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    parse_trace(ctx, 0);
    if (ctx->pinned[kS_Err])
        return fail(ctx, MIS2_EINTERNAL, "a vertex without an aggregated neighbour");
    if (n_agg) *n_agg = (int64_t)ctx->pinned[kS_Count1];
    return collect_sweeps(ctx, launches, ws, s);
}

int aggregate_impl(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                   int64_t *n_agg, uint8_t *roots, const Workspace &ws, hipStream_t s,
                   uint32_t *P1 = nullptr, uint32_t *P2 = nullptr) {
    int rc;
    const int64_t n = g->n;
    uint32_t *sc = ws.scalars;
    PlanScope ps{ctx, g, ctx->plan};
    if ((rc = apply_plan(ctx, g, ws, s, &ps.saved))) return rc;
    ps.armed = true;
    ctx->events_used = 0;
    std::vector<Launch> launches;
    const Geometry gm = geometry(ctx, n, lanes_for(ctx, g));

    // Phase 1: MIS-2 of G; roots numbered by increasing id, each labelled with
    // its neighbours.
    int32_t it1 = 0, it2 = 0;
    int long_rows = 0;
    if ((rc = phase1_labels(ctx, g, seed, ws, gm, s, roots, &it1, &launches, &long_rows)))
        return rc;
    if (P1)
        HIP_TRY(ctx, launch_graph_bounds(ws.list, sc + kS_Count1, ctx->batch.voff, ctx->batch.G,
                                         P1, s));

    // Phase 2: MIS-2 of the subgraph induced by the unlabelled vertices (same
    // ids and b, round counter from 0); roots with >= 2 unlabelled neighbours
    // become aggregates n1 + k.
    // the active count goes to slot 0 of the size counters (round 0)
    HIP_TRY(ctx, launch_fill_u32(ws.ctr, 0u, kCtrSlot, s));
    SegIO act_io{};
    act_io.wl_out = ws.wl1[0];
    act_io.cnt_out = ws.cnt1[0];
    act_io.trace_out = ws.ctr;
    act_io.n = n;
    act_io.seg = gm.seg;
    act_io.S = gm.S;
    HIP_TRY(ctx, launch_init_masked(gm.blocks, tparams(ctx, n, seed, 0), n, ws.label, ws.T, ws.M,
                                    act_io, round_fills(g, ws, true), s));
    if ((rc = run_rounds(ctx, g, seed, ws, gm, true, 1, s, &it2, &launches, &long_rows, nullptr,
                         true)))
        return rc;
    // the accepted roots, numbered by increasing id: per-tile counts (plain
    // stores), then the ordered scatter
    HIP_TRY(ctx, launch_accept_phase2(n, g->row_ptr, g->col, ws.T, ws.label, ws.flag, s));
    HIP_TRY(ctx, count_u8_nz(ws.flag, n, ws.blocksum, s));
    HIP_TRY(ctx, scatter_counted_u8_nz(ws.flag, n, ws.list, sc + kS_Count2, ws.blocksum, s));
    HIP_TRY(ctx, launch_label_roots(n, g->row_ptr, g->col, ws.list, sc + kS_Count2,
                                    sc + kS_Count1, true, ws.label, ws.aggsize, roots, 2, s));
    if (P2)
        HIP_TRY(ctx, launch_graph_bounds(ws.list, sc + kS_Count2, ctx->batch.voff, ctx->batch.G,
                                         P2, s));

    // Phase 3: each unlabelled vertex joins its best-coupled aggregate, all
    // counted on the labels frozen after phase 2.
    SegIO left_io{};
    left_io.wl_out = ws.wl2[0];
    left_io.cnt_out = ws.cnt2[0];
    left_io.n = n;
    left_io.seg = gm.seg;
    left_io.S = gm.S;
    HIP_TRY(ctx, launch_list_unlabelled(gm.blocks, n, ws.label, agg_id, left_io, s));
    SegIO p3_io{};
    p3_io.wl_in = ws.wl2[0];
    p3_io.cnt_in = ws.cnt2[0];
    p3_io.wl_out = ws.wl1[1];  // long rows, for the second kernel
    p3_io.cnt_out = ws.cnt1[1];
    p3_io.n = n;
    p3_io.seg = gm.seg;
    p3_io.S = gm.S;
    SegIO long_io = p3_io;
    long_io.wl_in = ws.wl1[1];
    long_io.cnt_in = ws.cnt1[1];
    long_io.wl_out = nullptr;
    long_io.cnt_out = nullptr;
    // phase 3 keeps rows of up to 8 chunks of L entries in registers and
    // hands longer ones to a one-row-per-wavefront pass: 4 lanes at least,
    // or every 27-point row would be long (27-point 100^3 aggregation with
    // 1 lane: 1.7 ms, with 4: 0.78 ms)
    const int p3_lanes = std::max(4, group_lanes(lanes_for(ctx, g)));
    HIP_TRY(ctx, launch_phase3(p3_lanes, gm.blocks, g->row_ptr, g->col, ws.label,
                               ws.aggsize, p3_io, long_io, agg_id, sc + kS_Err, s));

    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, sc, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    it1 = parse_trace(ctx, 0);
    it2 = parse_trace(ctx, 1);
    if (ctx->pinned[kS_Err])
        return fail(ctx, MIS2_EINTERNAL, "phase-3 vertex without an aggregated neighbour");
    if (n_agg) *n_agg = (int64_t)ctx->pinned[kS_Count1] + (int64_t)ctx->pinned[kS_Count2];
    (void)it1;
    (void)it2;
    return collect_sweeps(ctx, launches, ws, s);
}

// Coarse graph of an aggregation into caller buffers; *nnz_out (host) gets
// the coarse nnz.
int quotient_impl(mis2_ctx *ctx, const mis2_graph *g, const int32_t *agg, int64_t n_agg,
                  int64_t *crow, int32_t *ccol, int64_t *nnz_out, const Workspace &ws,
                  hipStream_t s) {
    QuotientWs q{ws.q.cnt,   ws.q.moff,  ws.q.members, ws.q.part, ws.q.big,
                 ws.q.big_count, ws.q.gbits, ws.q.gmeta, ws.q.cls};
    HIP_TRY(ctx, quotient_graph(g->row_ptr, g->col, g->n, g->nnz, agg, n_agg, crow, ccol, q, s));
    int64_t nnz = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&ctx->pinned[0], crow + n_agg, sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    memcpy(&nnz, ctx->pinned, sizeof nnz);
    if (nnz_out) *nnz_out = nnz;
    return MIS2_OK;
}

size_t coarsen_bytes(int64_t n, int64_t nnz) {
    const size_t un = (size_t)n, unz = (size_t)nnz;
    return workspace_bytes(n, MIS2_OP_COARSEN) + 2 * (align_up(8 * (un + 1)) + align_up(4 * unz));
}

// mis2_cgs_setup: the coarsening workspace, then the colouring and ordering
// arrays (see the carve there).
size_t cgs_bytes(int64_t n, int64_t nnz) {
    const size_t un = (size_t)n;
    return coarsen_bytes(n, nnz) + 7 * align_up(4 * un) + align_up(8 * (un + 1)) +
           align_up(8 * (size_t)scan_parts(n)) + align_up(4 * (size_t)(compact_blocks(n) + 1)) +
           align_up(4 * (un + 1)) + align_up(4 * 64);
}

// Clears ctx->batch when a batched call returns.
struct BatchScope {
    mis2_ctx *ctx;
    ~BatchScope() { ctx->batch = BatchInfo{}; }
};

}  // namespace

namespace mis2 {

size_t batch_bytes(int32_t G, int64_t n, int64_t nnz) {
    const size_t ug = (size_t)G + 1;
    return coarsen_bytes(n, nnz) + 2 * align_up(4 * (size_t)n) + 3 * align_up(8 * ug) +
           3 * align_up(4 * ug) + 2 * align_up(ug);
}

BatchArena carve_batch_arena(void *base, int32_t G, int64_t n, int64_t nnz) {
    BatchArena a;
    a.head = workspace_bytes(n, MIS2_OP_COARSEN);
    char *p = (char *)base + a.head;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    for (int i = 0; i < 2; i++) {
        a.crow[i] = (int64_t *)take(8 * ((size_t)n + 1));
        a.ccol[i] = (int32_t *)take(4 * (size_t)nnz);
    }
    const size_t ug = (size_t)G + 1;
    a.map = (int32_t *)take(4 * (size_t)n);
    a.gid = (int32_t *)take(4 * (size_t)n);
    a.voff = (int64_t *)take(8 * ug);
    a.newoff = (int64_t *)take(8 * ug);
    a.bnd = (int64_t *)take(8 * ug);
    a.gb = (uint32_t *)take(4 * ug);
    a.P1 = (uint32_t *)take(4 * ug);
    a.P2 = (uint32_t *)take(4 * ug);
    a.cont = (uint8_t *)take(ug);
    a.live = (uint8_t *)take(ug);
    return a;
}

int batch_level(mis2_ctx *ctx, const mis2_graph &cur, uint64_t seed, int64_t stop_below,
                int32_t *agg_dst, const BatchArena &ar, int64_t *crow_next, int32_t *ccol_next,
                BatchLevel *bl, hipStream_t s) {
    int rc;
    const int32_t cg = (int32_t)bl->voff.size() - 1;
    std::vector<uint32_t> gb(cg);
    for (int32_t i = 0; i < cg; i++) gb[i] = (uint32_t)id_bits(bl->voff[i + 1] - bl->voff[i]);
    HIP_TRY(ctx, hipMemcpyAsync(ar.voff, bl->voff.data(), 8 * ((size_t)cg + 1),
                                hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ar.gb, gb.data(), 4 * (size_t)cg, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_gather_i64(cur.row_ptr, ar.voff, (int64_t)cg + 1, ar.bnd, s));
    BatchInfo bt;
    bt.voff = ar.voff;
    bt.gb = ar.gb;
    bt.G = cg;
    while ((int64_t{1} << bt.steps) < (int64_t)cg + 1) bt.steps++;
    HIP_TRY(ctx, launch_graph_ids(cur.n, bt, ar.gid, s));
    bt.gid = ar.gid;
    BatchScope scope{ctx};
    ctx->batch = bt;

    Workspace ws;
    if (!carve(ctx->ws, ar.head, cur.n, MIS2_OP_COARSEN, &ws))
        return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
    // the next level's graph buffers are idle until the quotient below
    ws.colc = ccol_next;
    ws.lenc = (int32_t *)crow_next;
    int64_t na_all = 0;
    if ((rc = aggregate_impl(ctx, &cur, seed, agg_dst, &na_all, nullptr, ws, s, ar.P1, ar.P2)))
        return rc;
    std::vector<uint32_t> P1(cg + 1), P2(cg + 1);
    std::vector<int64_t> bnd(cg + 1);
    HIP_TRY(ctx, hipMemcpyAsync(P1.data(), ar.P1, 4 * ((size_t)cg + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(P2.data(), ar.P2, 4 * ((size_t)cg + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(bnd.data(), ar.bnd, 8 * ((size_t)cg + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));

    bl->nagg.assign(cg, 0);
    bl->nnz.assign(cg, 0);
    bl->cont.assign(cg, 0);
    std::vector<int64_t> newoff(cg + 1, 0);
    bl->next_voff.assign(1, 0);
    for (int32_t i = 0; i < cg; i++) {
        const int64_t ni = bl->voff[i + 1] - bl->voff[i];
        const int64_t na = (int64_t)(P1[i + 1] - P1[i]) + (int64_t)(P2[i + 1] - P2[i]);
        bl->nagg[i] = na;
        bl->nnz[i] = bnd[i + 1] - bnd[i];
        bl->cont[i] = bl->live[i] && bl->allow[i] && na != ni && na > 0 && na >= stop_below;
        newoff[i + 1] = newoff[i] + (bl->cont[i] ? na : 0);
        if (bl->cont[i]) bl->next_voff.push_back(newoff[i + 1]);
    }
    const int64_t n_next = newoff[cg];
    HIP_TRY(ctx, hipMemcpyAsync(ar.cont, bl->cont.data(), (size_t)cg, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ar.live, bl->live.data(), (size_t)cg, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ar.newoff, newoff.data(), 8 * ((size_t)cg + 1),
                                hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_batch_local(cur.n, bt, ar.P1, ar.P2, agg_dst, ar.live, ar.cont, ar.newoff,
                                    n_next > 0 ? ar.map : nullptr, s));
    bl->n_next = n_next;
    bl->nnz_next = 0;
    if (n_next > 0) {
        QuotientWs q{ws.q.cnt,       ws.q.moff,  ws.q.members, ws.q.part, ws.q.big,
                     ws.q.big_count, ws.q.gbits, ws.q.gmeta,   ws.q.cls};
        HIP_TRY(ctx, quotient_graph(cur.row_ptr, cur.col, cur.n, cur.nnz, ar.map, n_next, crow_next,
                                    ccol_next, q, s));
        HIP_TRY(ctx, hipMemcpyAsync(&ctx->pinned[0], crow_next + n_next, sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (n_next > 0) memcpy(&bl->nnz_next, ctx->pinned, sizeof(int64_t));
    return MIS2_OK;
}

}  // namespace mis2

extern "C" {

int mis2_aggregate(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                   int64_t *n_agg, uint8_t *roots, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (g->n > 0 && !agg_id) return fail(ctx, MIS2_EINVAL, "agg_id is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->trace[0].clear();
    ctx->trace[1].clear();
    ctx->sweeps.clear();
    if (g->n == 0) {
        if (n_agg) *n_agg = 0;
        return MIS2_OK;
    }
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_AGGREGATE, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    return aggregate_impl(ctx, g, seed, agg_id, n_agg, roots, ws, s);
}

int mis2_aggregate_basic(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                         int64_t *n_agg, uint8_t *roots, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (g->n > 0 && !agg_id) return fail(ctx, MIS2_EINVAL, "agg_id is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->trace[0].clear();
    ctx->trace[1].clear();
    ctx->sweeps.clear();
    if (g->n == 0) {
        if (n_agg) *n_agg = 0;
        return MIS2_OK;
    }
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_AGGREGATE, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    return aggregate_basic_impl(ctx, g, seed, agg_id, n_agg, roots, ws, s);
}

int mis2_quotient(mis2_ctx *ctx, const mis2_graph *g, const int32_t *agg_id, int64_t n_agg,
                  int64_t *coarse_row_ptr, int32_t *coarse_col, int64_t *coarse_nnz,
                  void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (n_agg < 0 || n_agg > g->n) return fail(ctx, MIS2_EINVAL, "n_agg out of range");
    if (!coarse_row_ptr || (g->n > 0 && !agg_id) || (g->nnz > 0 && !coarse_col))
        return fail(ctx, MIS2_EINVAL, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_COARSEN, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    return quotient_impl(ctx, g, agg_id, n_agg, coarse_row_ptr, coarse_col, coarse_nnz, ws, s);
}

// mis2_galerkin: member counts, offsets, cursors and lists, scan partials
// and a flag word; at least what validating the fine graph needs.
static size_t galerkin_bytes(int64_t n, int64_t n_agg) {
    const size_t ua = (size_t)n_agg;
    const size_t own = 2 * align_up(4 * ua) + align_up(8 * (ua + 1)) + align_up(4 * (size_t)n) +
                       align_up(8 * (size_t)scan_parts(n_agg)) + align_up(256);
    return std::max(own, workspace_bytes(n, MIS2_OP_MIS2));
}

int mis2_galerkin_workspace_bytes(int64_t n, int64_t n_agg, size_t *bytes) {
    if (!bytes || n < 0 || n_agg < 0) return MIS2_EINVAL;
    *bytes = galerkin_bytes(n, n_agg);
    return MIS2_OK;
}

int mis2_galerkin(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                  const int32_t *agg, const mis2_graph *coarse, double *coarse_val,
                  double *coarse_diag, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if ((rc = check_graph_args(ctx, coarse))) return rc;
    const int64_t n = g->n, na = coarse->n;
    if (na > n || (n > 0 && na == 0)) return fail(ctx, MIS2_EINVAL, "coarse n out of range");
    if ((n > 0 && (!diag || !agg || !coarse_diag)) || (g->nnz > 0 && !val) ||
        (coarse->nnz > 0 && !coarse_val))
        return fail(ctx, MIS2_EINVAL, "null pointer");
    if (n == 0) return MIS2_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const size_t need = galerkin_bytes(n, na);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "Galerkin workspace of %zu bytes needed, %zu set", need,
                    ctx->ws ? ctx->ws_bytes : (size_t)0);
    char *p = (char *)ctx->ws;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    uint32_t *cnt = (uint32_t *)take(4 * (size_t)na);
    uint32_t *cursor = (uint32_t *)take(4 * (size_t)na);
    int64_t *moff = (int64_t *)take(8 * ((size_t)na + 1));
    int32_t *members = (int32_t *)take(4 * (size_t)n);
    unsigned long long *part = (unsigned long long *)take(8 * (size_t)scan_parts(na));
    uint32_t *flag = (uint32_t *)take(256);
    if (ctx->validate) {
        // both graphs, before the arrays below are filled (same memory)
        Workspace ws;
        if ((rc = get_workspace(ctx, g, MIS2_OP_MIS2, &ws))) return rc;
        if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
        if ((rc = get_workspace(ctx, coarse, MIS2_OP_MIS2, &ws))) return rc;
        if ((rc = maybe_validate(ctx, coarse, ws, s))) return rc;
    }
    // ids in range before anything indexes by them
    HIP_TRY(ctx, launch_fill_u32(flag, 0u, 1, s));
    HIP_TRY(ctx, launch_check_ids(n, agg, coarse->nnz, coarse->col, na, flag, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[0] & 1u) return fail(ctx, MIS2_EINVAL, "aggregate id outside [0, %lld)", (long long)na);
    if (ctx->pinned[0] & 2u) return fail(ctx, MIS2_EINVAL, "coarse column outside [0, %lld)", (long long)na);
    // members of each aggregate by increasing id
    HIP_TRY(ctx, launch_fill_u32(cnt, 0u, na, s));
    HIP_TRY(ctx, launch_count_of(n, agg, cnt, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(cnt, na, moff, part, s));
    HIP_TRY(ctx, launch_fill_u32(cursor, 0u, na, s));
    HIP_TRY(ctx, launch_sorted_members(n, agg, na, moff, cursor, members, s));
    HIP_TRY(ctx, launch_galerkin(g->row_ptr, g->col, val, diag, agg, na, moff, members,
                                 coarse->row_ptr, coarse->col, coarse_val, coarse_diag, flag,
                                 g->nnz, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[0] & 4u)
        return fail(ctx, MIS2_EINVAL, "the coarse graph lacks a coupling of the aggregation");
    return MIS2_OK;
}

// Smoothed aggregation (see smoothed.hip).  Workspace: a fixed part, then
// arrays sized by the entries of P and AP, known only as the call proceeds.
namespace {
struct SmoothedWs {
    uint8_t *cls;  // [max(n, n_agg)] rows left to the large-set structure pass
    uint32_t *size, *cnt, *cursor, *flag;
    unsigned long long *part;
    int64_t *apptr, *moff;
    int32_t *prow_of, *members, *apcol;
    double *apval;
};

size_t smoothed_bytes(int64_t n, int64_t n_agg, int64_t p_nnz, int64_t ap_nnz) {
    const size_t un = (size_t)std::max<int64_t>(n, 1), ua = (size_t)std::max<int64_t>(n_agg, 1);
    size_t b = align_up(std::max(un, ua));
    b += align_up(4 * ua) + align_up(4 * std::max(un, ua)) + align_up(4 * ua) + align_up(64);
    b += align_up(8 * (size_t)scan_parts(std::max<int64_t>(n, n_agg)));
    b += align_up(8 * (un + 1)) + align_up(8 * (ua + 1));
    b += 2 * align_up(4 * (size_t)std::max<int64_t>(p_nnz, 1));
    b += align_up(4 * (size_t)std::max<int64_t>(ap_nnz, 1)) +
         align_up(8 * (size_t)std::max<int64_t>(ap_nnz, 1));
    return b;
}

SmoothedWs carve_smoothed(void *base, int64_t n, int64_t n_agg, int64_t p_nnz, int64_t ap_nnz) {
    const size_t un = (size_t)std::max<int64_t>(n, 1), ua = (size_t)std::max<int64_t>(n_agg, 1);
    char *p = (char *)base;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    SmoothedWs w;
    w.cls = (uint8_t *)take(std::max(un, ua));
    w.size = (uint32_t *)take(4 * ua);
    w.cnt = (uint32_t *)take(4 * std::max(un, ua));
    w.cursor = (uint32_t *)take(4 * ua);
    w.flag = (uint32_t *)take(64);
    w.part = (unsigned long long *)take(8 * (size_t)scan_parts(std::max<int64_t>(n, n_agg)));
    w.apptr = (int64_t *)take(8 * (un + 1));
    w.moff = (int64_t *)take(8 * (ua + 1));
    w.prow_of = (int32_t *)take(4 * (size_t)std::max<int64_t>(p_nnz, 1));
    w.members = (int32_t *)take(4 * (size_t)std::max<int64_t>(p_nnz, 1));
    w.apcol = (int32_t *)take(4 * (size_t)std::max<int64_t>(ap_nnz, 1));
    w.apval = (double *)take(8 * (size_t)std::max<int64_t>(ap_nnz, 1));
    return w;
}

// *out = the int64 at device address src, and the error flags (one sync).
int read_total(mis2_ctx *ctx, const int64_t *src, const uint32_t *flag, int64_t *out,
               uint32_t *flags, hipStream_t s) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, src, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned + 2, flag, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    *out = (int64_t)((uint64_t)ctx->pinned[0] | ((uint64_t)ctx->pinned[1] << 32));
    *flags = ctx->pinned[2];
    return MIS2_OK;
}
}  // namespace

int mis2_smoothed(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                  const int32_t *agg, int64_t n_agg, double omega, int64_t *prow, int32_t *pcol,
                  double *pval, int64_t p_cap, int64_t *crow, int32_t *ccol, double *cval,
                  int64_t c_cap, int64_t *p_nnz, int64_t *c_nnz, size_t *ws_need, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (p_nnz) *p_nnz = -1;
    if (c_nnz) *c_nnz = -1;
    if (ws_need) *ws_need = 0;
    const int64_t n = g->n;
    if (n_agg < 0 || (n > 0 && n_agg < 1) || n_agg > n || !prow || !crow || !p_nnz || !c_nnz ||
        (n > 0 && (!diag || !agg)) || (g->nnz > 0 && !val) || !std::isfinite(omega))
        return fail(ctx, MIS2_EINVAL, "mis2_smoothed: bad arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (n == 0) {
        HIP_TRY(ctx, launch_fill_u64((unsigned long long *)prow, 0ull, 1, s));
        HIP_TRY(ctx, launch_fill_u64((unsigned long long *)crow, 0ull, 1, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        *p_nnz = *c_nnz = 0;
        return MIS2_OK;
    }
    size_t need = smoothed_bytes(n, n_agg, 0, 0);
    if (!ctx->ws || ctx->ws_bytes < need) {
        if (ws_need) *ws_need = need;
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: workspace of %zu bytes needed", need);
    }
    SmoothedWs w = carve_smoothed(ctx->ws, n, n_agg, 0, 0);
    uint32_t flags = 0;
    // aggregate ids in range (checked before any is used as an index), and
    // the aggregate sizes
    HIP_TRY(ctx, launch_fill_u32(w.flag, 0u, 16, s));
    HIP_TRY(ctx, launch_check_ids(n, agg, 0, nullptr, n_agg, w.flag, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, w.flag, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[0] & 1u)
        return fail(ctx, MIS2_EINVAL, "mis2_smoothed: aggregate id outside [0, n_agg)");
    HIP_TRY(ctx, launch_fill_u32(w.size, 0u, n_agg, s));
    HIP_TRY(ctx, launch_count_of(n, agg, w.size, s));
    // P: structure (count, offsets, columns), then values
    HIP_TRY(ctx, launch_smoothed_sym(0, false, n, g->row_ptr, g->col, agg, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, w.cnt, nullptr, nullptr,
                                     w.flag + 1, w.cls, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(w.cnt, n, prow, w.part, s));
    int64_t pn = 0;
    if ((rc = read_total(ctx, prow + n, w.flag + 1, &pn, &flags, s))) return rc;
    *p_nnz = pn;
    if (pn > (int64_t)0x7FFFFFFF)
        return fail(ctx, MIS2_EINVAL, "mis2_smoothed: P has more than 2^31 - 1 entries");
    if (pn > p_cap || (pn > 0 && (!pcol || !pval)))
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: P has %lld entries, room for %lld",
                    (long long)pn, (long long)p_cap);
    need = smoothed_bytes(n, n_agg, pn, 0);
    if (ctx->ws_bytes < need) {
        if (ws_need) *ws_need = need;
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: workspace of %zu bytes needed", need);
    }
    w = carve_smoothed(ctx->ws, n, n_agg, pn, 0);
    HIP_TRY(ctx, launch_smoothed_sym(0, true, n, g->row_ptr, g->col, agg, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, nullptr, prow, pcol, w.flag + 1, w.cls,
                                     s));
    HIP_TRY(ctx, launch_p_values(n, pn, g->row_ptr, g->col, val, diag, agg, w.size, omega, prow,
                                 pcol, pval, w.prow_of, s));
    // AP = A P
    HIP_TRY(ctx, launch_smoothed_sym(1, false, n, g->row_ptr, g->col, agg, prow, pcol, nullptr,
                                     nullptr, nullptr, w.cnt, nullptr, nullptr, w.flag + 1, w.cls, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(w.cnt, n, w.apptr, w.part, s));
    int64_t apn = 0;
    if ((rc = read_total(ctx, w.apptr + n, w.flag + 1, &apn, &flags, s))) return rc;
    if (flags & 1u)
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: a row of A P has more than 2048 columns");
    need = smoothed_bytes(n, n_agg, pn, apn);
    if (ctx->ws_bytes < need) {
        if (ws_need) *ws_need = need;
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: workspace of %zu bytes needed", need);
    }
    w = carve_smoothed(ctx->ws, n, n_agg, pn, apn);
    HIP_TRY(ctx, launch_smoothed_sym(1, true, n, g->row_ptr, g->col, agg, prow, pcol, nullptr,
                                     nullptr, nullptr, nullptr, w.apptr, w.apcol, w.flag + 1, w.cls, s));
    HIP_TRY(ctx, launch_ap_values(n, apn, g->row_ptr, g->col, val, diag, prow, pcol, pval,
                                  w.apptr, w.apcol, w.apval, s));
    // R_a: the P entries of column a in increasing order (hence increasing row)
    HIP_TRY(ctx, launch_fill_u32(w.cnt, 0u, n_agg, s));
    HIP_TRY(ctx, launch_count_of(pn, pcol, w.cnt, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(w.cnt, n_agg, w.moff, w.part, s));
    HIP_TRY(ctx, launch_fill_u32(w.cursor, 0u, n_agg, s));
    HIP_TRY(ctx, launch_sorted_members(pn, pcol, n_agg, w.moff, w.cursor, w.members, s));
    // Ac = P^T (A P)
    HIP_TRY(ctx, launch_smoothed_sym(2, false, n_agg, g->row_ptr, g->col, agg, w.apptr, w.apcol,
                                     w.moff, w.members, w.prow_of, w.cnt, nullptr, nullptr,
                                     w.flag + 1, w.cls, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(w.cnt, n_agg, crow, w.part, s));
    int64_t cn = 0;
    if ((rc = read_total(ctx, crow + n_agg, w.flag + 1, &cn, &flags, s))) return rc;
    if (flags & 1u)
        return fail(ctx, MIS2_ENOSPACE,
                    "mis2_smoothed: a row of the coarse operator has more than 2048 columns");
    *c_nnz = cn;
    if (cn > c_cap || (cn > 0 && (!ccol || !cval)))
        return fail(ctx, MIS2_ENOSPACE, "mis2_smoothed: the coarse operator has %lld entries, "
                    "room for %lld", (long long)cn, (long long)c_cap);
    HIP_TRY(ctx, launch_smoothed_sym(2, true, n_agg, g->row_ptr, g->col, agg, w.apptr, w.apcol,
                                     w.moff, w.members, w.prow_of, nullptr, crow, ccol,
                                     w.flag + 1, w.cls, s));
    HIP_TRY(ctx, launch_c_values(n_agg, cn, w.moff, w.members, w.prow_of, pval, w.apptr, w.apcol,
                                 w.apval, crow, ccol, cval, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return MIS2_OK;
}

int mis2_cgs_workspace_bytes(int64_t n, int64_t nnz, size_t *bytes) {
    if (!bytes || n < 0 || nnz < 0) return MIS2_EINVAL;
    *bytes = cgs_bytes(n, nnz);
    return MIS2_OK;
}

int mis2_cgs_setup(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int point,
                   mis2_cgs_plan *plan, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (!plan || plan->n != g->n || !plan->color_off ||
        (g->n > 0 && (!plan->cluster || !plan->cluster_color || !plan->rows || !plan->pos ||
                      !plan->cluster_off)))
        return fail(ctx, MIS2_EINVAL, "bad plan (arrays of n = graph's n entries)");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t n = g->n;
    plan->n_clusters = 0;
    plan->n_colors = 0;
    plan->color_off[0] = 0;
    if (n == 0) return MIS2_OK;
    const size_t need = cgs_bytes(n, g->nnz);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "cluster Gauss-Seidel workspace of %zu bytes needed, %zu set",
                    need, ctx->ws ? ctx->ws_bytes : (size_t)0);
    const size_t head = workspace_bytes(n, MIS2_OP_COARSEN);
    Workspace ws;
    if (!carve(ctx->ws, head, n, MIS2_OP_COARSEN, &ws))
        return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    char *p = (char *)ctx->ws + head;
    auto take = [&](size_t sz) {
        char *r = p;
        p += align_up(sz);
        return (void *)r;
    };
    int64_t *crow[2];
    int32_t *ccol[2];
    for (int i = 0; i < 2; i++) {
        crow[i] = (int64_t *)take(8 * ((size_t)n + 1));
        ccol[i] = (int32_t *)take(4 * (size_t)g->nnz);
    }
    const size_t un = (size_t)n;
    uint32_t *pr = (uint32_t *)take(4 * un);
    int32_t *cround = (int32_t *)take(4 * un);
    uint32_t *cnt = (uint32_t *)take(4 * un);
    int64_t *moff = (int64_t *)take(8 * (un + 1));
    uint32_t *cursor = (uint32_t *)take(4 * un);
    int32_t *members = (int32_t *)take(4 * un);
    int32_t *corder = (int32_t *)take(4 * un);
    uint32_t *ssz = (uint32_t *)take(4 * un);
    unsigned long long *part = (unsigned long long *)take(8 * (size_t)scan_parts(n));
    uint32_t *blocksum = (uint32_t *)take(4 * (size_t)(compact_blocks(n) + 1));
    uint32_t *hist = (uint32_t *)take(4 * (un + 1));
    uint32_t *scal = (uint32_t *)take(4 * 64);

    // clusters and the graph to colour
    mis2_graph cg = *g;
    int64_t nc = n;
    if (!point) {
        ws.colc = ccol[1];  // idle until the quotient, as in mis2_coarsen
        ws.lenc = (int32_t *)crow[1];
        if ((rc = aggregate_impl(ctx, g, seed, plan->cluster, &nc, nullptr, ws, s))) return rc;
        int64_t cnnz = 0;
        if ((rc = quotient_impl(ctx, g, plan->cluster, nc, crow[0], ccol[0], &cnnz, ws, s)))
            return rc;
        cg = mis2_graph{nc, cnnz, crow[0], ccol[0]};
    } else {
        HIP_TRY(ctx, launch_iota(n, plan->cluster, s));
    }
    // Jones-Plassmann colouring of cg; every round colours at least the
    // smallest uncoloured tuple, so at most nc rounds
    HIP_TRY(ctx, launch_jp_init(nc, tuple_params(nc, seed, 0), pr, cround, plan->cluster_color, s));
    HIP_TRY(ctx, launch_fill_u32(scal, 0u, 64, s));
    for (int r = 0;; r++) {
        if (r > nc) return fail(ctx, MIS2_EINTERNAL, "colouring made no progress");
        HIP_TRY(ctx, launch_fill_u32(scal, 0u, 1, s));
        HIP_TRY(ctx, launch_jp_round(nc, cg.row_ptr, cg.col, pr, cround, plan->cluster_color, r,
                                     scal, scal + 1, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, scal, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (ctx->pinned[0] == 0) break;
    }
    const int32_t n_colors = (int32_t)ctx->pinned[1] + 1;
    // rows of each cluster in increasing id
    HIP_TRY(ctx, launch_fill_u32(cnt, 0u, nc, s));
    HIP_TRY(ctx, launch_count_of(n, plan->cluster, cnt, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(cnt, nc, moff, part, s));
    HIP_TRY(ctx, launch_fill_u32(cursor, 0u, nc, s));
    HIP_TRY(ctx, launch_sorted_members(n, plan->cluster, nc, moff, cursor, members, s));
    // clusters by colour, then id
    std::vector<uint32_t> h((size_t)n_colors);
    HIP_TRY(ctx, launch_fill_u32(hist, 0u, n_colors, s));
    HIP_TRY(ctx, launch_color_hist(nc, plan->cluster_color, n_colors, hist, s));
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), hist, 4 * (size_t)n_colors, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    for (int32_t c = 0; c < n_colors; c++) plan->color_off[c + 1] = plan->color_off[c] + h[c];
    if (plan->color_off[n_colors] != nc)
        return fail(ctx, MIS2_EINTERNAL, "colour histogram does not add up");
    for (int32_t c = 0; c < n_colors; c++)
        HIP_TRY(ctx, compact_u32_eq((const uint32_t *)plan->cluster_color, (uint32_t)c, nc,
                                    corder + plan->color_off[c], scal + 2, blocksum, s));
    HIP_TRY(ctx, launch_gather_sizes(nc, corder, cnt, ssz, s));
    HIP_TRY(ctx, exclusive_scan_u32_i64(ssz, nc, plan->cluster_off, part, s));
    HIP_TRY(ctx, launch_place_rows(nc, corder, moff, members, plan->cluster_off, plan->rows, s));
    HIP_TRY(ctx, launch_scatter_pos(n, plan->rows, plan->pos, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    plan->n_clusters = nc;
    plan->n_colors = n_colors;
    return MIS2_OK;
}

int mis2_cgs_apply(mis2_ctx *ctx, const mis2_graph *g, const double *val, const double *diag,
                   const mis2_cgs_plan *plan, const double *b, double *x, int32_t sweeps,
                   int symmetric, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (!plan || plan->n != g->n || sweeps < 0 || plan->n_colors < 0 || !plan->color_off)
        return fail(ctx, MIS2_EINVAL, "bad plan or sweep count");
    if (g->n > 0 && (!diag || !b || !x || !plan->rows || !plan->pos || !plan->cluster_off ||
                     (g->nnz > 0 && !val)))
        return fail(ctx, MIS2_EINVAL, "null pointer");
    if (g->n > 0 && plan->color_off[plan->n_colors] != plan->n_clusters)
        return fail(ctx, MIS2_EINVAL, "plan's colour offsets do not cover its clusters");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t *co = plan->color_off;
    // every cluster a single row (cluster_off[k] == k): one lane per row
    const bool point = plan->n_clusters == g->n;
    auto pass = [&](int32_t c, bool backward) {
        return point ? launch_cgs_point(g->row_ptr, g->col, val, diag, b, x, plan->rows, co[c],
                                        co[c + 1], s)
                     : launch_cgs_sweep(g->row_ptr, g->col, val, diag, b, x, plan->rows, plan->pos,
                                        plan->cluster_off, co[c], co[c + 1], backward, s);
    };
    for (int32_t t = 0; t < sweeps; t++) {
        for (int32_t c = 0; c < plan->n_colors; c++) HIP_TRY(ctx, pass(c, false));
        if (!symmetric) continue;
        for (int32_t c = plan->n_colors - 1; c >= 0; c--) HIP_TRY(ctx, pass(c, true));
    }
    return MIS2_OK;
}

int mis2_coarsen_workspace_bytes(int64_t n, int64_t nnz, size_t *bytes) {
    if (!bytes || n < 0 || nnz < 0) return MIS2_EINVAL;
    *bytes = coarsen_bytes(n, nnz);
    return MIS2_OK;
}

int mis2_coarsen(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int64_t stop_below,
                 int32_t max_levels, int32_t *agg_out, int64_t agg_cap, int64_t *level_n,
                 int64_t *level_nnz, int64_t *level_nagg, int32_t *n_levels, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (max_levels < 0 || agg_cap < 0 || !n_levels ||
        (max_levels > 0 && (!level_n || !level_nnz || !level_nagg)))
        return fail(ctx, MIS2_EINVAL, "bad coarsening arguments");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    *n_levels = 0;
    const size_t need = coarsen_bytes(g->n, g->nnz);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "coarsening workspace of %zu bytes needed, %zu set", need,
                    ctx->ws ? ctx->ws_bytes : (size_t)0);
    const size_t head = workspace_bytes(g->n, MIS2_OP_COARSEN);
    char *tail = (char *)ctx->ws + head;
    int64_t *crow[2];
    int32_t *ccol[2];
    for (int i = 0; i < 2; i++) {
        crow[i] = (int64_t *)tail;
        tail += align_up(8 * ((size_t)g->n + 1));
        ccol[i] = (int32_t *)tail;
        tail += align_up(4 * (size_t)g->nnz);
    }
    mis2_graph cur = *g;
    {
        Workspace ws;
        if (!carve(ctx->ws, head, g->n, MIS2_OP_COARSEN, &ws))
            return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
        if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    }
    int64_t off = 0;
    int32_t lv = 0;
    while (lv < max_levels && cur.n >= stop_below && cur.n > 0) {
        if (off + cur.n > agg_cap)
            return fail(ctx, MIS2_ENOSPACE, "agg_cap %lld too small for level %d",
                        (long long)agg_cap, lv);
        Workspace ws;
        if (!carve(ctx->ws, head, cur.n, MIS2_OP_COARSEN, &ws))
            return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
        // the coarse-graph buffers the quotient of this level writes are idle
        // until then: they hold the compacted adjacency meanwhile
        ws.colc = ccol[(lv + 1) & 1];
        ws.lenc = (int32_t *)crow[(lv + 1) & 1];
        int64_t na = 0;
        if ((rc = aggregate_impl(ctx, &cur, seed, agg_out + off, &na, nullptr, ws, s))) return rc;
        level_n[lv] = cur.n;
        level_nnz[lv] = cur.nnz;
        level_nagg[lv] = na;
        lv++;
        *n_levels = lv;
        if (na == cur.n) break;  // no progress
        int64_t cnnz = 0;
        if ((rc = quotient_impl(ctx, &cur, agg_out + off, na, crow[lv & 1], ccol[lv & 1], &cnnz, ws,
                                s)))
            return rc;
        off += cur.n;
        cur.n = na;
        cur.nnz = cnnz;
        cur.row_ptr = crow[lv & 1];
        cur.col = ccol[lv & 1];
    }
    return MIS2_OK;
}

int mis2_batch_workspace_bytes(int32_t n_graphs, int64_t n, int64_t nnz, size_t *bytes) {
    if (!bytes || n_graphs < 0 || n < 0 || nnz < 0) return MIS2_EINVAL;
    *bytes = batch_bytes(n_graphs, n, nnz);
    return MIS2_OK;
}

int mis2_aggregate_batched(mis2_ctx *ctx, const mis2_graph *g, int32_t n_graphs,
                           const int64_t *vtx_off, uint64_t seed, int64_t stop_below,
                           int32_t max_levels, int32_t *agg_out, int64_t agg_cap,
                           int64_t *level_n, int64_t *level_nnz, int64_t *level_nagg,
                           int32_t *n_levels, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    const int32_t G = n_graphs;
    if (G < 0 || !vtx_off || max_levels < 0 || agg_cap < 0 || (G > 0 && !n_levels) ||
        (G > 0 && max_levels > 0 && (!level_n || !level_nnz || !level_nagg)))
        return fail(ctx, MIS2_EINVAL, "bad batched coarsening arguments");
    if (vtx_off[0] != 0 || vtx_off[G] != g->n)
        return fail(ctx, MIS2_EINVAL, "vtx_off must run from 0 to n");
    for (int32_t i = 0; i < G; i++)
        if (vtx_off[i + 1] < vtx_off[i]) return fail(ctx, MIS2_EINVAL, "vtx_off decreases at %d", i);
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (int32_t i = 0; i < G; i++) n_levels[i] = 0;
    for (int64_t i = 0; i < (int64_t)G * max_levels; i++) level_n[i] = level_nnz[i] = level_nagg[i] = 0;
    if (G == 0 || g->n == 0 || max_levels == 0) return MIS2_OK;
    const size_t need = batch_bytes(G, g->n, g->nnz);
    if (!ctx->ws || ctx->ws_bytes < need)
        return fail(ctx, MIS2_ENOSPACE, "batched workspace of %zu bytes needed, %zu set", need,
                    ctx->ws ? ctx->ws_bytes : (size_t)0);
    const BatchArena ar = carve_batch_arena(ctx->ws, G, g->n, g->nnz);
    {
        Workspace ws;
        if (!carve(ctx->ws, ar.head, g->n, MIS2_OP_COARSEN, &ws))
            return fail(ctx, MIS2_ENOSPACE, "workspace carve failed");
        if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    }

    // graphs of the current union: their ids in the call and vertex offsets
    BatchLevel bl;
    std::vector<int32_t> ids(G);
    bl.voff.assign(vtx_off, vtx_off + G + 1);
    bl.live.resize(G);
    bl.allow.resize(G);
    for (int32_t i = 0; i < G; i++) {
        ids[i] = i;
        const int64_t ni = bl.voff[i + 1] - bl.voff[i];
        bl.live[i] = ni > 0 && ni >= stop_below;
    }
    if (std::find(bl.live.begin(), bl.live.end(), 1) == bl.live.end()) return MIS2_OK;
    mis2_graph cur = *g;
    int64_t off = 0;
    for (int32_t lv = 0; lv < max_levels; lv++) {
        const int32_t cg = (int32_t)ids.size();
        if (off + cur.n > agg_cap)
            return fail(ctx, MIS2_ENOSPACE, "agg_cap %lld too small for level %d",
                        (long long)agg_cap, lv);
        for (int32_t i = 0; i < cg; i++) bl.allow[i] = lv + 1 < max_levels;
        const int nx = (lv + 1) & 1;
        if ((rc = batch_level(ctx, cur, seed, stop_below, agg_out + off, ar, ar.crow[nx],
                              ar.ccol[nx], &bl, s)))
            return rc;
        std::vector<int32_t> next_ids;
        for (int32_t i = 0; i < cg; i++) {
            if (bl.live[i]) {
                const int64_t k = (int64_t)lv * G + ids[i];
                level_n[k] = bl.voff[i + 1] - bl.voff[i];
                level_nnz[k] = bl.nnz[i];
                level_nagg[k] = bl.nagg[i];
                n_levels[ids[i]] = lv + 1;
            }
            if (bl.cont[i]) next_ids.push_back(ids[i]);
        }
        off += cur.n;
        if (next_ids.empty()) break;
        ids = next_ids;
        bl.voff = bl.next_voff;
        bl.live.assign(ids.size(), 1);
        bl.allow.resize(ids.size());
        cur.n = bl.n_next;
        cur.nnz = bl.nnz_next;
        cur.row_ptr = ar.crow[nx];
        cur.col = ar.ccol[nx];
    }
    return MIS2_OK;
}

}  // extern "C"
