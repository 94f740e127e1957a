// abi.hip -- the C ABI declared in include/mis2.h: contexts, workspace, and the
// host side of Algorithm 1 (MIS-2) and Algorithm 3 (aggregation).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>

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

int lanes_for(const mis2_ctx *ctx, const mis2_graph *g) {
    if (ctx->plan.lanes) return ctx->plan.lanes;
    // Section V-D: one thread per row below an average degree of 16, lanes
    // cooperating on a row above it; here the group grows with the degree.
    const double avg = g->n > 0 ? (double)g->nnz / (double)g->n : 0.0;
    if (avg < 4) return 1;
    if (avg < 8) return 4;
    if (avg < 16) return 8;
    if (avg < 32) return 16;
    if (avg < 64) return 32;
    return 64;
}

int blocks_for(const mis2_ctx *ctx, int64_t rows, int lanes) {
    if (ctx->plan.blocks) return ctx->plan.blocks;
    const int64_t per = kBlock / lanes;
    int64_t b = (rows + per - 1) / per;
    const int64_t cap = (int64_t)ctx->num_cus * 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
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
    return MIS2_OK;
}

// The round loop of Algorithm 1.  Round 0 starts either from the identity
// worklists (whole graph) or from a list of the active vertices whose size
// is *d_active (induced subgraph; T and M already initialised).  Rounds are
// issued one at a time; after each, both worklist sizes are read back.
int run_rounds(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, const Workspace &ws,
               const int32_t *active_list, const uint32_t *d_active, int phase, hipStream_t s,
               int32_t *iters_out) {
    const int lanes = lanes_for(ctx, g);
    std::vector<int64_t> &tr = ctx->trace[phase];
    tr.clear();
    int64_t c1 = g->n, c2 = g->n;  // upper bounds for round 0
    if (d_active) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, d_active, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        c1 = c2 = ctx->pinned[0];
    }
    int round = 0;
    while (c1 > 0) {
        tr.push_back(c1);
        tr.push_back(c2);
        const int cur = round & 1, nxt = cur ^ 1;
        const bool first = (round == 0);
        const uint32_t *in1 = first ? d_active : ws.ring + 0 * kRing + round % kRing;
        const uint32_t *in2 = first ? d_active : ws.ring + 1 * kRing + round % kRing;
        SweepIO col_io{first ? active_list : ws.wl2[cur],
                       in2,
                       g->n,
                       ws.wl2[nxt],
                       ws.ring + 1 * kRing + (round + 1) % kRing,
                       ws.ring + 1 * kRing + (round + 2) % kRing,
                       round < kTraceCap ? ws.trace + 2 * round + 1 : nullptr};
        SweepIO dec_io{first ? active_list : ws.wl1[cur],
                       in1,
                       g->n,
                       ws.wl1[nxt],
                       ws.ring + 0 * kRing + (round + 1) % kRing,
                       ws.ring + 0 * kRing + (round + 2) % kRing,
                       round < kTraceCap ? ws.trace + 2 * round + 0 : nullptr};
        HIP_TRY(ctx, launch_refresh_column(lanes, blocks_for(ctx, c2, lanes), g->row_ptr, g->col,
                                           ws.T, ws.M, col_io, s));
        const TupleParams next = tuple_params(g->n, seed, (uint64_t)round + 1);
        HIP_TRY(ctx, launch_decide(lanes, blocks_for(ctx, c1, lanes), g->row_ptr, g->col, ws.T,
                                   ws.M, next, dec_io, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, ws.ring + 0 * kRing + (round + 1) % kRing, 4,
                                    hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned + 1, ws.ring + 1 * kRing + (round + 1) % kRing, 4,
                                    hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        c1 = ctx->pinned[0];
        c2 = ctx->pinned[1];
        round++;
        if (c1 > 0 && round >= (1 << 30))
            return fail(ctx, MIS2_EINTERNAL, "round counter overflow");
    }
    *iters_out = round;
    return MIS2_OK;
}

}  // namespace

namespace mis2 {

size_t workspace_bytes(int64_t n, int op) {
    if (n < 0) return 0;
    const size_t un = (size_t)n;
    size_t b = 0;
    b += align_up(4 * un) * 2;                 // T, M
    b += align_up(4 * un) * 4;                 // wl1[2], wl2[2]
    b += align_up(4 * 2 * kRing);              // ring
    b += align_up(4 * 2 * kTraceCap);          // trace
    b += align_up(4 * kScalars);               // scalars
    if (op != MIS2_OP_MIS2) {
        b += align_up(4 * un) * 3;             // label, list, aggsize
        b += align_up(un);                     // flag
        b += align_up(4 * (size_t)(compact_blocks(n) + 1));  // blocksum
        b += align_up(4 * un);                 // active
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
    ws->wl1[0] = (int32_t *)take(4 * un);
    ws->wl1[1] = (int32_t *)take(4 * un);
    ws->wl2[0] = (int32_t *)take(4 * un);
    ws->wl2[1] = (int32_t *)take(4 * un);
    ws->ring = (uint32_t *)take(4 * 2 * kRing);
    ws->trace = (uint32_t *)take(4 * 2 * kTraceCap);
    ws->scalars = (uint32_t *)take(4 * kScalars);
    if (op != MIS2_OP_MIS2) {
        ws->label = (int32_t *)take(4 * un);
        ws->list = (int32_t *)take(4 * un);
        ws->aggsize = (int32_t *)take(4 * un);
        ws->flag = (uint8_t *)take(un);
        ws->blocksum = (uint32_t *)take(4 * (size_t)(compact_blocks(n) + 1));
        ws->active = (int32_t *)take(4 * un);
    }
    return true;
}

}  // namespace mis2

extern "C" {

int mis2_create(mis2_ctx **out, int device) {
    if (!out) return MIS2_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return MIS2_EINVAL;
    mis2_ctx *ctx = new mis2_ctx();
    ctx->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return MIS2_EHIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->num_cus = prop.multiProcessorCount;
    if (hipHostMalloc((void **)&ctx->pinned, 64 * sizeof(uint32_t), hipHostMallocDefault) !=
        hipSuccess) {
        delete ctx;
        return MIS2_EHIP;
    }
    *out = ctx;
    return MIS2_OK;
}

void mis2_destroy(mis2_ctx *ctx) {
    if (!ctx) return;
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
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
            if (value != 0 && (value < 1 || value > 64 || (value & (value - 1))))
                return fail(ctx, MIS2_EINVAL, "lanes per row must be 0 or a power of two <= 64");
            ctx->plan.lanes = (int)value;
            return MIS2_OK;
        case MIS2_OPT_GRID_BLOCKS:
            if (value < 0 || value > (1 << 20))
                return fail(ctx, MIS2_EINVAL, "grid blocks out of range");
            ctx->plan.blocks = (int)value;
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
    if (g->n == 0) {
        if (n_roots) *n_roots = 0;
        if (n_iters) *n_iters = 0;
        return MIS2_OK;
    }
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_MIS2, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;

    HIP_TRY(ctx, launch_init_tuples(tuple_params(g->n, seed, 0), g->n, ws.T, ws.ring, s));
    int32_t iters = 0;
    if ((rc = run_rounds(ctx, g, seed, ws, nullptr, nullptr, 0, s, &iters))) return rc;
    HIP_TRY(ctx, launch_fill_u32(ws.scalars + kS_Roots, 0u, 1, s));
    HIP_TRY(ctx, launch_status(g->n, ws.T, status, ws.scalars + kS_Roots, s));
    if (n_roots) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, ws.scalars + kS_Roots, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        *n_roots = ctx->pinned[0];
    }
    if (n_iters) *n_iters = iters;
    return MIS2_OK;
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

int mis2_aggregate(mis2_ctx *ctx, const mis2_graph *g, uint64_t seed, int32_t *agg_id,
                   int64_t *n_agg, uint8_t *roots, void *stream) {
    int rc = check_graph_args(ctx, g);
    if (rc) return rc;
    if (g->n > 0 && !agg_id) return fail(ctx, MIS2_EINVAL, "agg_id is NULL");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    ctx->trace[0].clear();
    ctx->trace[1].clear();
    if (g->n == 0) {
        if (n_agg) *n_agg = 0;
        return MIS2_OK;
    }
    Workspace ws;
    if ((rc = get_workspace(ctx, g, MIS2_OP_AGGREGATE, &ws))) return rc;
    if ((rc = maybe_validate(ctx, g, ws, s))) return rc;
    const int64_t n = g->n;
    uint32_t *sc = ws.scalars;

    // Phase 1: MIS-2 of G; roots numbered by increasing id, each labelled with
    // its neighbours.
    HIP_TRY(ctx, launch_init_tuples(tuple_params(n, seed, 0), n, ws.T, ws.ring, s));
    int32_t it1 = 0, it2 = 0;
    if ((rc = run_rounds(ctx, g, seed, ws, nullptr, nullptr, 0, s, &it1))) return rc;
    HIP_TRY(ctx, launch_fill_u32(sc, 0u, kScalars, s));
    HIP_TRY(ctx, launch_fill_i32(ws.label, -1, n, s));
    if (roots) HIP_TRY(ctx, launch_fill_u8(roots, 0, n, s));
    HIP_TRY(ctx, compact_u32_eq(ws.T, kIn, n, ws.list, sc + kS_Count1, ws.blocksum, s));
    HIP_TRY(ctx, launch_label_roots(n, g->row_ptr, g->col, ws.list, sc + kS_Count1, nullptr, false,
                                    ws.label, roots, 1, s));

    // Phase 2: MIS-2 of the subgraph induced by the unlabelled vertices (same
    // ids and b, round counter from 0); roots with >= 2 unlabelled neighbours
    // become aggregates n1 + k.
    HIP_TRY(ctx, launch_init_masked(tuple_params(n, seed, 0), n, ws.label, ws.T, ws.M, ws.ring, s));
    HIP_TRY(ctx, compact_i32_eq(ws.label, -1, n, ws.active,
                                sc + kS_Active, ws.blocksum, s));
    if ((rc = run_rounds(ctx, g, seed, ws, ws.active, sc + kS_Active, 1, s, &it2))) return rc;
    HIP_TRY(ctx, launch_accept_phase2(n, g->row_ptr, g->col, ws.T, ws.label, ws.flag, s));
    HIP_TRY(ctx, compact_u8_nz(ws.flag, n, ws.list, sc + kS_Count2, ws.blocksum, s));
    HIP_TRY(ctx, launch_label_roots(n, g->row_ptr, g->col, ws.list, sc + kS_Count2,
                                    sc + kS_Count1, true, ws.label, roots, 2, s));

    // Phase 3: aggsize over the frozen labels, then each unlabelled vertex
    // joins its best-coupled aggregate.
    HIP_TRY(ctx, launch_fill_i32(ws.aggsize, 0, n, s));
    HIP_TRY(ctx, launch_aggsize(n, ws.label, ws.aggsize, s));
    HIP_TRY(ctx, launch_copy_i32(ws.label, agg_id, n, s));
    HIP_TRY(ctx, compact_i32_eq(ws.label, -1, n, ws.list, sc + kS_Left, ws.blocksum, s));
    HIP_TRY(ctx, launch_phase3(n, g->row_ptr, g->col, ws.label, ws.aggsize, ws.list, sc + kS_Left,
                               agg_id, sc + kS_Err, s));

    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, sc, 8 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->pinned[kS_Err])
        return fail(ctx, MIS2_EINTERNAL, "phase-3 vertex without an aggregated neighbour");
    if (n_agg) *n_agg = (int64_t)ctx->pinned[kS_Count1] + (int64_t)ctx->pinned[kS_Count2];
    (void)it1;
    (void)it2;
    return MIS2_OK;
}

}  // extern "C"
