// serve.hip -- continuous batching of coarsening jobs on one GPU.
//
// A server owns one device arena (caller-allocated) sized for a union of at
// most max_vertices vertices, max_nnz stored entries and max_graphs graphs.
// Jobs (multilevel coarsening of one CSR graph each, as mis2_coarsen) wait in
// a FIFO queue.  Every step:
//   1. admits queued jobs, in arrival order, while the union still fits the
//      arena (vertices, entries and graph slots): the job's CSR is copied to
//      the end of the union with its ids shifted;
//   2. runs one aggregation level (Algorithm 3) on the whole union -- graphs
//      at different levels side by side, since a level's result depends only
//      on that level's graph and the seed;
//   3. copies each graph's labels to its job's output, and keeps the coarse
//      graphs of the jobs that go on as the start of the next union.
// So a job that arrives while others are mid-way joins at the next level
// boundary instead of waiting for the whole batch to finish.
#include <string.h>

#include <deque>

#include "internal.h"

using namespace mis2;

namespace {

constexpr size_t kAlignS = 256;
size_t align_s(size_t x) { return (x + kAlignS - 1) / kAlignS * kAlignS; }

// Appends a CSR (row_ptr[0] = 0) at vertex offset voff / entry offset eoff of
// the union: dst_rp[voff + i] = src_rp[i] + eoff (i <= n) and
// dst_col[eoff + j] = src_col[j] + voff (j < nnz).
__global__ __launch_bounds__(kBlock) void k_append_csr(const int64_t *__restrict__ src_rp,
                                                       const int32_t *__restrict__ src_col,
                                                       int64_t n, int64_t nnz, int64_t voff,
                                                       int64_t eoff, int64_t *__restrict__ dst_rp,
                                                       int32_t *__restrict__ dst_col) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n; i += stride)
        dst_rp[voff + i] = src_rp[i] + eoff;
    for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < nnz; j += stride)
        dst_col[eoff + j] = src_col[j] + (int32_t)voff;
}

struct Job {
    mis2_job_result res;
    mis2_graph g;        // the caller's level-0 CSR
    int32_t *agg_out;    // the caller's label array
    int64_t agg_cap;
    int64_t agg_off = 0; // where the next level's labels go
};

}  // namespace

struct mis2_server {
    mis2_ctx *ctx = nullptr;
    BatchArena ar;
    int32_t *agg_scratch = nullptr;  // [max_vertices] union labels of one step
    int64_t vcap = 0, ecap = 0;
    int32_t gcap = 0;
    uint64_t seed = 0;
    int64_t stop_below = 0;
    int32_t max_levels = 0;
    int cur = 0;                       // union buffer of the next step
    std::vector<Job> jobs;             // every submitted job, by submission index
    std::deque<int32_t> queue;         // submitted, not admitted
    std::vector<int32_t> active;       // jobs in the union, in union order
    std::vector<int64_t> voff{0};      // their vertex offsets
    int64_t n_u = 0, nnz_u = 0;        // union size
    std::deque<int32_t> done;          // finished, not yet polled
    std::string err;
};

namespace {

size_t server_bytes(int64_t v, int64_t e, int32_t g) {
    return batch_bytes(g, v, e) + align_s(4 * (size_t)v);
}

int sfail(mis2_server *s, int code, const char *msg) {
    s->err = msg;
    return code;
}

}  // namespace

extern "C" {

int mis2_server_bytes(int64_t max_vertices, int64_t max_nnz, int32_t max_graphs, size_t *bytes) {
    if (!bytes || max_vertices <= 0 || max_nnz < 0 || max_graphs <= 0) return MIS2_EINVAL;
    *bytes = server_bytes(max_vertices, max_nnz, max_graphs);
    return MIS2_OK;
}

int mis2_server_create(mis2_server **out, int device, void *arena, size_t arena_bytes,
                       int64_t max_vertices, int64_t max_nnz, int32_t max_graphs, uint64_t seed,
                       int64_t stop_below, int32_t max_levels) {
    if (!out) return MIS2_EINVAL;
    *out = nullptr;
    if (!arena || max_vertices <= 0 || max_vertices > INT32_MAX - 2 || max_nnz < 0 ||
        max_graphs <= 0 || max_levels < 1 || max_levels > MIS2_SERVE_MAX_LEVELS ||
        ((uintptr_t)arena % kAlignS) != 0 ||
        arena_bytes < server_bytes(max_vertices, max_nnz, max_graphs))
        return MIS2_EINVAL;
    mis2_server *s = new mis2_server();
    int rc = mis2_create(&s->ctx, device);
    if (rc) {
        delete s;
        return rc;
    }
    // unions change from step to step: tuned plans are looked up, never timed
    if ((rc = mis2_set_option(s->ctx, MIS2_OPT_AUTOTUNE, 2))) {
        mis2_destroy(s->ctx);
        delete s;
        return rc;
    }
    if ((rc = mis2_set_workspace(s->ctx, arena, arena_bytes))) {
        mis2_destroy(s->ctx);
        delete s;
        return rc;
    }
    s->ar = carve_batch_arena(arena, max_graphs, max_vertices, max_nnz);
    s->agg_scratch = (int32_t *)((char *)arena + batch_bytes(max_graphs, max_vertices, max_nnz));
    s->vcap = max_vertices;
    s->ecap = max_nnz;
    s->gcap = max_graphs;
    s->seed = seed;
    s->stop_below = stop_below;
    s->max_levels = max_levels;
    *out = s;
    return MIS2_OK;
}

void mis2_server_destroy(mis2_server *s) {
    if (!s) return;
    mis2_destroy(s->ctx);
    delete s;
}

const char *mis2_server_last_error(const mis2_server *s) {
    if (!s) return "null server";
    if (!s->err.empty()) return s->err.c_str();
    return mis2_last_error(s->ctx);
}

int mis2_server_submit(mis2_server *s, const mis2_graph *g, int32_t *agg_out, int64_t agg_cap,
                       int64_t tag) {
    if (!s) return MIS2_EINVAL;
    s->err.clear();
    if (!g || g->n < 0 || g->nnz < 0 || (g->n > 0 && !g->row_ptr) || (g->nnz > 0 && !g->col))
        return sfail(s, MIS2_EINVAL, "bad graph");
    if (g->n > s->vcap || g->nnz > s->ecap)
        return sfail(s, MIS2_ENOSPACE, "job larger than the server's union capacity");
    if (agg_cap < g->n || (g->n > 0 && !agg_out))
        return sfail(s, MIS2_EINVAL, "agg_out must hold at least n labels");
    Job j;
    memset(&j.res, 0, sizeof j.res);
    j.res.tag = tag;
    j.g = *g;
    j.agg_out = agg_out;
    j.agg_cap = agg_cap;
    const int32_t id = (int32_t)s->jobs.size();
    s->jobs.push_back(j);
    if (g->n == 0 || g->n < s->stop_below)
        s->done.push_back(id);  // no level, as mis2_coarsen
    else
        s->queue.push_back(id);
    return MIS2_OK;
}

int mis2_server_step(mis2_server *s, void *stream, int32_t *n_pending) {
    if (!s) return MIS2_EINVAL;
    s->err.clear();
    hipStream_t st = (hipStream_t)stream;
    mis2_ctx *ctx = s->ctx;
    if (hipSetDevice(ctx->device) != hipSuccess) return sfail(s, MIS2_EHIP, "hipSetDevice failed");
    int64_t *rp = s->ar.crow[s->cur];
    int32_t *cl = s->ar.ccol[s->cur];
    // 1. admission, first come first served
    while (!s->queue.empty()) {
        Job &j = s->jobs[s->queue.front()];
        if (s->n_u + j.g.n > s->vcap || s->nnz_u + j.g.nnz > s->ecap ||
            (int32_t)s->active.size() >= s->gcap)
            break;
        int64_t blocks = (std::max(j.g.n + 1, j.g.nnz) + kBlock - 1) / kBlock;
        blocks = std::max<int64_t>(1, std::min<int64_t>(blocks, 8192));
        hipLaunchKernelGGL(k_append_csr, dim3((unsigned)blocks), dim3(kBlock), 0, st, j.g.row_ptr,
                           j.g.col, j.g.n, j.g.nnz, s->n_u, s->nnz_u, rp, cl);
        if (hipGetLastError() != hipSuccess) return sfail(s, MIS2_EHIP, "append launch failed");
        s->active.push_back(s->queue.front());
        s->queue.pop_front();
        s->n_u += j.g.n;
        s->nnz_u += j.g.nnz;
        s->voff.push_back(s->n_u);
    }
    if (s->active.empty()) {
        if (n_pending) *n_pending = (int32_t)s->queue.size();
        return MIS2_OK;
    }
    // 2. one level of every graph in the union
    const int32_t cg = (int32_t)s->active.size();
    BatchLevel bl;
    bl.voff = s->voff;
    bl.live.assign(cg, 1);
    bl.allow.resize(cg);
    std::vector<uint8_t> room(cg);
    for (int32_t i = 0; i < cg; i++) {
        const Job &j = s->jobs[s->active[i]];
        const int64_t ni = s->voff[i + 1] - s->voff[i];
        // another level needs room for up to ni more labels
        room[i] = j.agg_off + 2 * ni <= j.agg_cap;
        bl.allow[i] = j.res.n_levels + 1 < s->max_levels && room[i];
    }
    mis2_graph cur{s->n_u, s->nnz_u, rp, cl};
    const int nx = s->cur ^ 1;
    int rc = batch_level(ctx, cur, s->seed, s->stop_below, s->agg_scratch, s->ar, s->ar.crow[nx],
                         s->ar.ccol[nx], &bl, st);
    if (rc) return rc;
    // 3. labels out, finished jobs off, coarse graphs on
    std::vector<int32_t> next;
    for (int32_t i = 0; i < cg; i++) {
        Job &j = s->jobs[s->active[i]];
        const int64_t ni = s->voff[i + 1] - s->voff[i];
        if (hipMemcpyAsync(j.agg_out + j.agg_off, s->agg_scratch + s->voff[i], 4 * (size_t)ni,
                           hipMemcpyDeviceToDevice, st) != hipSuccess)
            return sfail(s, MIS2_EHIP, "label copy failed");
        const int l = j.res.n_levels;
        j.res.level_n[l] = ni;
        j.res.level_nnz[l] = bl.nnz[i];
        j.res.level_nagg[l] = bl.nagg[i];
        j.res.n_levels = l + 1;
        j.agg_off += ni;
        if (bl.cont[i]) {
            next.push_back(s->active[i]);
        } else {
            // stopped only for want of room in agg_out
            j.res.truncated = !room[i] && l + 1 < s->max_levels && bl.nagg[i] != ni &&
                              bl.nagg[i] > 0 && bl.nagg[i] >= s->stop_below;
            s->done.push_back(s->active[i]);
        }
    }
    if (hipStreamSynchronize(st) != hipSuccess) return sfail(s, MIS2_EHIP, "stream sync failed");
    s->active = next;
    s->voff = bl.next_voff;
    s->n_u = bl.n_next;
    s->nnz_u = bl.nnz_next;
    s->cur = nx;
    if (n_pending) *n_pending = (int32_t)(s->queue.size() + s->active.size());
    return MIS2_OK;
}

int mis2_server_poll(mis2_server *s, mis2_job_result *out, int32_t cap, int32_t *count) {
    if (!s || cap < 0 || (cap > 0 && !out) || !count) return MIS2_EINVAL;
    int32_t k = 0;
    while (k < cap && !s->done.empty()) {
        out[k++] = s->jobs[s->done.front()].res;
        s->done.pop_front();
    }
    *count = k;
    return MIS2_OK;
}

}  // extern "C"
