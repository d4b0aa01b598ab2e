// Batched C-AMS: many independent problems of different sizes advanced by
// one Newton iteration together.  The setup of each instance (basis,
// assembly, coarse operator and its inverse, smoother pivots) is enqueued on
// a few side streams so that the instances' small kernels overlap; the
// C-AMS iterations then run as ONE launch per kernel for all instances: a
// work list names (instance, block) for every workgroup, so each launch
// covers the concatenated cells of the whole batch, and instances that have
// converged drop out (their workgroups return at once).  A fixed number of
// iterations is captured once into a HIP graph and replayed until every
// instance has stopped; the host reads one counter between replays.
//
// The graph is tuned per batch: on the first call every candidate number of
// iterations per graph runs the same first iterations from the same state,
// timed with events, and the state is reset before the real solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cams_internal.h"

using namespace cams;

namespace {

constexpr int kSide = 4;                     // setup streams (the device has 4 hardware queues per process)
constexpr int kGraphIters[] = {2, 4, 8};     // candidates of the tuner (even: the ping-pong parity repeats)
constexpr int kNumCand = 3;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Host form of the device XCD mapping: dispatch id -> logical id such that
// each of the 8 XCDs (which receive dispatch ids round-robin) takes one
// contiguous range of logical work items.
int xcd_swizzle_host(int wg, int n)
{
    const int q = n / 8, rem = n % 8;
    const int xcd = wg % 8, slot = wg / 8;
    return xcd < rem ? xcd * (q + 1) + slot : rem * (q + 1) + (xcd - rem) * q + slot;
}

enum { L_FLAT = 0, L_SBLOCK, L_RESTRICT, L_NODES, L_ROWS, L_NUM };

}  // namespace

struct cams_batch {
    std::vector<cams_ctx *> ctx;
    hipStream_t user = nullptr;      // the contexts' stream: ordered before and after each call
    hipStream_t stream = nullptr;    // batched launches and graph replays (created, capturable)
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {}, ev[4] = {};
    bool mixed = false, bf16 = false;
    int n_pre = 0, n_post = 0, maxit = 0;
    // work lists (host copies, uploaded by cams_batch_set_workspace)
    std::vector<WorkItem> lists[L_NUM];
    std::vector<InstDev> h_inst;
    size_t off_inst = 0, off_list[L_NUM] = {}, off_ndone = 0, off_res = 0, off_pptr = 0, need = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    InstDev *inst = nullptr;
    WorkItem *work[L_NUM] = {};
    int32_t *ndone = nullptr;
    BatchResult *res = nullptr;
    double **pptr = nullptr;
    // pinned host staging
    char *host = nullptr;
    size_t host_bytes = 0;
    // captured iterations
    hipGraphExec_t exec[kNumCand] = {};
    int chosen = -1;                 // index into kGraphIters once tuned
    double tune_ms[kNumCand] = {};   // ms per iteration of each candidate (first call)
    std::string err;
    float t_setup_ms = 0.f, t_iter_ms = 0.f;
    int iters_launched = 0;
};

namespace {

cams_status bfail(cams_batch *b, cams_status s, const std::string &m)
{
    if (b) b->err = m;
    return s;
}

BatchLaunch L(const cams_batch *b, int which)
{
    return BatchLaunch{b->inst, b->work[which], (int)b->lists[which].size(), b->stream};
}

void enqueue_batch_iteration(cams_batch *b, int par)
{
    const int count = (int)b->ctx.size();
    launch_batch_residual(L(b, L_FLAT), par, b->mixed);
    launch_batch_finalize(b->inst, count, b->ndone, b->stream);
    if (b->n_pre > 0) {
        launch_batch_smooth(L(b, L_SBLOCK), b->n_pre, 0, b->mixed);
        launch_batch_sub_pre(L(b, L_FLAT), b->mixed);
    }
    launch_batch_restrict(L(b, L_RESTRICT));
    launch_batch_sum_planes(L(b, L_NODES));
    launch_batch_gemv(L(b, L_ROWS));
    launch_batch_prolong(L(b, L_FLAT), b->mixed, b->bf16);
    launch_batch_r1(L(b, L_FLAT), b->mixed);
    if (b->n_post > 0) launch_batch_smooth(L(b, L_SBLOCK), b->n_post, 1, b->mixed);
}

// Capture `iters` iterations (iters even) into an executable graph.
hipGraphExec_t capture(cams_batch *b, int iters)
{
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    CAMS_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    for (int it = 0; it < iters; ++it) enqueue_batch_iteration(b, it & 1);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) throw HipError(e, "hipStreamEndCapture", __LINE__);
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) throw HipError(e, "hipGraphInstantiate", __LINE__);
    return ex;
}

int32_t *host_ndone(cams_batch *b) { return (int32_t *)b->host; }
BatchResult *host_res(cams_batch *b) { return (BatchResult *)(b->host + 256); }
double **host_pptr(cams_batch *b) { return (double **)(b->host + 256 + align_up(b->ctx.size() * sizeof(BatchResult))); }

int read_ndone(cams_batch *b)
{
    CAMS_HIP(hipMemcpyAsync(host_ndone(b), b->ndone, sizeof(int32_t), hipMemcpyDeviceToHost, b->stream));
    CAMS_HIP(hipStreamSynchronize(b->stream));
    return *host_ndone(b);
}

void reset_iteration(cams_batch *b)
{
    launch_batch_reset(L(b, L_FLAT));
    *host_ndone(b) = 0;
    CAMS_HIP(hipMemcpyAsync(b->ndone, host_ndone(b), sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
}

// Choose the iterations per graph: every candidate runs the same
// kTuneIters iterations from the same (reset) state, timed with events;
// the state is reset again afterwards.  Within 5% the candidate with fewer
// iterations per graph wins (fewer iterations wasted after the last stop).
void tune(cams_batch *b)
{
    constexpr int kTuneIters = 8;
    for (int k = 0; k < kNumCand; ++k) {
        reset_iteration(b);
        CAMS_HIP(hipEventRecord(b->ev[2], b->stream));
        for (int q = 0; q < kTuneIters / kGraphIters[k]; ++q) CAMS_HIP(hipGraphLaunch(b->exec[k], b->stream));
        CAMS_HIP(hipEventRecord(b->ev[3], b->stream));
        CAMS_HIP(hipEventSynchronize(b->ev[3]));
        float ms = 0.f;
        CAMS_HIP(hipEventElapsedTime(&ms, b->ev[2], b->ev[3]));
        b->tune_ms[k] = ms / kTuneIters;
    }
    int best = 0;
    for (int k = 1; k < kNumCand; ++k)
        if (b->tune_ms[k] < b->tune_ms[best]) best = k;
    for (int k = 0; k < best; ++k)
        if (b->tune_ms[k] <= 1.05 * b->tune_ms[best]) {
            best = k;
            break;
        }
    b->chosen = best;
    reset_iteration(b);
}

}  // namespace

extern "C" {

cams_status cams_batch_create(cams_ctx *const *ctxs, int32_t count, void *hip_stream, cams_batch **out)
{
    if (!out) return CAMS_E_ARG;
    *out = nullptr;
    if (!ctxs || count <= 0) return CAMS_E_ARG;
    const hipStream_t st = (hipStream_t)hip_stream;
    const cams_options &O = ctxs[0] ? ctxs[0]->opt : cams_options{};
    for (int i = 0; i < count; ++i) {
        const cams_ctx *c = ctxs[i];
        if (!c) return CAMS_E_ARG;
        if (c->stream != st) return CAMS_E_ARG;                 // one stream for the whole batch
        if (c->opt.smoother != CAMS_SMOOTH_BLOCK_ILU0) return CAMS_E_ARG;
        if (c->opt.precision != O.precision || c->opt.n_pre != O.n_pre || c->opt.n_post != O.n_post)
            return CAMS_E_ARG;
        if (c->g.dim != 3 && c->g.dim != 2) return CAMS_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return CAMS_E_ARG;                  // an instance twice
    }
    cams_batch *b = new (std::nothrow) cams_batch;
    if (!b) return CAMS_E_NOMEM;
    b->ctx.assign(ctxs, ctxs + count);
    b->user = st;
    b->mixed = O.precision != CAMS_FP64;
    b->bf16 = O.precision == CAMS_MIXED_BF16;
    b->n_pre = O.n_pre;
    b->n_post = O.n_post;
    for (int i = 0; i < count; ++i) b->maxit = std::max(b->maxit, ctxs[i]->opt.lin_maxit);

    // work lists, instance-major, then reordered for the XCD mapping
    for (int i = 0; i < count; ++i) {
        const cams_ctx *c = ctxs[i];
        const GridDev &g = c->g;
        const int nflat = (g.N + kBlock - 1) / kBlock;
        for (int k = 0; k < nflat; ++k) b->lists[L_FLAT].push_back({i, k});
        const int nsb = ((g.nx + 7) / 8) * ((g.ny + 7) / 8) * ((g.nz + 7) / 8);
        for (int k = 0; k < nsb; ++k) b->lists[L_SBLOCK].push_back({i, k});
        for (int k = 0; k < g.Nc * c->max_planes; ++k) b->lists[L_RESTRICT].push_back({i, k});
        for (int k = 0; k < (g.Nc + kBlock - 1) / kBlock; ++k) b->lists[L_NODES].push_back({i, k});
        for (int k = 0; k < (g.Nc + kBlock / 64 - 1) / (kBlock / 64); ++k) b->lists[L_ROWS].push_back({i, k});
    }
    for (int l = 0; l < L_NUM; ++l) {
        std::vector<WorkItem> &v = b->lists[l];
        std::vector<WorkItem> w(v.size());
        for (size_t t = 0; t < v.size(); ++t) w[t] = v[xcd_swizzle_host((int)t, (int)v.size())];
        v.swap(w);
    }
    if (b->lists[L_RESTRICT].size() > 0x7fffffffu || b->lists[L_FLAT].size() > 0x7fffffffu) {
        delete b;
        return CAMS_E_ARG;
    }
    size_t o = 0;
    b->off_inst = o;
    o = align_up(o + count * sizeof(InstDev));
    for (int l = 0; l < L_NUM; ++l) {
        b->off_list[l] = o;
        o = align_up(o + b->lists[l].size() * sizeof(WorkItem));
    }
    b->off_ndone = o;
    o = align_up(o + sizeof(int32_t));
    b->off_res = o;
    o = align_up(o + count * sizeof(BatchResult));
    b->off_pptr = o;
    o = align_up(o + count * sizeof(double *));
    b->need = o;
    *out = b;
    return CAMS_OK;
}

size_t cams_batch_workspace_bytes(const cams_batch *b) { return b ? b->need : 0; }

cams_status cams_batch_set_workspace(cams_batch *b, void *ws_dev, size_t bytes)
{
    if (!b) return CAMS_E_ARG;
    if (!ws_dev || ((uintptr_t)ws_dev & 255)) return bfail(b, CAMS_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < b->need) return bfail(b, CAMS_E_NOMEM, "batch workspace too small");
    for (cams_ctx *c : b->ctx)
        if (!c->has_ws) return bfail(b, CAMS_E_STATE, "every context needs its workspace first");
    try {
        const int count = (int)b->ctx.size();
        if (!b->host) {
            b->host_bytes = 256 + align_up(count * sizeof(BatchResult)) + align_up(count * sizeof(double *));
            CAMS_HIP(hipHostMalloc((void **)&b->host, b->host_bytes, hipHostMallocDefault));
            CAMS_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            for (int s = 0; s < kSide; ++s) {
                CAMS_HIP(hipStreamCreateWithFlags(&b->side[s], hipStreamNonBlocking));
                CAMS_HIP(hipEventCreateWithFlags(&b->join[s], hipEventDisableTiming));
            }
            CAMS_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
            for (int e = 0; e < 4; ++e) CAMS_HIP(hipEventCreate(&b->ev[e]));
        }
        for (int e = 0; e < kNumCand; ++e)
            if (b->exec[e]) {
                (void)hipGraphExecDestroy(b->exec[e]);
                b->exec[e] = nullptr;
            }
        char *w = (char *)ws_dev;
        b->ws = w;
        b->ws_bytes = bytes;
        b->inst = (InstDev *)(w + b->off_inst);
        for (int l = 0; l < L_NUM; ++l) b->work[l] = (WorkItem *)(w + b->off_list[l]);
        b->ndone = (int32_t *)(w + b->off_ndone);
        b->res = (BatchResult *)(w + b->off_res);
        b->pptr = (double **)(w + b->off_pptr);
        b->h_inst.resize(count);
        for (int i = 0; i < count; ++i) {
            const cams_ctx *c = b->ctx[i];
            InstDev &d = b->h_inst[i];
            memset(&d, 0, sizeof(d));
            d.g = c->g;
            d.a = c->a;
            d.fe = c->opt.restriction == CAMS_R_FE;
            d.bf16 = b->bf16;
            d.n_pre = c->opt.n_pre;
            d.n_post = c->opt.n_post;
            d.max_planes = c->max_planes;
            d.nparts = (c->g.N + kBlock - 1) / kBlock;
            d.maxit = c->opt.lin_maxit;
            d.rtol2 = c->opt.lin_rtol * c->opt.lin_rtol;
        }
        CAMS_HIP(hipMemcpyAsync(b->inst, b->h_inst.data(), count * sizeof(InstDev), hipMemcpyHostToDevice,
                                b->stream));
        for (int l = 0; l < L_NUM; ++l)
            if (!b->lists[l].empty())
                CAMS_HIP(hipMemcpyAsync(b->work[l], b->lists[l].data(), b->lists[l].size() * sizeof(WorkItem),
                                        hipMemcpyHostToDevice, b->stream));
        CAMS_HIP(hipStreamSynchronize(b->stream));   // the host vectors must outlive the copies
    } catch (const HipError &e) {
        return bfail(b, CAMS_E_DEVICE, std::string("batch_set_workspace: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

cams_status cams_batch_newton_iteration(cams_batch *b, const double *const *pn_dev, double *const *p_dev,
                                        int32_t *status_out, cams_stats *stats)
{
    if (!b) return CAMS_E_ARG;
    if (!pn_dev || !p_dev) return bfail(b, CAMS_E_ARG, "null pressure tables");
    if (!b->ws) return bfail(b, CAMS_E_STATE, "no batch workspace");
    const int count = (int)b->ctx.size();
    for (int i = 0; i < count; ++i) {
        if (!pn_dev[i] || !p_dev[i]) return bfail(b, CAMS_E_ARG, "null pressure");
        const cams_ctx *c = b->ctx[i];
        if (!c->has_rock) return bfail(b, CAMS_E_STATE, "every context needs set_rock first");
        if (b->h_inst[i].a.T != c->a.T || b->h_inst[i].a.ictl != c->a.ictl)
            return bfail(b, CAMS_E_STATE, "a context's workspace changed; set the batch workspace again");
    }
    try {
        // order after the caller's work on the contexts' stream
        CAMS_HIP(hipEventRecord(b->fork, b->user));
        CAMS_HIP(hipStreamWaitEvent(b->stream, b->fork, 0));
        memcpy(host_pptr(b), p_dev, count * sizeof(double *));
        CAMS_HIP(hipMemcpyAsync(b->pptr, host_pptr(b), count * sizeof(double *), hipMemcpyHostToDevice, b->stream));
        *host_ndone(b) = 0;
        CAMS_HIP(hipMemcpyAsync(b->ndone, host_ndone(b), sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
        CAMS_HIP(hipEventRecord(b->ev[0], b->stream));

        // setup of every instance, spread over the side streams
        CAMS_HIP(hipEventRecord(b->fork, b->stream));
        for (int s = 0; s < kSide; ++s) CAMS_HIP(hipStreamWaitEvent(b->side[s], b->fork, 0));
        for (int i = 0; i < count; ++i) {
            cams_ctx *c = b->ctx[i];
            const hipStream_t own = c->stream;
            c->stream = b->side[i % kSide];
            try {
                enqueue_clear_status(c);
                launch_impose_wells(c, p_dev[i]);
                if (!c->has_basis) enqueue_basis_local(c);
                enqueue_assemble(c, p_dev[i], pn_dev[i]);
                enqueue_coarse(c);
                launch_iter_reset(c);
            } catch (...) {
                c->stream = own;
                throw;
            }
            c->stream = own;
        }
        for (int s = 0; s < kSide; ++s) {
            CAMS_HIP(hipEventRecord(b->join[s], b->side[s]));
            CAMS_HIP(hipStreamWaitEvent(b->stream, b->join[s], 0));
        }
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipEventRecord(b->ev[1], b->stream));

        // batched iterations: replay captured graphs until every instance stopped
        if (!b->exec[0])
            for (int k = 0; k < kNumCand; ++k) b->exec[k] = capture(b, kGraphIters[k]);
        if (b->chosen < 0) tune(b);
        const int k = b->chosen;
        int launched = 0, done = 0;
        const int limit = b->maxit + 1;   // the device stops every instance by then
        int ahead = 8;
        while (launched < limit + kGraphIters[kNumCand - 1]) {
            const int reps = std::max(1, ahead / kGraphIters[k]);
            for (int q = 0; q < reps; ++q) CAMS_HIP(hipGraphLaunch(b->exec[k], b->stream));
            launched += reps * kGraphIters[k];
            done = read_ndone(b);
            if (done >= count) break;
            ahead = std::min(32, ahead * 2);
        }
        b->iters_launched = launched;
        launch_batch_update(BatchLaunch{b->inst, b->work[L_FLAT], (int)b->lists[L_FLAT].size(), b->stream},
                            b->pptr);
        launch_batch_gather(b->inst, count, b->res, b->stream);
        CAMS_HIP(hipMemcpyAsync(host_res(b), b->res, count * sizeof(BatchResult), hipMemcpyDeviceToHost, b->stream));
        CAMS_HIP(hipEventRecord(b->ev[2], b->stream));
        CAMS_HIP(hipStreamWaitEvent(b->user, b->ev[2], 0));
        CAMS_HIP(hipStreamSynchronize(b->stream));
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipEventElapsedTime(&b->t_setup_ms, b->ev[0], b->ev[1]));
        CAMS_HIP(hipEventElapsedTime(&b->t_iter_ms, b->ev[1], b->ev[2]));
        if (done < count) return bfail(b, CAMS_E_DEVICE, "batched iteration did not stop every instance");
    } catch (const HipError &e) {
        return bfail(b, CAMS_E_DEVICE, std::string("batch_newton_iteration: ") + hipGetErrorString(e.code));
    }
    cams_status worst = CAMS_OK;
    for (int i = 0; i < count; ++i) {
        const BatchResult &r = host_res(b)[i];
        cams_ctx *c = b->ctx[i];
        cams_status s = CAMS_OK;
        if (r.status & F_SINGULAR_COARSE) s = CAMS_E_BREAKDOWN;
        else if (r.status) s = CAMS_E_BREAKDOWN;
        else if (r.outcome == 1) s = CAMS_E_NOT_CONVERGED;
        else if (r.outcome == 2) s = CAMS_E_BREAKDOWN;
        c->has_basis = c->has_system = c->has_coarse = true;
        cams_stats st;
        memset(&st, 0, sizeof(st));
        st.newton_iters = 1;
        st.lin_iters_total = st.lin_iters_last = r.it;
        st.relres_last = r.r0n2 > 0 ? std::sqrt(r.rn2 / r.r0n2) : 0.0;
        st.eps_norm_last = std::sqrt(r.eps2);
        // the setup phases of all instances overlap: their common wall time is
        // reported as t_coarse_ms (basis and assembly included)
        st.t_coarse_ms = b->t_setup_ms;
        st.t_iterate_ms = b->t_iter_ms;
        c->last = st;
        if (stats) stats[i] = st;
        if (status_out) status_out[i] = s;
        if (s != CAMS_OK && worst == CAMS_OK) worst = s;
    }
    if (worst != CAMS_OK) return bfail(b, worst, "at least one instance failed (see the per-instance status)");
    return CAMS_OK;
}

cams_status cams_batch_tuning(const cams_batch *b, int32_t *iters_per_graph, double *ms_per_iter_candidates,
                              int32_t ncand)
{
    if (!b) return CAMS_E_ARG;
    if (iters_per_graph) *iters_per_graph = b->chosen >= 0 ? kGraphIters[b->chosen] : 0;
    if (ms_per_iter_candidates)
        for (int k = 0; k < std::min<int>(ncand, kNumCand); ++k) ms_per_iter_candidates[k] = b->tune_ms[k];
    return CAMS_OK;
}

const char *cams_batch_last_error(const cams_batch *b) { return b ? b->err.c_str() : "null batch"; }

void cams_batch_destroy(cams_batch *b)
{
    if (!b) return;
    for (int k = 0; k < kNumCand; ++k)
        if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
    for (int s = 0; s < kSide; ++s) {
        if (b->side[s]) (void)hipStreamDestroy(b->side[s]);
        if (b->join[s]) (void)hipEventDestroy(b->join[s]);
    }
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int e = 0; e < 4; ++e)
        if (b->ev[e]) (void)hipEventDestroy(b->ev[e]);
    if (b->host) (void)hipHostFree(b->host);
    delete b;
}

}  // extern "C"
