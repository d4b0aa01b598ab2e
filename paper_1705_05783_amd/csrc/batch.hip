// Batched C-AMS: many independent problems of different sizes advanced by
// one Newton iteration together.  The setup of each instance (basis,
// assembly, coarse operator, smoother pivots) is enqueued on a few side
// streams so that the instances' small kernels overlap; the factorisation
// and inverse of the MSFE coarse operators then run batched (one launch per
// panel step for all instances, their GEMM tiles in one grid), and the
// C-AMS iterations as ONE launch per kernel for all instances.
// Each batched kernel is persistent: as many workgroups as the device holds
// at once walk a work list of (instance, block) items in device memory.
// A fixed number of iterations is captured once into a HIP graph and
// replayed until every instance has stopped; between replays the host reads
// the per-instance results and, once the instances still running hold
// clearly fewer cells than the lists cover, uploads lists compacted to them
// (the graph reads the list lengths from device memory, so it stays valid).
//
// Tuning, on the first call of a batch: the smoother's workgroup size (128,
// 256 or 512 threads per 8x8x8 block: fewer threads keep more of the
// latency-bound sweeps in flight per compute unit) is chosen by timing the
// batch's own smoothing steps; then every candidate number of iterations per
// graph runs the same first iterations from the same state, timed with
// events, and the state is reset before the real solve.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cams_internal.h"

using namespace cams;

namespace {

constexpr int kSide = 4;                     // setup streams (the device has 4 hardware queues per process)
constexpr int kGraphIters[] = {2, 4, 8};     // candidates of the tuner (even: the ping-pong parity repeats)
constexpr int kNumCand = 3;
// smoother forms the tuner compares: 128, 256 or 512 threads per block, and
// (FP32 only) four blocks along x per 512-thread workgroup (0)
constexpr int kSmoothNT[] = {128, 256, 512, 0};
constexpr int kNumSmooth = 4;

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

enum { L_FLAT = 0, L_SBLOCK, L_RESTRICT, L_NODES, L_ROWS, L_SROW, L_NUM };

}  // namespace

namespace cams {

int resident_workgroups(const void *kernel, int threads)
{
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({kernel, threads});
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per_cu = 0;
    CAMS_HIP(hipGetDevice(&dev));
    CAMS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CAMS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
    const int n = std::max(1, per_cu) * std::max(1, cus);
    cache[{kernel, threads}] = n;
    return n;
}

}  // namespace cams

// LDS classes of the batched local basis solves (bytes per workgroup):
// small systems are launched apart from the 7^3 interiors so that many of
// them share a compute unit.
constexpr int kBasisClasses = 4;
constexpr size_t kBasisClassBytes[kBasisClasses] = {16 << 10, 40 << 10, 80 << 10, 160 << 10};

struct cams_batch {
    std::vector<cams_ctx *> ctx;
    hipStream_t user = nullptr;      // the contexts' stream: ordered before and after each call
    hipStream_t stream = nullptr;    // batched launches and graph replays (created, capturable)
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {}, ev[4] = {};
    bool mixed = false, bf16 = false;
    int precision = CAMS_FP64;
    int n_pre = 0, n_post = 0, maxit = 0;
    // full work lists per kind, instance-major (host); the device holds the
    // lists of the instances still running (XCD order) and their lengths
    std::vector<WorkItem> lists[L_NUM];
    std::vector<InstDev> h_inst;
    std::vector<double> cells;       // cells per instance
    std::vector<char> listed;        // instance in the device lists
    double listed_cells = 0.0;
    size_t off_inst = 0, off_list[L_NUM + 1] = {}, off_nwork = 0, off_res = 0, off_pptr = 0, off_lu_steps = 0,
           off_lu_gemms = 0, need = 0;
    // batched factorisation of the MSFE instances (plan built with the workspace)
    std::vector<cams_ctx *> fe;
    size_t lu_steps_cap = 0, lu_gemms_cap = 0;
    BatchGjPlan lu;
    GjPivotDesc *d_steps = nullptr;
    GemmDesc *d_gemms = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    InstDev *inst = nullptr;
    WorkItem *work[L_NUM + 1] = {};  // [L_NUM]: the full flat list (update, reset)
    int32_t *nwork = nullptr;        // list lengths, L_NUM + 1 entries
    BatchResult *res = nullptr;
    double **pptr = nullptr;
    // pinned host staging: counters, results, pressure table, lists
    char *host = nullptr;
    size_t host_bytes = 0, host_lists = 0;
    int compactions = 0;
    // captured iterations
    hipGraphExec_t exec[kNumCand] = {};
    int chosen = -1;                 // index into kGraphIters once tuned
    double tune_ms[kNumCand] = {};   // ms per iteration of each candidate (first call)
    int smooth_nt = 512;             // threads per smoother block (tuned on the first call)
    int forced_nt = -1;              // smoother form set by the caller (-1: tuned)
    double smooth_ms[kNumSmooth] = {};
    // local basis solves of every instance, per stage (open axes 1..3) and
    // LDS class: work items (instance, region) and the class's largest system
    std::vector<WorkItem> blist[4][kBasisClasses];
    int bcap[4][kBasisClasses] = {};
    size_t off_blist[4][kBasisClasses] = {};
    int from_cache = -1;             // last tuning: 1 from the process-wide cache, 0 measured, -1 none
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

// A batched launch over list `which` (L_NUM: the full flat list); `prime`
// launches nothing (occupancy queries only).
BatchLaunch L(const cams_batch *b, int which, bool prime = false)
{
    const size_t n = b->lists[which == L_NUM ? L_FLAT : which].size();
    return BatchLaunch{b->inst, b->work[which], b->nwork + which, prime ? 0 : (int)n, b->stream};
}

void enqueue_batch_iteration(cams_batch *b, int par, bool prime = false)
{
    const int count = (int)b->ctx.size();
    launch_batch_residual(L(b, L_FLAT, prime), par, b->mixed, b->n_pre > 0);
    if (!prime) launch_batch_finalize(b->inst, count, b->stream);
    const int sl = b->smooth_nt == 0 ? L_SROW : L_SBLOCK;
    if (b->n_pre > 0) {
        launch_batch_smooth(L(b, sl, prime), b->n_pre, 0, b->mixed, b->smooth_nt);
        launch_batch_sub_pre(L(b, L_FLAT, prime), b->mixed);
    }
    launch_batch_restrict(L(b, L_RESTRICT, prime), b->precision);
    launch_batch_node_sum(L(b, L_NODES, prime));
    launch_batch_gemv(L(b, L_ROWS, prime));
    launch_batch_prolong(L(b, L_FLAT, prime), b->mixed, b->bf16);
    if (b->n_post > 0) launch_batch_smooth(L(b, sl, prime), b->n_post, 1, b->mixed, b->smooth_nt);
}

WorkItem *host_list(cams_batch *b, int l);

// Upload the lists restricted to the instances with keep[i] set, each list
// in XCD order; the lengths go to nwork.  Only called when no launch that
// reads the lists can be pending (after a stream synchronisation).
void upload_lists(cams_batch *b, const std::vector<char> &keep)
{
    int32_t *counts = (int32_t *)b->host;
    std::vector<WorkItem> v;
    for (int l = 0; l < L_NUM; ++l) {
        v.clear();
        for (const WorkItem &w : b->lists[l])
            if (keep[w.inst]) v.push_back(w);
        WorkItem *dst = host_list(b, l);
        const int n = (int)v.size();
        for (int t = 0; t < n; ++t) dst[t] = v[xcd_swizzle_host(t, n)];
        counts[l] = n;
        if (n > 0)
            CAMS_HIP(hipMemcpyAsync(b->work[l], dst, n * sizeof(WorkItem), hipMemcpyHostToDevice, b->stream));
    }
    counts[L_NUM] = (int)b->lists[L_FLAT].size();
    CAMS_HIP(hipMemcpyAsync(b->nwork, counts, (L_NUM + 1) * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
    b->listed = keep;
    b->listed_cells = 0.0;
    for (size_t i = 0; i < keep.size(); ++i)
        if (keep[i]) b->listed_cells += b->cells[i];
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

// Pinned host layout: [0, 256) list lengths, results, pressure table, then
// the list staging area.
BatchResult *host_res(cams_batch *b) { return (BatchResult *)(b->host + 256); }
double **host_pptr(cams_batch *b) { return (double **)(b->host + 256 + align_up(b->ctx.size() * sizeof(BatchResult))); }
WorkItem *host_list(cams_batch *b, int l)
{
    size_t o = b->host_lists;
    for (int k = 0; k < l; ++k) o += align_up(b->lists[k].size() * sizeof(WorkItem));
    return (WorkItem *)(b->host + o);
}

void read_results(cams_batch *b)
{
    const int count = (int)b->ctx.size();
    launch_batch_gather(b->inst, count, b->res, b->stream);
    CAMS_HIP(hipMemcpyAsync(host_res(b), b->res, count * sizeof(BatchResult), hipMemcpyDeviceToHost, b->stream));
}

void reset_iteration(cams_batch *b)
{
    launch_batch_reset(L(b, L_NUM));
}

// Tuning results shared by the batches of one process, keyed by what the
// choice depends on: precision, smoothing counts, whether an instance
// alternates block grids, and the powers of two of the batch's total cells
// and instance count.  A batch whose key is cached takes the stored choice
// (and timings) instead of timing the candidates again.
struct TuneKey {
    int precision, n_pre, n_post, alt, cells_log2, count_log2;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(precision, n_pre, n_post, alt, cells_log2, count_log2) <
               std::tie(o.precision, o.n_pre, o.n_post, o.alt, o.cells_log2, o.count_log2);
    }
};
struct TuneEntry {
    int smooth_nt, chosen;
    double tune_ms[kNumCand], smooth_ms[kNumSmooth];
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune_cache;

TuneKey tune_key(const cams_batch *b)
{
    double cells = 0.0;
    int alt = 0;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        cells += b->cells[i];
        alt |= b->ctx[i]->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0;
    }
    return TuneKey{b->precision, b->n_pre, b->n_post, alt, (int)std::floor(std::log2(std::max(cells, 1.0))),
                   (int)std::floor(std::log2((double)b->ctx.size()))};
}

// Choose the smoother's workgroup size: each candidate runs the same
// smoothing steps over the whole batch (eager launches, timed with events).
// The steps only write the smoother's own output vectors, which every
// iteration rewrites before reading them.
void tune_smoother(cams_batch *b)
{
    const int steps = std::max(1, b->n_post > 0 ? b->n_post : b->n_pre);
    const int kind = b->n_post > 0 ? 1 : 0;
    int best = 0;
    for (int k = 0; k < kNumSmooth; ++k) {
        if (kSmoothNT[k] == 0 && !b->mixed) continue;   // the row form is FP32 only
        const int sl = kSmoothNT[k] == 0 ? L_SROW : L_SBLOCK;
        launch_batch_smooth(L(b, sl), steps, kind, b->mixed, kSmoothNT[k]);   // warm
        CAMS_HIP(hipEventRecord(b->ev[2], b->stream));
        launch_batch_smooth(L(b, sl), steps, kind, b->mixed, kSmoothNT[k]);
        CAMS_HIP(hipEventRecord(b->ev[3], b->stream));
        CAMS_HIP(hipEventSynchronize(b->ev[3]));
        float ms = 0.f;
        CAMS_HIP(hipEventElapsedTime(&ms, b->ev[2], b->ev[3]));
        b->smooth_ms[k] = ms / steps;
        if (b->smooth_ms[k] < b->smooth_ms[best]) best = k;   // compared with measured sizes only
    }
    b->smooth_nt = kSmoothNT[best];
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
        if (!block_smoother(c->opt)) return CAMS_E_ARG;             // batches run block smoothers
        if (c->opt.basis_type != CAMS_BASIS_B4) return CAMS_E_ARG;   // the batch builds B4 bases
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
    b->precision = O.precision;
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
        const int nsrow = ((g.nx + 31) / 32) * ((g.ny + 7) / 8) * ((g.nz + 7) / 8);   // groups of 4 x-blocks
        for (int k = 0; k < nsrow; ++k) b->lists[L_SROW].push_back({i, k});
        for (int k = 0; k < g.Nc; ++k) b->lists[L_RESTRICT].push_back({i, k});
        for (int k = 0; k < (g.Nc + kBlock - 1) / kBlock; ++k) b->lists[L_NODES].push_back({i, k});
        for (int k = 0; k < (g.Nc + kBlock / 64 - 1) / (kBlock / 64); ++k) b->lists[L_ROWS].push_back({i, k});
    }
    for (int i = 0; i < count; ++i) b->cells.push_back((double)ctxs[i]->g.N);
    // basis work lists: each instance's regions of a stage, by LDS class
    for (int i = 0; i < count; ++i) {
        const cams_ctx *c = ctxs[i];
        for (int f = 1; f <= 3; ++f)
            for (int q = c->regoff[f]; q < c->regoff[f] + c->nreg[f]; ++q) {
                const Region &R = c->regions[q];
                const int st[3] = {1, R.len[0], R.len[0] * R.len[1]};
                int bw = 1;
                for (int a = 0; a < 3; ++a)
                    if (R.freemask & (1 << a)) bw = st[a];
                const int need = R.len[0] * R.len[1] * R.len[2] * (bw + 1 + 8);
                int k = 0;
                while (k < kBasisClasses - 1 && (size_t)need * sizeof(double) > kBasisClassBytes[k]) ++k;
                b->blist[f][k].push_back({i, q});
                b->bcap[f][k] = std::max(b->bcap[f][k], need);
            }
    }
    for (int l = 0; l < L_NUM; ++l)
        if (b->lists[l].size() > 0x7fffffffu) {
            delete b;
            return CAMS_E_ARG;
        }
    size_t o = 0;
    b->off_inst = o;
    o = align_up(o + count * sizeof(InstDev));
    for (int l = 0; l <= L_NUM; ++l) {
        b->off_list[l] = o;
        o = align_up(o + b->lists[l == L_NUM ? L_FLAT : l].size() * sizeof(WorkItem));
    }
    for (int f = 1; f <= 3; ++f)
        for (int k = 0; k < kBasisClasses; ++k) {
            b->off_blist[f][k] = o;
            o = align_up(o + b->blist[f][k].size() * sizeof(WorkItem));
        }
    b->off_nwork = o;
    o = align_up(o + (L_NUM + 1) * sizeof(int32_t));
    b->off_res = o;
    o = align_up(o + count * sizeof(BatchResult));
    b->off_pptr = o;
    o = align_up(o + count * sizeof(double *));
    for (int i = 0; i < count; ++i)
        if (ctxs[i]->opt.restriction == CAMS_R_FE) {
            const size_t T = (ctxs[i]->g.Nc + 63) / 64;
            b->fe.push_back(ctxs[i]);
            b->lu_steps_cap += T;        // one pivot step per panel
            b->lu_gemms_cap += 10 * T + 1;   // per panel at most 9 descriptors, and the mirror
        }
    b->off_lu_steps = o;
    o = align_up(o + b->lu_steps_cap * sizeof(GjPivotDesc));
    b->off_lu_gemms = o;
    o = align_up(o + b->lu_gemms_cap * sizeof(GemmDesc));
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
            b->host_lists = 256 + align_up(count * sizeof(BatchResult)) + align_up(count * sizeof(double *));
            b->host_bytes = b->host_lists;
            for (int l = 0; l < L_NUM; ++l) b->host_bytes += align_up(b->lists[l].size() * sizeof(WorkItem));
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
        for (int l = 0; l <= L_NUM; ++l) b->work[l] = (WorkItem *)(w + b->off_list[l]);
        b->nwork = (int32_t *)(w + b->off_nwork);
        b->res = (BatchResult *)(w + b->off_res);
        b->d_steps = (GjPivotDesc *)(w + b->off_lu_steps);
        b->d_gemms = (GemmDesc *)(w + b->off_lu_gemms);
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
            d.alt = c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0;
            d.nparts = (c->g.N + kBlock - 1) / kBlock;
            d.maxit = c->opt.lin_maxit;
            d.rtol2 = c->opt.lin_rtol * c->opt.lin_rtol;
        }
        CAMS_HIP(hipMemcpyAsync(b->inst, b->h_inst.data(), count * sizeof(InstDev), hipMemcpyHostToDevice,
                                b->stream));
        // the full flat list (XCD order) for the update and the reset
        {
            const std::vector<WorkItem> &v = b->lists[L_FLAT];
            std::vector<WorkItem> full(v.size());
            for (size_t t = 0; t < v.size(); ++t) full[t] = v[xcd_swizzle_host((int)t, (int)v.size())];
            CAMS_HIP(hipMemcpyAsync(b->work[L_NUM], full.data(), full.size() * sizeof(WorkItem),
                                    hipMemcpyHostToDevice, b->stream));
            CAMS_HIP(hipStreamSynchronize(b->stream));   // `full` must outlive the copy
        }
        plan_batch_gj(b->fe, b->lu);
        if (b->lu.piv.size() > b->lu_steps_cap || b->lu.gemms.size() > b->lu_gemms_cap)
            return bfail(b, CAMS_E_STATE, "factorisation plan exceeds its capacity");
        if (!b->lu.piv.empty())
            CAMS_HIP(hipMemcpyAsync(b->d_steps, b->lu.piv.data(), b->lu.piv.size() * sizeof(GjPivotDesc),
                                    hipMemcpyHostToDevice, b->stream));
        if (!b->lu.gemms.empty())
            CAMS_HIP(hipMemcpyAsync(b->d_gemms, b->lu.gemms.data(), b->lu.gemms.size() * sizeof(GemmDesc),
                                    hipMemcpyHostToDevice, b->stream));
        upload_lists(b, std::vector<char>(count, 1));
        for (int f = 1; f <= 3; ++f)
            for (int k = 0; k < kBasisClasses; ++k)
                if (!b->blist[f][k].empty())
                    CAMS_HIP(hipMemcpyAsync(w + b->off_blist[f][k], b->blist[f][k].data(),
                                            b->blist[f][k].size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                                            b->stream));
        // occupancy of every batched kernel, before any capture
        enqueue_batch_iteration(b, 0, true);
        launch_batch_reset(L(b, L_NUM, true));
        launch_batch_update(L(b, L_NUM, true), nullptr);
        CAMS_HIP(hipStreamSynchronize(b->stream));
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
        CAMS_HIP(hipEventRecord(b->ev[0], b->stream));

        // setup of every instance, spread over the side streams.  When every
        // instance needs its basis, the local solves of each stage run as
        // batched launches over all instances' regions (by LDS class)
        // between a first per-instance phase (vertices, assembly) and a
        // second (rounding, coarse operator and its factorisation);
        // otherwise each instance builds what it lacks in one phase.
        bool all_basis = true;
        for (const cams_ctx *c : b->ctx) all_basis = all_basis && !c->has_basis;
        auto per_instance = [&](auto fn) {
            CAMS_HIP(hipEventRecord(b->fork, b->stream));
            for (int s = 0; s < kSide; ++s) CAMS_HIP(hipStreamWaitEvent(b->side[s], b->fork, 0));
            for (int i = 0; i < count; ++i) {
                cams_ctx *c = b->ctx[i];
                const hipStream_t own = c->stream;
                c->stream = b->side[i % kSide];
                try {
                    fn(c, i);
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
        };
        auto coarse_setup = [&](cams_ctx *c) {
            enqueue_coarse_operator(c);
            if (c->opt.restriction == CAMS_R_FE)
                launch_coarse_factor_prepare(c);   // factorised below, batched
            else
                launch_coarse_factor(c);
            launch_iter_reset(c);
        };
        if (all_basis) {
            per_instance([&](cams_ctx *c, int i) {
                enqueue_clear_status(c);
                launch_impose_wells(c, p_dev[i]);
                launch_basis_vertices(c);
                enqueue_assemble(c, p_dev[i], pn_dev[i]);
            });
            for (int f = 1; f <= 3; ++f)
                for (int k = 0; k < kBasisClasses; ++k)
                    launch_batch_basis_regions(b->inst, (const WorkItem *)(b->ws + b->off_blist[f][k]),
                                               (int)b->blist[f][k].size(), f, b->bcap[f][k], b->stream);
            per_instance([&](cams_ctx *c, int) {
                if (c->opt.precision != CAMS_FP64) launch_round_basis(c);
                coarse_setup(c);
            });
        } else {
            per_instance([&](cams_ctx *c, int i) {
                enqueue_clear_status(c);
                launch_impose_wells(c, p_dev[i]);
                if (!c->has_basis) enqueue_basis_local(c);
                enqueue_assemble(c, p_dev[i], pn_dev[i]);
                coarse_setup(c);
            });
        }
        launch_batch_gj(b->lu, b->d_steps, b->d_gemms, b->stream);
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipEventRecord(b->ev[1], b->stream));

        // batched iterations: replay captured graphs until every instance stopped
        bool all_listed = true;
        for (char k : b->listed) all_listed = all_listed && k;
        if (!all_listed) upload_lists(b, std::vector<char>(count, 1));
        int cached_chosen = -1;
        if (!b->exec[0]) {
            b->from_cache = -1;
            if (b->forced_nt >= 0) {
                b->smooth_nt = b->forced_nt;
            } else {
                std::lock_guard<std::mutex> lock(g_tune_mu);
                const auto it = g_tune_cache.find(tune_key(b));
                if (it != g_tune_cache.end()) {
                    const TuneEntry &e = it->second;
                    b->smooth_nt = e.smooth_nt;
                    cached_chosen = e.chosen;
                    std::copy(e.tune_ms, e.tune_ms + kNumCand, b->tune_ms);
                    std::copy(e.smooth_ms, e.smooth_ms + kNumSmooth, b->smooth_ms);
                }
            }
            if (b->forced_nt < 0 && cached_chosen < 0) tune_smoother(b);
            for (int k = 0; k < kNumCand; ++k) b->exec[k] = capture(b, kGraphIters[k]);
        }
        if (b->chosen < 0) {
            if (cached_chosen >= 0) {
                b->chosen = cached_chosen;
                b->from_cache = 1;
            } else {
                tune(b);
                if (b->forced_nt < 0) {
                    b->from_cache = 0;
                    TuneEntry e{b->smooth_nt, b->chosen, {}, {}};
                    std::copy(b->tune_ms, b->tune_ms + kNumCand, e.tune_ms);
                    std::copy(b->smooth_ms, b->smooth_ms + kNumSmooth, e.smooth_ms);
                    std::lock_guard<std::mutex> lock(g_tune_mu);
                    g_tune_cache[tune_key(b)] = e;
                }
            }
        }
        const int k = b->chosen;
        int launched = 0, done = 0;
        const int limit = b->maxit + 1;   // the device stops every instance by then
        int ahead = 8;
        while (launched < limit + kGraphIters[kNumCand - 1]) {
            const int reps = std::max(1, ahead / kGraphIters[k]);
            for (int q = 0; q < reps; ++q) CAMS_HIP(hipGraphLaunch(b->exec[k], b->stream));
            launched += reps * kGraphIters[k];
            read_results(b);
            CAMS_HIP(hipStreamSynchronize(b->stream));
            std::vector<char> running(count, 0);
            double running_cells = 0.0;
            done = 0;
            for (int i = 0; i < count; ++i) {
                if (host_res(b)[i].done) {
                    ++done;
                } else {
                    running[i] = 1;
                    running_cells += b->cells[i];
                }
            }
            if (done >= count) break;
            // compact once the running instances cover well under the listed cells
            if (running_cells < 0.7 * b->listed_cells) {
                upload_lists(b, running);
                ++b->compactions;
            }
            ahead = std::min(32, ahead * 2);
        }
        b->iters_launched = launched;
        launch_batch_update(L(b, L_NUM), b->pptr);
        read_results(b);
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
        c->has_basis = c->has_system = true;
        // the batch leaves a dense inverse in Ainv; a context whose own
        // coarse solve is the block-tridiagonal form must factorise again
        // before cams_iterate (it would read Ainv as plane blocks)
        c->has_coarse = !c->blocktri;
        c->has_cfac = false;   // Ainv was overwritten by the batch's own inverse
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

cams_status cams_batch_tuning(const cams_batch *b, int32_t *iters_per_graph, int32_t *smoother_threads,
                              int32_t *smoother_blocks, double *ms_per_iter_candidates,
                              double *ms_per_smooth_step_candidates, int32_t ncand)
{
    if (!b) return CAMS_E_ARG;
    if (iters_per_graph) *iters_per_graph = b->chosen >= 0 ? kGraphIters[b->chosen] : 0;
    const bool row = b->smooth_nt == 0;
    if (smoother_threads) *smoother_threads = b->exec[0] ? (row ? 512 : b->smooth_nt) : 0;
    if (smoother_blocks) *smoother_blocks = b->exec[0] ? (row ? 4 : 1) : 0;
    for (int k = 0; k < std::min<int>(ncand, kNumCand); ++k)
        if (ms_per_iter_candidates) ms_per_iter_candidates[k] = b->tune_ms[k];
    for (int k = 0; k < std::min<int>(ncand, kNumSmooth); ++k)
        if (ms_per_smooth_step_candidates) ms_per_smooth_step_candidates[k] = b->smooth_ms[k];
    return CAMS_OK;
}

cams_status cams_batch_tuning_source(const cams_batch *b, int32_t *from_cache)
{
    if (!b || !from_cache) return CAMS_E_ARG;
    *from_cache = b->from_cache;
    return CAMS_OK;
}

void cams_batch_clear_tuning_cache(void)
{
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.clear();
}

cams_status cams_batch_set_smoother(cams_batch *b, int32_t threads, int32_t blocks)
{
    if (!b) return CAMS_E_ARG;
    int nt;
    if (threads == 0 && blocks == 0) nt = -1;
    else if (blocks == 1 && (threads == 128 || threads == 256 || threads == 512)) nt = threads;
    else if (blocks == 4 && threads == 512 && b->mixed) nt = 0;
    else return bfail(b, CAMS_E_ARG, "smoother form: (128|256|512, 1), (512, 4) in mixed precision, or (0, 0)");
    if (nt == b->forced_nt) return CAMS_OK;
    b->forced_nt = nt;
    // the captured iterations hold the smoother launches: capture (and tune) again
    for (int k = 0; k < kNumCand; ++k)
        if (b->exec[k]) {
            (void)hipGraphExecDestroy(b->exec[k]);
            b->exec[k] = nullptr;
        }
    b->chosen = -1;
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
