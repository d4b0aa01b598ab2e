// C ABI of libcams: argument validation, workspace layout and the host-side
// sequencing of the C-AMS kernels (Table "cams").  All device work goes to
// the caller's stream; host reads happen only where a norm decides control
// flow (Newton and linear stopping tests).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "cams_internal.h"

using namespace cams;

namespace cams {
void launch_gemm_sub(cams_ctx *c, double *C, int ldc, const double *A, int lda, const double *B, int ldb, int M,
                     int Nn, int K);
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

cams_status fail(cams_ctx *c, cams_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

int num_blocks(int n, int r) { return (n + r - 1) / r; }

// Vertex coordinate of primal block a: start + floor(len/2).
std::vector<int32_t> vertex_coords(int n, int r)
{
    const int nb = num_blocks(n, r);
    std::vector<int32_t> v(nb);
    for (int a = 0; a < nb; ++a) {
        const int s = a * r, e = std::min((a + 1) * r, n);
        v[a] = s + (e - s) / 2;
    }
    return v;
}

struct Segment {
    int s, len;
    bool free_axis;
};

// Per axis: vertex coordinates as fixed one-cell segments and the maximal
// runs between them (including the stubs next to the domain boundary).
std::vector<Segment> segments(int n, const std::vector<int32_t> &v, bool active)
{
    std::vector<Segment> out;
    if (!active) {
        out.push_back({0, 1, false});
        return out;
    }
    int x = 0;
    for (size_t a = 0; a <= v.size(); ++a) {
        const int stop = a < v.size() ? v[a] : n;
        if (stop > x) out.push_back({x, stop - x, true});
        if (a < v.size()) out.push_back({v[a], 1, false});
        x = stop + 1;
    }
    return out;
}

// The mixed-precision solves read an FP32 copy of the dense MSFE inverse
// where the symmetric coarse GEMV runs (above kGemvLds nodes, no plane
// blocks): half the bytes per coarse solve, one rounding per factorisation.
bool uses_inverse32(const cams_options &O, bool blocktri, int nc)
{
    return O.restriction == CAMS_R_FE && !blocktri && nc > kGemvLds && O.precision != CAMS_FP64;
}

struct Layout {
    size_t *off;
    size_t total = 0;
    size_t add(size_t bytes)
    {
        size_t o = total;
        total = align_up(total + bytes);
        return o;
    }
};

void sync_status(cams_ctx *c, int32_t *flags)
{
    CAMS_HIP(hipMemcpyAsync(c->host, c->a.status, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    CAMS_HIP(hipStreamSynchronize(c->stream));
    memcpy(flags, c->host, sizeof(int32_t));
}

double read_scalar(cams_ctx *c, const double *dev)
{
    CAMS_HIP(hipMemcpyAsync(c->host, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CAMS_HIP(hipStreamSynchronize(c->stream));
    return c->host[0];
}

void clear_status(cams_ctx *c)
{
    // a one-word host-to-device copy keeps graph capture free of memset nodes
    int32_t zero[4] = {0, 0, 0, 0};
    memcpy(c->host + 8, zero, sizeof(zero));
    CAMS_HIP(hipMemcpyAsync(c->a.status, c->host + 8, sizeof(zero), hipMemcpyHostToDevice, c->stream));
}

float elapsed_ms(cams_ctx *c, int a, int b)
{
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace

namespace cams {

constexpr int kProfPairs = 4096;

void prof_begin(cams_ctx *c, double bytes, int launches)
{
    if (c->prof_used >= kProfPairs) return;   // pool full until the next collection
    if ((int)c->prof_ev.size() < 2 * (c->prof_used + 1)) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return;
        if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return; }
        c->prof_ev.push_back(e0);
        c->prof_ev.push_back(e1);
    }
    if ((int)c->prof_tag.size() <= c->prof_used) {
        c->prof_tag.push_back(0);
        c->prof_bytes_pair.push_back(0.0);
        c->prof_count_pair.push_back(0);
    }
    c->prof_tag[c->prof_used] = c->prof_iter;
    c->prof_bytes_pair[c->prof_used] = bytes;
    c->prof_count_pair[c->prof_used] = launches;
    (void)hipEventRecord(c->prof_ev[2 * c->prof_used], c->stream);
}

void prof_end(cams_ctx *c)
{
    if (c->prof_used >= kProfPairs) return;
    (void)hipEventRecord(c->prof_ev[2 * c->prof_used + 1], c->stream);
    ++c->prof_used;
}

// After a stream synchronisation: add up the recorded pairs whose iteration
// index is below `valid_below` (later ones returned early after convergence).
static void prof_collect(cams_ctx *c, int valid_below)
{
    for (int q = 0; q < c->prof_used; ++q) {
        if (c->prof_tag[q] >= valid_below) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->prof_ev[2 * q], c->prof_ev[2 * q + 1]) != hipSuccess) continue;
        c->prof_ms += ms;
        c->prof_bytes += c->prof_bytes_pair[q];
        c->prof_launches += c->prof_count_pair[q];
    }
    c->prof_used = 0;
}

// Learned scratch layout: [feat | phi | ratio | fallback regions | network workspace (chunk)].
static size_t learned_scratch_need(const cams_ctx *c)
{
    const size_t nf = (size_t)c->nfull;
    return align_up(nf * 3 * 729 * 4) + align_up(nf * 8 * 729 * 4) + align_up(nf * 8) +
           align_up(nf * sizeof(Region)) + align_up(cnn_bf16_bytes());
}

// Basis with the network predicting the interiors of full dual blocks:
// vertices, edges and faces exact; stub interiors exact; full interiors from
// the network, then the local-equation check and exact re-solves of the
// blocks whose ratio exceeds fallback_tol.
static void build_basis_learned(cams_ctx *c)
{
    char *s = c->learned_scratch;
    const size_t nf = (size_t)c->nfull;
    float *feat = (float *)s;
    s += align_up(nf * 3 * 729 * 4);
    float *phi = (float *)s;
    s += align_up(nf * 8 * 729 * 4);
    double *ratio = (double *)s;
    s += align_up(nf * 8);
    Region *fb = (Region *)s;
    s += align_up(nf * sizeof(Region));
    float *ws = (float *)s;
    launch_basis_vertices(c);
    for (int nfree = 1; nfree <= 2; ++nfree)
        launch_basis_regions(c, nfree, c->a.regions + c->regoff[nfree], c->nreg[nfree]);
    const Region *full = c->a.regions + c->regoff[3];
    launch_basis_regions(c, 3, full + c->nfull, c->nreg[3] - c->nfull);   // stubs
    cnn_features(c, full, c->nfull, feat);
    // inference on matrix cores (BF16 weights and activations, FP32 accumulation)
    cnn_forward_bf16(c->stream, c->learned_params, feat, c->nfull, ws, phi);
    cnn_scatter(c, full, c->nfull, phi);
    cnn_block_residual(c, full, c->nfull, ratio);
    std::vector<double> &r = c->block_ratio;
    r.assign(nf, 0.0);
    CAMS_HIP(hipMemcpyAsync(r.data(), ratio, nf * 8, hipMemcpyDeviceToHost, c->stream));
    CAMS_HIP(hipStreamSynchronize(c->stream));
    std::vector<Region> host_full(c->regions.begin() + c->regoff[3], c->regions.begin() + c->regoff[3] + c->nfull);
    c->fallback_list.clear();
    for (size_t b = 0; b < nf; ++b)
        if (!(r[b] <= c->fallback_tol)) c->fallback_list.push_back(host_full[b]);
    c->learned_blocks = c->nfull - (int)c->fallback_list.size();
    c->fallback_blocks = (int)c->fallback_list.size();
    if (!c->fallback_list.empty()) {
        CAMS_HIP(hipMemcpyAsync(fb, c->fallback_list.data(), c->fallback_list.size() * sizeof(Region),
                                hipMemcpyHostToDevice, c->stream));
        launch_basis_regions(c, 3, fb, (int)c->fallback_list.size());
        CAMS_HIP(hipStreamSynchronize(c->stream));   // the host list must outlive the copy
    }
}

}  // namespace cams

extern "C" {

const char *cams_status_string(cams_status s)
{
    switch (s) {
    case CAMS_OK: return "ok";
    case CAMS_E_ARG: return "invalid argument";
    case CAMS_E_STATE: return "call out of order";
    case CAMS_E_DEVICE: return "HIP runtime error";
    case CAMS_E_NOMEM: return "workspace missing or too small";
    case CAMS_E_NOT_CONVERGED: return "not converged";
    case CAMS_E_BREAKDOWN: return "numerical breakdown";
    }
    return "unknown status";
}

const char *cams_last_error(const cams_ctx *c) { return c ? c->err.c_str() : "null context"; }

cams_status cams_create(const cams_grid *grid, const cams_fluid *fluid, const cams_options *opt, void *hip_stream,
                        cams_ctx **out)
{
    if (!out) return CAMS_E_ARG;
    *out = nullptr;
    if (!grid || !fluid || !opt) return CAMS_E_ARG;
    const cams_grid &G = *grid;
    const bool three_d = G.nz > 1;
    const int n[3] = {G.nx, G.ny, G.nz};
    int r[3] = {G.rx, G.ry, three_d ? G.rz : 1};
    for (int a = 0; a < 3; ++a) {
        const bool active = a < 2 || three_d;
        if (!active) {
            if (n[a] != 1) return CAMS_E_ARG;
            continue;
        }
        if (n[a] < 2 || r[a] < 2 || r[a] > kMaxRatio || r[a] > n[a]) return CAMS_E_ARG;
        std::vector<int32_t> v = vertex_coords(n[a], r[a]);
        for (size_t b = 1; b < v.size(); ++b)
            if (v[b] - v[b - 1] < 2) return CAMS_E_ARG;  // adjacent vertex lines are not supported
    }
    const double N = (double)G.nx * G.ny * G.nz;
    if (N > 2.0e9) return CAMS_E_ARG;
    if (!(G.dx > 0) || !(G.dy > 0) || !(G.dz > 0)) return CAMS_E_ARG;
    const cams_fluid &F = *fluid;
    if (!(F.rho0 > 0) || !(F.c >= 0) || !(F.mu > 0) || !(F.dt > 0) || !isfinite(F.p0) || !isfinite(F.c))
        return CAMS_E_ARG;
    const cams_options &O = *opt;
    if (O.restriction != CAMS_R_FV && O.restriction != CAMS_R_FE) return CAMS_E_ARG;
    if (O.n_pre < 0 || O.n_pre > 64 || O.n_post < 0 || O.n_post > 64) return CAMS_E_ARG;
    if (O.precision != CAMS_FP64 && O.precision != CAMS_MIXED_FP32 && O.precision != CAMS_MIXED_BF16)
        return CAMS_E_ARG;
    if (O.smoother != CAMS_SMOOTH_BLOCK_ILU0 && O.smoother != CAMS_SMOOTH_RB_ILU0 &&
        O.smoother != CAMS_SMOOTH_BLOCK_ALT_ILU0 && O.smoother != CAMS_SMOOTH_NAT_ILU0)
        return CAMS_E_ARG;
    if (O.precision != CAMS_FP64 && !block_smoother(O)) return CAMS_E_ARG;
    if (!(O.lin_rtol > 0) || O.lin_maxit < 1 || !(O.newton_tol > 0) || O.newton_maxit < 1) return CAMS_E_ARG;
    if (!(O.lin_atol >= 0) || !isfinite(O.lin_atol)) return CAMS_E_ARG;
    if (O.basis_type < CAMS_BASIS_B4 || O.basis_type > CAMS_BASIS_B3 || !(O.basis_tol >= 0)) return CAMS_E_ARG;
    if (!(O.coarse_tol >= 0)) return CAMS_E_ARG;
    const int nb[3] = {num_blocks(n[0], r[0]), num_blocks(n[1], r[1]), num_blocks(n[2], r[2])};
    const double Nc = (double)nb[0] * nb[1] * nb[2];
    if (Nc > 32768) return CAMS_E_ARG;  // dense coarse operator limit

    cams_ctx *c = new (std::nothrow) cams_ctx();
    if (!c) return CAMS_E_NOMEM;
    c->grid = G;
    c->grid.rz = r[2];
    c->fluid = F;
    c->opt = O;
    c->stream = (hipStream_t)hip_stream;
    GridDev &g = c->g;
    g.nx = G.nx; g.ny = G.ny; g.nz = G.nz;
    g.N = G.nx * G.ny * G.nz;
    g.sxy = G.nx * G.ny;
    g.dx = G.dx; g.dy = G.dy; g.dz = G.dz;
    g.dV = G.dx * G.dy * G.dz;
    for (int a = 0; a < 3; ++a) { g.nb[a] = nb[a]; g.r[a] = r[a]; }
    g.Nc = nb[0] * nb[1] * nb[2];
    g.dim = three_d ? 3 : 2;
    // large MSFE coarse grids: block-tridiagonal elimination over z-planes
    c->blocktri = O.restriction == CAMS_R_FE && three_d && g.Nc > kBlockTriMin && nb[2] >= 3;
    c->fl = {F.rho0, F.c, F.p0, F.mu, F.dt};

    // per-axis tables: vc (nb), lo (n), isv (n, stored as int32)
    cams_ctx &t = *c;
    std::vector<Segment> seg[3];
    for (int a = 0; a < 3; ++a) {
        std::vector<int32_t> v = (a < 2 || three_d) ? vertex_coords(n[a], r[a]) : std::vector<int32_t>{0};
        t.tab_off[a][0] = t.tab.size();
        for (int32_t x : v) t.tab.push_back(x);
        t.tab_off[a][1] = t.tab.size();
        for (int x = 0; x < n[a]; ++x) {
            int lo = 0;
            for (size_t b = 0; b < v.size(); ++b)
                if (v[b] <= x) lo = (int)b;
            t.tab.push_back(lo);
        }
        t.tab_off[a][2] = t.tab.size();
        // isv packed 4 per int32 word (uint8 view)
        std::vector<uint8_t> isv(n[a], 0);
        for (int32_t x : v) isv[x] = 1;
        const size_t words = (n[a] + 3) / 4;
        size_t base = t.tab.size();
        t.tab.resize(base + words, 0);
        memcpy(t.tab.data() + base, isv.data(), n[a]);
        seg[a] = segments(n[a], v, a < 2 || three_d);
        // restriction-owner boxes: primal blocks (MSFV) or [v_a, v_{a+1}) with
        // the first box starting at 0 and the last ending at n (MSFE)
        t.tab_off[a][3] = t.tab.size();
        const int nba = (int)v.size();
        for (int b = 0; b <= nba; ++b) {
            int x;
            if (O.restriction == CAMS_R_FV) x = std::min(b * r[a], n[a]);
            else x = b == 0 ? 0 : (b == nba ? n[a] : v[b]);
            t.tab.push_back(x);
        }
    }
    // x-groups of boxes for the row form of the residual-restriction: greedy,
    // at most kRowBoxes boxes and kRowCells cells per group
    {
        const int nbx = nb[0];
        std::vector<int32_t> obx(t.tab.begin() + t.tab_off[0][3], t.tab.begin() + t.tab_off[0][3] + nbx + 1);
        for (int v = 0; v < 2; ++v) {
            auto xs = [&](int b) { return v == 1 ? obx[b] : std::min(b * r[0], n[0]); };
            std::vector<int32_t> starts{0};
            bool ok = true;
            for (int b = 0; b < nbx && ok; ++b) {
                if (xs(b + 1) - xs(b) > kRowCells) ok = false;
                const int g0 = starts.back();
                if (b > g0 && (b + 1 - g0 > kRowBoxes || xs(b + 1) - xs(g0) > kRowCells)) starts.push_back(b);
            }
            starts.push_back(nbx);
            if (!ok) {   // cannot happen with ratios up to kMaxRatio (boxes of at most 12 cells)
                delete c;
                return CAMS_E_ARG;
            }
            t.tab_gx[v] = t.tab.size();
            c->g.ngx[v] = (int)starts.size() - 1;
            bool even = n[0] % 2 == 0;
            for (int b = 0; b <= nbx; ++b) even = even && xs(b) % 2 == 0;
            t.row_pairs[v] = even;
            for (int32_t x : starts) t.tab.push_back(x);
        }
    }
    // dual regions by number of open axes
    std::vector<Region> by[4];
    for (const Segment &sz : seg[2])
        for (const Segment &sy : seg[1])
            for (const Segment &sx : seg[0]) {
                int fm = (sx.free_axis ? 1 : 0) | (sy.free_axis ? 2 : 0) | (sz.free_axis ? 4 : 0);
                int nf = __builtin_popcount(fm);
                if (nf == 0) continue;
                Region R;
                R.s[0] = sx.s; R.s[1] = sy.s; R.s[2] = sz.s;
                R.len[0] = sx.len; R.len[1] = sy.len; R.len[2] = sz.len;
                R.freemask = fm;
                R.pad = 0;
                by[nf].push_back(R);
            }
    // interiors that are full dual blocks (7x7x7 at ratio 8) first: the
    // learned basis predicts exactly those
    std::stable_partition(by[3].begin(), by[3].end(),
                          [](const Region &R) { return R.len[0] == 7 && R.len[1] == 7 && R.len[2] == 7; });
    c->nfull = 0;
    for (const Region &R : by[3])
        if (R.len[0] == 7 && R.len[1] == 7 && R.len[2] == 7) ++c->nfull;
    int off = 0;
    for (int f = 0; f < 4; ++f) {
        c->nreg[f] = (int)by[f].size();
        c->regoff[f] = off;
        off += c->nreg[f];
        c->maxm[f] = 1;
        c->maxbw[f] = 1;
        for (const Region &R : by[f]) {
            t.regions.push_back(R);
            // local system size and bandwidth (stride of the last open axis)
            const int st[3] = {1, R.len[0], R.len[0] * R.len[1]};
            int bw = 1;
            for (int a = 0; a < 3; ++a)
                if (R.freemask & (1 << a)) bw = st[a];
            c->maxm[f] = std::max(c->maxm[f], R.len[0] * R.len[1] * R.len[2]);
            c->maxbw[f] = std::max(c->maxbw[f], bw);
        }
    }
    c->region_total = off;
    if (O.basis_type == CAMS_BASIS_B1 || O.basis_type == CAMS_BASIS_B2) {
        // which regions take a region's values as Dirichlet data: a region's
        // cells reach, across its open axes, cells of lower-dimensional
        // regions (edges for faces, faces for interiors)
        std::vector<int32_t> rid((size_t)g.N, -1);
        const int nx = G.nx, ny = G.ny, nz = G.nz;
        auto for_cells = [&](const Region &R, auto fn) {
            for (int z = R.s[2]; z < R.s[2] + R.len[2]; ++z)
                for (int y = R.s[1]; y < R.s[1] + R.len[1]; ++y)
                    for (int x = R.s[0]; x < R.s[0] + R.len[0]; ++x) fn(x, y, z);
        };
        for (int q = 0; q < off; ++q)
            for_cells(t.regions[q], [&](int x, int y, int z) { rid[x + (size_t)nx * (y + (size_t)ny * z)] = q; });
        std::vector<std::vector<int32_t>> dep(off);
        for (int q = 0; q < off; ++q) {
            const Region &R = t.regions[q];
            for_cells(R, [&](int x, int y, int z) {
                const int xyz[3] = {x, y, z}, nn[3] = {nx, ny, nz};
                for (int a = 0; a < 3; ++a) {
                    if (!(R.freemask & (1 << a))) continue;
                    for (int dir = -1; dir <= 1; dir += 2) {
                        int v[3] = {xyz[0], xyz[1], xyz[2]};
                        v[a] += dir;
                        if (v[a] < 0 || v[a] >= nn[a] || (v[a] >= R.s[a] && v[a] < R.s[a] + R.len[a])) continue;
                        const int r = rid[v[0] + (size_t)nx * (v[1] + (size_t)ny * v[2])];
                        if (r >= 0 && r != q) dep[r].push_back(q);
                    }
                }
            });
        }
        c->dep_ptr.assign(1, 0);
        c->dep_idx.clear();
        for (int q = 0; q < off; ++q) {
            std::sort(dep[q].begin(), dep[q].end());
            dep[q].erase(std::unique(dep[q].begin(), dep[q].end()), dep[q].end());
            c->dep_idx.insert(c->dep_idx.end(), dep[q].begin(), dep[q].end());
            c->dep_ptr.push_back((int32_t)c->dep_idx.size());
        }
    }

    // workspace layout
    Layout L;
    L.off = c->off;
    constexpr int kMaxArrays = (int)(sizeof(c->off) / sizeof(c->off[0]));
    int k = 0;
    auto put = [&](size_t o) {
        if (k < kMaxArrays) c->off[k] = o;
        ++k;
    };
    const size_t n8 = (size_t)g.N * 8;
    const size_t nc = (size_t)g.Nc;
    c->nparts = std::max((g.N + kBlock - 1) / kBlock, g.Nc);
    put(L.add(3 * n8));        // 0 T
    put(L.add(n8));            // 1 phi
    put(L.add(n8));            // 2 q
    put(L.add(3 * n8));        // 3 W
    put(L.add(n8));            // 4 diag
    put(L.add(n8));            // 5 r0
    put(L.add(n8));            // 6 r
    put(L.add(n8));            // 7 dp0
    put(L.add(n8));            // 8 dp1
    put(L.add(n8));            // 9 d0
    put(L.add(n8));            // 10 d1
    put(L.add(n8));            // 11 d2
    put(L.add(n8));            // 12 z
    put(L.add(n8));            // 13 x
    const size_t npiv = O.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0 ? 2 : 1;   // pivot sets
    put(L.add(npiv * n8));     // 14 invd
    put(L.add(8 * n8));        // 15 P
    put(L.add(nc * nc * 8));   // 16 Ac
    put(L.add(nc * nc * 8));   // 17 Ainv
    put(L.add(nc * nc * 8));   // 18 work
    put(L.add(nc * 8));        // 19 rc
    put(L.add(nc * 8));        // 20 xc
    put(L.add((size_t)c->nparts * 8));  // 21 partial
    put(L.add(64 * 8));        // 22 scal
    put(L.add(nc * 2 * 4));    // 23 piv + perm
    put(L.add(64 * 4));        // 24 status
    put(L.add((size_t)g.N));   // 25 dmask
    const size_t wcap = (size_t)g.N / 8 + 64;
    put(L.add(wcap * 4));      // 26 wcell
    put(L.add(wcap * 8));      // 27 wp
    put(L.add(t.tab.size() * 4));            // 28 tables
    put(L.add(t.regions.size() * sizeof(Region) + 16));  // 29 regions
    put(L.add(nc * 8 * 8));    // 30 restriction slot sums
    put(L.add((nc + 64) * 4));   // 31 iteration control
    put(L.add(O.restriction == CAMS_R_FE ? nc * 216 * 8 : 0));   // 32 coarse-operator box partials
    const bool mixed = O.precision != CAMS_FP64;
    const size_t n4 = mixed ? (size_t)g.N * 4 : 0;
    put(L.add(3 * n4));        // 33 W32
    put(L.add(n4));            // 34 diag32
    put(L.add(npiv * n4));     // 35 invd32
    put(L.add(O.precision == CAMS_MIXED_FP32 ? 8 * n4 : 0));   // 36 P32
    put(L.add(O.precision == CAMS_MIXED_BF16 ? 4 * n4 : 0));   // 37 Pbf (8 x 2 bytes per cell)
    put(L.add(n4));            // 38 r1f
    put(L.add(n4));            // 39 d0f
    put(L.add(n4));            // 40 d1f
    put(L.add(n4));            // 41 d2f
    put(L.add(n4));            // 42 zf
    put(L.add(0));             // 43 (unused)
    {   // 44 Gauss-Jordan GEMM descriptors (MSFE): 8 per 64-column panel of each inverted matrix
        const size_t mats = c->blocktri ? (size_t)nb[2] : 1, dim = c->blocktri ? (size_t)nb[0] * nb[1] : nc;
        put(L.add(O.restriction == CAMS_R_FE ? mats * ((dim + 63) / 64) * 12 * sizeof(GemmDesc) : 0));
        put(L.add(O.restriction == CAMS_R_FE ? (c->blocktri ? 2 : 1) * (5 * dim * 64 + 64 * 64) * 8 : 0));   // 45 old column blocks, their transposes, G (per chain)
    }
    {   // 46-51 basis types B1-B3
        const bool pdep = O.basis_type == CAMS_BASIS_B1 || O.basis_type == CAMS_BASIS_B2;
        const bool diag = O.basis_type == CAMS_BASIS_B1 || O.basis_type == CAMS_BASIS_B3;
        const size_t nreg = (size_t)c->region_total;
        put(L.add(pdep ? 3 * n8 : 0));                  // 46 bcoef
        put(L.add(diag ? n8 : 0));                      // 47 bdiag
        put(L.add(pdep ? 3 * n8 : 0));                  // 48 bsnap
        put(L.add(pdep && diag ? n8 : 0));              // 49 bdsnap
        put(L.add(pdep ? nreg * 4 : 0));                // 50 rflag
        put(L.add(pdep ? nreg * sizeof(Region) : 0));   // 51 rlist
    }
    put(L.add((size_t)2 * G.ny * G.nz * 8));   // 52 Tb: west and east boundary-face transmissibilities
    put(L.add(O.coarse_tol > 0 ? nc * 27 * 8 : 0));   // 53 Acs: coarse operator at its last factorisation
    {   // 54 tile partials of the symmetric coarse GEMV (dense MSFE inverses above kGemvLds nodes)
        const size_t T = (nc + 63) / 64;
        put(L.add(O.restriction == CAMS_R_FE && !c->blocktri && nc > (size_t)kGemvLds ? T * T * 64 * 8 : 0));
        // 55 its FP32 copy for the mixed-precision solves
        put(L.add(uses_inverse32(O, c->blocktri, (int)nc) ? nc * nc * 4 : 0));
    }
    if (k > kMaxArrays) {  // more arrays than offset slots: a build error, never a silent overflow
        delete c;
        return CAMS_E_NOMEM;
    }
    c->need = L.total;

    *out = c;
    return CAMS_OK;
}

size_t cams_workspace_bytes(const cams_ctx *c) { return c ? c->need : 0; }

int64_t cams_num_coarse(const cams_ctx *c) { return c ? c->g.Nc : 0; }

int32_t cams_coarse_planes(const cams_ctx *c) { return c && c->blocktri ? c->g.nb[2] : 0; }

cams_status cams_set_workspace(cams_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c || !dev_ptr) return CAMS_E_ARG;
    if (((uintptr_t)dev_ptr) % kAlign) return fail(c, CAMS_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < c->need) return fail(c, CAMS_E_NOMEM, "workspace too small");
    const size_t *off = c->off;
    char *w = (char *)dev_ptr;
    Arrays &a = c->a;
    const int N = c->g.N;
    a.T = (double *)(w + off[0]);
    a.phi = (double *)(w + off[1]);
    a.q = (double *)(w + off[2]);
    a.W = (double *)(w + off[3]);
    a.diag = (double *)(w + off[4]);
    a.r0 = (double *)(w + off[5]);
    a.r = (double *)(w + off[6]);
    a.dp[0] = (double *)(w + off[7]);
    a.dp[1] = (double *)(w + off[8]);
    a.d0 = (double *)(w + off[9]);
    a.d1 = (double *)(w + off[10]);
    a.d2 = (double *)(w + off[11]);
    a.z = (double *)(w + off[12]);
    a.x = (double *)(w + off[13]);
    a.invd = (double *)(w + off[14]);
    a.P = (double *)(w + off[15]);
    a.Ac = (double *)(w + off[16]);
    a.Ainv = (double *)(w + off[17]);
    a.work = (double *)(w + off[18]);
    a.rc = (double *)(w + off[19]);
    a.xc = (double *)(w + off[20]);
    a.partial = (double *)(w + off[21]);
    a.scal = (double *)(w + off[22]);
    a.piv = (int32_t *)(w + off[23]);
    a.status = (int32_t *)(w + off[24]);
    a.dmask = (uint8_t *)(w + off[25]);
    a.wcell = (int32_t *)(w + off[26]);
    a.wp = (double *)(w + off[27]);
    a.tab = (int32_t *)(w + off[28]);
    a.regions = (Region *)(w + off[29]);
    a.slots = (double *)(w + off[30]);
    a.boxp = (double *)(w + off[32]);
    a.ictl = (int32_t *)(w + off[31]);
    a.W32 = (float *)(w + off[33]);
    a.diag32 = (float *)(w + off[34]);
    a.invd32 = (float *)(w + off[35]);
    a.P32 = (float *)(w + off[36]);
    a.Pbf = (uint16_t *)(w + off[37]);
    a.r1f = (float *)(w + off[38]);
    a.d0f = (float *)(w + off[39]);
    a.d1f = (float *)(w + off[40]);
    a.d2f = (float *)(w + off[41]);
    a.zf = (float *)(w + off[42]);
    a.gjd = (void *)(w + off[44]);
    a.gjcb = (double *)(w + off[45]);
    a.bcoef = (double *)(w + off[46]);
    a.bdiag = (double *)(w + off[47]);
    a.bsnap = (double *)(w + off[48]);
    a.bdsnap = (double *)(w + off[49]);
    a.rflag = (int32_t *)(w + off[50]);
    a.rlist = (Region *)(w + off[51]);
    a.Tb = (double *)(w + off[52]);
    a.Acs = (double *)(w + off[53]);
    a.gpart = (double *)(w + off[54]);
    a.Ainv32 = uses_inverse32(c->opt, c->blocktri, c->g.Nc) ? (float *)(w + off[55]) : nullptr;
    c->ainv32_ok = false;
    if (!c->host) {
        // first device interaction of the context: pinned scalars and timers
        if (hipHostMalloc((void **)&c->host, 4096, hipHostMallocDefault) != hipSuccess) {
            c->host = nullptr;
            return fail(c, CAMS_E_DEVICE, "hipHostMalloc of the scalar buffer failed");
        }
        for (int e = 0; e < 8; ++e)
            if (hipEventCreate(&c->ev[e]) != hipSuccess) c->ev[e] = nullptr;
        // the second elimination chain of the block-tridiagonal factorisation
        // (default priority); without it both chains run on the caller's stream
        if (c->blocktri) {
            if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) c->side = nullptr;
            if (c->side && (hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
                            hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess)) {
                if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
                (void)hipStreamDestroy(c->side);
                c->side = nullptr;
                c->fork_ev = nullptr;
            }
        }
    }
    const cams_ctx &t = *c;
    for (int ax = 0; ax < 3; ++ax) {
        c->g.vc[ax] = a.tab + t.tab_off[ax][0];
        c->g.lo[ax] = a.tab + t.tab_off[ax][1];
        c->g.isv[ax] = (const uint8_t *)(a.tab + t.tab_off[ax][2]);
        c->g.ob[ax] = a.tab + t.tab_off[ax][3];
    }
    for (int v = 0; v < 2; ++v) c->g.gx[v] = a.tab + t.tab_gx[v];
    try {
        CAMS_HIP(hipMemcpyAsync(a.tab, t.tab.data(), t.tab.size() * 4, hipMemcpyHostToDevice, c->stream));
        if (!t.regions.empty())
            CAMS_HIP(hipMemcpyAsync(a.regions, t.regions.data(), t.regions.size() * sizeof(Region),
                                    hipMemcpyHostToDevice, c->stream));
        std::vector<uint8_t> zero((size_t)N, 0);
        CAMS_HIP(hipMemcpyAsync(a.dmask, zero.data(), (size_t)N, hipMemcpyHostToDevice, c->stream));
        std::vector<int32_t> zctl((size_t)c->g.Nc + 64, 0);
        CAMS_HIP(hipMemcpyAsync(a.ictl, zctl.data(), zctl.size() * 4, hipMemcpyHostToDevice, c->stream));
        // absolute linear tolerance, squared, for the device stopping test
        std::vector<double> zscal(64, 0.0);
        zscal[S_ATOL2] = c->opt.lin_atol * c->opt.lin_atol;
        CAMS_HIP(hipMemcpyAsync(a.scal, zscal.data(), zscal.size() * 8, hipMemcpyHostToDevice, c->stream));
        clear_status(c);
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("set_workspace: ") + hipGetErrorString(e.code));
    }
    c->ws = w;
    c->ws_bytes = bytes;
    c->has_ws = true;
    c->has_rock = c->has_basis = c->has_system = c->has_coarse = c->has_bcoef = c->has_cfac = false;
    c->ac_zeroed = false;
    c->gj_ready = false;
    c->nwells = 0;
    return CAMS_OK;
}

cams_status cams_set_rock(cams_ctx *c, const double *perm_dev, const double *phi_dev, const double *q_dev)
{
    if (!c) return CAMS_E_ARG;
    if (!c->has_ws) return fail(c, CAMS_E_STATE, "set_rock before set_workspace");
    if (!perm_dev || !phi_dev) return fail(c, CAMS_E_ARG, "perm and phi are required");
    const size_t nb = (size_t)c->g.N * 8;
    try {
        clear_status(c);
        launch_check_rock(c, perm_dev, phi_dev);
        CAMS_HIP(hipMemcpyAsync(c->a.phi, phi_dev, nb, hipMemcpyDeviceToDevice, c->stream));
        if (q_dev) CAMS_HIP(hipMemcpyAsync(c->a.q, q_dev, nb, hipMemcpyDeviceToDevice, c->stream));
        launch_transmissibility(c, perm_dev);
        CAMS_HIP(hipGetLastError());
        int32_t flags = 0;
        sync_status(c, &flags);
        if (flags & F_BAD_INPUT) return fail(c, CAMS_E_ARG, "permeability must be > 0, porosity in (0,1]");
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("set_rock: ") + hipGetErrorString(e.code));
    }
    c->has_q = q_dev != nullptr;
    c->has_rock = true;
    c->has_basis = c->has_system = c->has_coarse = false;
    c->learned_suspended = false;
    return CAMS_OK;
}

cams_status cams_invalidate_basis(cams_ctx *c)
{
    if (!c) return CAMS_E_ARG;
    c->has_basis = c->has_coarse = false;
    return CAMS_OK;
}

cams_status cams_set_wells(cams_ctx *c, const int64_t *cells, const double *p, int32_t n)
{
    if (!c) return CAMS_E_ARG;
    if (!c->has_ws) return fail(c, CAMS_E_STATE, "set_wells before set_workspace");
    const size_t wcap = (size_t)c->g.N / 8 + 64;
    if (n < 0 || (size_t)n > wcap || (n > 0 && (!cells || !p))) return fail(c, CAMS_E_ARG, "bad well list");
    if (n == 0 && !(c->fl.c > 0) && !c->bc.on[0] && !c->bc.on[1])
        return fail(c, CAMS_E_ARG, "no wells, no Dirichlet face and c = 0: singular system");
    std::vector<uint8_t> mask((size_t)c->g.N, 0);
    std::vector<int32_t> ci(n);
    std::vector<double> pv(n);
    for (int t = 0; t < n; ++t) {
        if (cells[t] < 0 || cells[t] >= c->g.N || !isfinite(p[t])) return fail(c, CAMS_E_ARG, "bad well cell");
        if (mask[cells[t]]) return fail(c, CAMS_E_ARG, "duplicate well cell");
        mask[cells[t]] = 1;
        ci[t] = (int32_t)cells[t];
        pv[t] = p[t];
    }
    try {
        CAMS_HIP(hipMemcpyAsync(c->a.dmask, mask.data(), mask.size(), hipMemcpyHostToDevice, c->stream));
        if (n > 0) {
            CAMS_HIP(hipMemcpyAsync(c->a.wcell, ci.data(), (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
            CAMS_HIP(hipMemcpyAsync(c->a.wp, pv.data(), (size_t)n * 8, hipMemcpyHostToDevice, c->stream));
        }
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("set_wells: ") + hipGetErrorString(e.code));
    }
    c->nwells = n;
    c->has_system = c->has_coarse = false;
    return CAMS_OK;
}

}  // extern "C"

namespace cams {

// Device work of the setup phases, enqueued without host synchronisation;
// shared by the single-problem entry points and the batched solve.
void enqueue_assemble(cams_ctx *c, const double *p, const double *pn)
{
    launch_assemble(c, p, pn);
    launch_reduce(c, c->a.partial, (c->g.N + kBlock - 1) / kBlock, c->a.scal + S_EPS2);
}

void enqueue_basis_local(cams_ctx *c)
{
    launch_basis(c);
    if (c->opt.precision != CAMS_FP64) launch_round_basis(c);
}

void enqueue_coarse_operator(cams_ctx *c)
{
    launch_coarse_operator(c);
    launch_ilu_setup(c);
    if (c->opt.precision != CAMS_FP64) launch_convert_matrix32(c);
}

void enqueue_coarse(cams_ctx *c)
{
    enqueue_coarse_operator(c);
    launch_coarse_factor(c);
}

void enqueue_clear_status(cams_ctx *c) { clear_status(c); }

}  // namespace cams

// B1/B2 adaptive update (Sec. 4.1.2, adaptive updating of the multiscale
// operators): re-solve the dual regions whose local coefficients changed by
// more than basis_tol since their last solve (every region when basis_tol
// is 0), and every region that takes a re-solved region's values as
// boundary data; the others keep their basis values.  Returns the number
// of regions re-solved.
static int update_basis_adaptive(cams_ctx *c)
{
    const int first = c->regoff[1], count = c->region_total - first;
    const double tol = c->opt.basis_tol;
    std::vector<int32_t> flag((size_t)count, 1);
    if (tol > 0) {
        launch_region_change(c, first, count, tol);
        CAMS_HIP(hipMemcpyAsync(flag.data(), c->a.rflag + first, (size_t)count * 4, hipMemcpyDeviceToHost,
                                c->stream));
        CAMS_HIP(hipStreamSynchronize(c->stream));
        // regions are listed by stage and depend only on earlier stages: one
        // forward pass carries the marks through edges, faces and interiors
        for (int q = 0; q < count; ++q)
            if (flag[q])
                for (int32_t e = c->dep_ptr[first + q]; e < c->dep_ptr[first + q + 1]; ++e)
                    flag[c->dep_idx[e] - first] = 1;
    }
    std::vector<Region> list;
    int per[4] = {0, 0, 0, 0};
    for (int f = 1; f <= c->g.dim; ++f)
        for (int q = c->regoff[f]; q < c->regoff[f] + c->nreg[f]; ++q)
            if (flag[q - first]) {
                list.push_back(c->regions[q]);
                ++per[f];
            }
    if (list.empty()) return 0;
    clear_status(c);
    CAMS_HIP(hipMemcpyAsync(c->a.rlist, list.data(), list.size() * sizeof(Region), hipMemcpyHostToDevice, c->stream));
    int at = 0;
    for (int f = 1; f <= c->g.dim; ++f) {
        launch_basis_regions(c, f, c->a.rlist + at, per[f]);
        at += per[f];
    }
    launch_region_snapshot(c, c->a.rlist, (int)list.size());
    if (c->opt.precision != CAMS_FP64) launch_round_basis(c);
    CAMS_HIP(hipGetLastError());
    CAMS_HIP(hipStreamSynchronize(c->stream));   // the host list must outlive the copy
    return (int)list.size();
}

static cams_status check_basis_status(cams_ctx *c)
{
    int32_t flags = 0;
    sync_status(c, &flags);
    if (flags) return fail(c, CAMS_E_BREAKDOWN, "basis: non-positive local pivot or inconsistent region");
    return CAMS_OK;
}

extern "C" {

cams_status cams_assemble(cams_ctx *c, const double *p_dev, const double *pn_dev, double *eps_norm_out)
{
    if (!c) return CAMS_E_ARG;
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "assemble before set_rock");
    if (!p_dev || !pn_dev) return fail(c, CAMS_E_ARG, "null pressure");
    try {
        enqueue_assemble(c, p_dev, pn_dev);
        if (c->opt.basis_type == CAMS_BASIS_B1 || c->opt.basis_type == CAMS_BASIS_B2) {
            launch_basis_coeffs(c, p_dev, pn_dev);   // local-problem coefficients at this iterate
            c->has_bcoef = true;
        }
        CAMS_HIP(hipGetLastError());
        if (eps_norm_out) {
            double e2 = read_scalar(c, c->a.scal + S_EPS2);
            *eps_norm_out = sqrt(e2);
            c->last.eps_norm_last = *eps_norm_out;
        }
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("assemble: ") + hipGetErrorString(e.code));
    }
    c->has_system = true;
    c->has_coarse = false;
    return CAMS_OK;
}

cams_status cams_build_basis(cams_ctx *c)
{
    if (!c) return CAMS_E_ARG;
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "build_basis before set_rock");
    const int kind = c->opt.basis_type;
    if ((kind == CAMS_BASIS_B1 || kind == CAMS_BASIS_B2) && !c->has_bcoef)
        return fail(c, CAMS_E_STATE, "pressure-dependent basis (B1/B2): assemble at an iterate first");
    try {
        if (kind == CAMS_BASIS_B3) launch_basis_coeffs(c, nullptr, nullptr);
        clear_status(c);
        c->learned_blocks = c->fallback_blocks = 0;
        c->block_ratio.clear();
        if (c->learned_params && c->nfull > 0 && !c->learned_suspended) {
            build_basis_learned(c);
            if (c->opt.precision != CAMS_FP64) launch_round_basis(c);
        } else {
            enqueue_basis_local(c);
        }
        CAMS_HIP(hipGetLastError());
        int32_t flags = 0;
        sync_status(c, &flags);
        if (flags) return fail(c, CAMS_E_BREAKDOWN, "basis: non-positive local pivot or inconsistent region");
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("build_basis: ") + hipGetErrorString(e.code));
    }
    c->has_basis = true;
    c->has_coarse = c->has_cfac = false;
    return CAMS_OK;
}

cams_status cams_coarse_op(cams_ctx *c)
{
    if (!c) return CAMS_E_ARG;
    if (!c->has_basis) return fail(c, CAMS_E_STATE, "coarse_op before build_basis");
    if (!c->has_system) return fail(c, CAMS_E_STATE, "coarse_op before assemble");
    try {
        clear_status(c);
        enqueue_coarse_operator(c);
        // adaptive coarse factorisation: keep the last inverse while the
        // operator's entries stay within coarse_tol of the factorised ones
        bool factor = true;
        if (c->opt.coarse_tol > 0 && c->has_cfac) {
            launch_coarse_change(c, false);
            const double chg = read_scalar(c, c->a.scal + S_CCHG);
            factor = !(chg <= c->opt.coarse_tol);
        }
        if (factor) {
            launch_coarse_factor(c);
            if (c->opt.coarse_tol > 0) launch_coarse_change(c, true);
            c->has_cfac = true;
            ++c->n_factor;
        }
        CAMS_HIP(hipGetLastError());
        int32_t flags = 0;
        sync_status(c, &flags);
        if (flags & F_SINGULAR_COARSE) {
            c->has_cfac = false;
            return fail(c, CAMS_E_BREAKDOWN, "singular coarse operator");
        }
        if (flags & F_BAD_PIVOT) return fail(c, CAMS_E_BREAKDOWN, "non-positive ILU(0) pivot");
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("coarse_op: ") + hipGetErrorString(e.code));
    }
    c->has_coarse = true;
    return CAMS_OK;
}

cams_status cams_smooth_apply(cams_ctx *c, const double *z, double *x)
{
    if (!c || !z || !x) return CAMS_E_ARG;
    if (!c->has_coarse) return fail(c, CAMS_E_STATE, "smoother factor is built by coarse_op");
    try {
        launch_smooth(c, z, x, c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0 ? 2 : 1, nullptr);
        CAMS_HIP(hipGetLastError());
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("smooth_apply: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

// Enqueue one C-AMS iteration (Table "cams" steps 2, 5-7).  The residual
// kernel of iteration `it` reads dp[it % 2], folds in the corrections of the
// previous iteration and writes dp[(it + 1) % 2]; it also decides on the
// device whether to stop.  Every other kernel returns at once when the
// stop flag is set, so iterations enqueued past convergence cost only their
// launches.
static void enqueue_iteration(cams_ctx *c, int it)
{
    c->prof_iter = it;
    const cams_options &O = c->opt;
    Arrays &a = c->a;
    const int32_t *done = a.ictl + 1;
    // The block smoother's post-smoothing runs on A e = r from e = d1 (the
    // prolongated coarse correction) instead of on A d2 = r - A d1 from zero:
    // the same iterates, e = d1 + d2, without forming r1.  The correction
    // folded into the next residual is then d0 + e.
    // Without pre-smoothing the restriction acts on the new residual and is
    // computed by the residual kernel itself (partials per owner box); the
    // stopping test runs with the coarse solve.
    const int flat_parts = (c->g.N + kBlock - 1) / kBlock;
    if (O.precision != CAMS_FP64) {
        // FP64 residual and update; FP32 corrections (iterative refinement)
        const float *pend0 = O.n_pre > 0 ? a.d0f : nullptr;
        const float *pend1 = O.n_post > 0 ? a.d2f : a.d1f;
        if (O.n_pre > 0) {
            launch_residual_ctl32(c, a.dp[it & 1], pend0, pend1, nullptr, a.dp[(it + 1) & 1], a.r1f);
            launch_finalize_ctl(c, flat_parts);
            launch_bilu_smooth32(c, (const double *)a.r, a.d0f, O.n_pre, done);
            launch_sub64_lo(c, a.d0f, a.r, done);
            launch_restrict(c, a.r);
            launch_gemv(c, a.rc, a.xc, done);
        } else {
            // the stopping test runs with the coarse solve
            launch_residual_restrict32(c, a.dp[it & 1], pend0, pend1, nullptr, a.dp[(it + 1) & 1], a.r1f);
            launch_gemv(c, a.rc, a.xc, done, c->g.Nc);
        }
        if (O.n_post > 0 && bilu_first_fused(c)) {   // Eq. (12) inside the first smoothing step
            launch_bilu_smooth32_from_coarse(c, (const float *)a.r1f, a.d2f, O.n_post, done);
            return;
        }
        launch_prolong32(c, a.xc, a.d1f, done);
        if (O.n_post > 0) launch_bilu_smooth32(c, (const float *)a.r1f, a.d2f, O.n_post, done, a.d1f);
        return;
    }
    const bool block = block_smoother(O);
    const double *pend0 = O.n_pre > 0 ? a.d0 : nullptr;
    const double *pend1 = O.n_post > 0 && block ? a.d2 : a.d1;
    const double *pend2 = O.n_post > 0 && !block ? a.d2 : nullptr;
    if (O.n_pre > 0) {
        launch_residual_ctl(c, a.dp[it & 1], pend0, pend1, pend2, a.dp[(it + 1) & 1]);
        launch_finalize_ctl(c, flat_parts);
        launch_smooth(c, a.r, a.d0, O.n_pre, done);
        launch_stencil_sub(c, a.r, a.d0, a.r, done);
        launch_restrict(c, a.r);
        launch_gemv(c, a.rc, a.xc, done);              // Eq. (15): coarse solve
    } else {
        launch_residual_restrict(c, a.dp[it & 1], pend0, pend1, pend2, a.dp[(it + 1) & 1]);
        launch_gemv(c, a.rc, a.xc, done, c->g.Nc);     // Eq. (15), with the stopping test
    }
    if (O.n_post > 0 && block && bilu_first_fused(c)) {
        launch_bilu_smooth_from_coarse(c, a.r, a.d2, O.n_post, done);   // Eq. (12) inside the first step
        return;
    }
    launch_prolong(c, a.xc, a.d1, done);               // Eq. (12)
    if (O.n_post > 0) {
        if (block) {
            launch_bilu_smooth(c, a.r, a.d2, O.n_post, done, a.d1);
        } else {
            launch_stencil_sub(c, a.r, a.d1, a.r, done);   // r1 = r - A d1
            launch_smooth(c, a.r, a.d2, O.n_post, done);
        }
    }
}

cams_status cams_iterate(cams_ctx *c, double *p_dev, cams_stats *stats)
{
    if (!c) return CAMS_E_ARG;
    if (!p_dev) return fail(c, CAMS_E_ARG, "null pressure");
    if (!c->has_coarse) return fail(c, CAMS_E_STATE, "iterate before coarse_op");
    const cams_options &O = c->opt;
    const int N = c->g.N;
    Arrays &a = c->a;
    int it = 0, outcome = 0;
    double nr0 = 0.0, nr = 0.0;
    try {
        launch_iter_reset(c);
        int launched = 0, ahead = 4;
        double prev_nr = -1.0;
        // stagnation: the residual norm has not fallen below kStagDrop times
        // its best value for kStagWindow iterations
        double best_nr = -1.0;
        int it_best = 0;
        // the red-black and natural-order smoother kernels have no stop
        // flag: check every iteration; so does a norm history (one entry
        // per iteration)
        const bool sync_each = !block_smoother(O) || c->hist;
        for (;;) {
            const int batch = sync_each ? 1 : ahead;
            for (int q = 0; q < batch && launched <= O.lin_maxit; ++q) enqueue_iteration(c, launched++);
            int32_t ctl[3];
            CAMS_HIP(hipMemcpyAsync(c->host + 16, a.ictl, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            CAMS_HIP(hipMemcpyAsync(c->host + 20, a.scal + S_R0N2, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream));
            CAMS_HIP(hipStreamSynchronize(c->stream));
            memcpy(ctl, c->host + 16, sizeof(ctl));
            nr0 = sqrt(c->host[20]);
            nr = sqrt(c->host[21]);
            it = ctl[0];
            if (c->hist) {
                // the last residual kernel wrote the accumulated update to
                // dp[it & 1] (or dp[(it + 1) & 1] when it stopped there):
                // nonlinear error at p + that update
                cams_history &h = *c->hist;
                const double *dpl = a.dp[ctl[1] ? ((it + 1) & 1) : (it & 1)];
                launch_eps_at(c, h.p, dpl, h.pn, a.scal + S_EPSH);
                CAMS_HIP(hipMemcpyAsync(c->host + 24, a.scal + S_EPSH, sizeof(double), hipMemcpyDeviceToHost,
                                        c->stream));
                CAMS_HIP(hipStreamSynchronize(c->stream));
                if (h.count < h.cap) {
                    h.res[h.count] = nr;
                    h.err[h.count] = sqrt(c->host[24]);
                    h.newton[h.count] = h.nu;
                }
                ++h.count;
            }
            if (ctl[1]) {
                outcome = ctl[2];
                break;
            }
            if (launched > O.lin_maxit) {  // cannot happen: the device stops at lin_maxit
                outcome = 1;
                break;
            }
            if (best_nr < 0.0 || nr < kStagDrop * best_nr) {
                best_nr = nr;
                it_best = it;
            } else if (it - it_best >= kStagWindow) {
                // Nothing is in flight (the stream was synchronised): the
                // last residual kernel, of iteration it - 1, wrote dp[it & 1];
                // report that iterate, as at the iteration limit.
                it -= 1;
                outcome = 3;
                break;
            }
            // enqueue about as many iterations as the observed rate needs
            if (prev_nr > 0.0 && nr < prev_nr && nr0 > 0.0) {
                const double rate = pow(nr / prev_nr, 1.0 / std::max(1, batch));
                const double need = log(std::max(O.lin_rtol * nr0, O.lin_atol) / nr) / log(rate);
                ahead = (int)std::min(32.0, std::max(2.0, ceil(need)));
            }
            prev_nr = nr;
        }
        launch_axpy(c, p_dev, a.dp[(it + 1) & 1], N);
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipStreamSynchronize(c->stream));
        if (c->prof_kernel) prof_collect(c, it);
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("iterate: ") + hipGetErrorString(e.code));
    }
    c->last.lin_iters_last = it;
    c->last.relres_last = nr0 > 0 ? nr / nr0 : 0.0;
    if (stats) {
        stats->lin_iters_last = it;
        stats->relres_last = c->last.relres_last;
    }
    if (outcome == 1) return fail(c, CAMS_E_NOT_CONVERGED, "linear iteration limit reached");
    if (outcome == 3) return fail(c, CAMS_E_NOT_CONVERGED, "linear iterations stagnated");
    if (outcome == 2) return fail(c, CAMS_E_BREAKDOWN, "non-finite residual norm");
    return CAMS_OK;
}

cams_status cams_newton_step(cams_ctx *c, const double *pn_dev, double *p_dev, cams_stats *stats)
{
    if (!c) return CAMS_E_ARG;
    if (!pn_dev || !p_dev) return fail(c, CAMS_E_ARG, "null pressure");
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "newton_step before set_rock");
    cams_stats st;
    memset(&st, 0, sizeof(st));
    cams_status s = CAMS_OK;
    c->n_factor = 0;
    try {
        launch_impose_wells(c, p_dev);
        CAMS_HIP(hipGetLastError());
        // B1/B2 depend on the iterate: built after the first assembly and
        // updated adaptively at every Newton iteration (below)
        const bool pdep = c->opt.basis_type == CAMS_BASIS_B1 || c->opt.basis_type == CAMS_BASIS_B2;
        if (!c->has_basis && !pdep) {
            CAMS_HIP(hipEventRecord(c->ev[0], c->stream));
            s = cams_build_basis(c);
            if (s != CAMS_OK) return s;
            CAMS_HIP(hipEventRecord(c->ev[1], c->stream));
            CAMS_HIP(hipEventSynchronize(c->ev[1]));
            st.t_basis_ms = elapsed_ms(c, 0, 1);
            st.basis_regions_rebuilt = c->region_total;
        }
        st.fallback_blocks = c->fallback_blocks;
        for (int nit = 0;; ++nit) {
            double en = 0.0;
            CAMS_HIP(hipEventRecord(c->ev[2], c->stream));
            s = cams_assemble(c, p_dev, pn_dev, &en);
            if (s != CAMS_OK) break;
            CAMS_HIP(hipEventRecord(c->ev[3], c->stream));
            CAMS_HIP(hipEventSynchronize(c->ev[3]));
            st.t_assemble_ms += elapsed_ms(c, 2, 3);
            st.eps_norm_last = en;
            if (!isfinite(en)) { s = fail(c, CAMS_E_BREAKDOWN, "non-finite nonlinear error"); break; }
            if (en <= c->opt.newton_tol) break;
            if (nit >= c->opt.newton_maxit) { s = fail(c, CAMS_E_NOT_CONVERGED, "Newton iteration limit"); break; }
            if (pdep) {
                CAMS_HIP(hipEventRecord(c->ev[0], c->stream));
                int rebuilt = c->region_total;
                if (!c->has_basis) {
                    s = cams_build_basis(c);
                } else {
                    rebuilt = update_basis_adaptive(c);
                    st.basis_updates += 1;
                    s = check_basis_status(c);
                }
                if (s != CAMS_OK) break;
                CAMS_HIP(hipEventRecord(c->ev[1], c->stream));
                CAMS_HIP(hipEventSynchronize(c->ev[1]));
                st.t_basis_ms += elapsed_ms(c, 0, 1);
                st.basis_regions_rebuilt += rebuilt;
                c->has_coarse = false;
            }
            s = cams_coarse_op(c);
            if (s != CAMS_OK) break;
            if (c->hist) c->hist->nu = nit;
            CAMS_HIP(hipEventRecord(c->ev[4], c->stream));
            cams_stats ls;
            memset(&ls, 0, sizeof(ls));
            s = cams_iterate(c, p_dev, &ls);
            CAMS_HIP(hipEventRecord(c->ev[5], c->stream));
            CAMS_HIP(hipEventSynchronize(c->ev[5]));
            st.t_coarse_ms += elapsed_ms(c, 3, 4);
            st.t_iterate_ms += elapsed_ms(c, 4, 5);
            st.newton_iters += 1;
            st.lin_iters_total += ls.lin_iters_last;
            st.lin_iters_last = ls.lin_iters_last;
            st.relres_last = ls.relres_last;
            // global check of the learned basis: a solve that needs more
            // than twice the exact basis' iterations, or does not converge,
            // replaces the network's basis by local solves from here on
            if (c->learned_params && c->nfull > 0 && !c->learned_suspended && c->guard_iters > 0 &&
                (s == CAMS_E_NOT_CONVERGED || ls.lin_iters_last > 2 * c->guard_iters)) {
                c->learned_suspended = true;
                CAMS_HIP(hipEventRecord(c->ev[0], c->stream));
                s = cams_build_basis(c);
                if (s != CAMS_OK) break;
                CAMS_HIP(hipEventRecord(c->ev[1], c->stream));
                CAMS_HIP(hipEventSynchronize(c->ev[1]));
                st.t_basis_ms += elapsed_ms(c, 0, 1);
                st.basis_regions_rebuilt += c->region_total;
                st.basis_rebuilds += 1;
                continue;   // the next Newton iteration assembles at the iterate reached
            }
            if (s != CAMS_OK) break;
        }
    } catch (const HipError &e) {
        s = fail(c, CAMS_E_DEVICE, std::string("newton_step: ") + hipGetErrorString(e.code));
    }
    st.coarse_factorizations = c->n_factor;
    c->last = st;
    if (stats) *stats = st;
    return s;
}

cams_status cams_set_face_dirichlet(cams_ctx *c, int32_t face, double pressure)
{
    if (!c) return CAMS_E_ARG;
    if (face != 0 && face != 1) return fail(c, CAMS_E_ARG, "face must be 0 (west, x = 0) or 1 (east)");
    if (isnan(pressure)) {
        c->bc.on[face] = 0;
    } else {
        if (!isfinite(pressure)) return fail(c, CAMS_E_ARG, "face pressure must be finite (NaN removes it)");
        c->bc.on[face] = 1;
        c->bc.p[face] = pressure;
    }
    c->has_system = c->has_coarse = false;
    return CAMS_OK;
}

cams_status cams_conservative_sweep(cams_ctx *c, const double *pn_dev, double *p_dev, double *flux_dev)
{
    if (!c) return CAMS_E_ARG;
    if (!pn_dev || !p_dev || !flux_dev) return fail(c, CAMS_E_ARG, "null pressure or flux array");
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "conservative_sweep before set_rock");
    if (c->blocktri)
        return fail(c, CAMS_E_ARG, "conservative_sweep needs the dense coarse inverse (at most 4096 coarse nodes)");
    if (!c->has_basis) {
        const cams_status s = cams_build_basis(c);
        if (s != CAMS_OK) return s;
    }
    const int32_t restriction = c->opt.restriction;
    try {
        clear_status(c);
        launch_iter_reset(c);                 // clears the stop flag the restriction tests
        enqueue_assemble(c, p_dev, pn_dev);
        // the MSFV coarse operator R^FV A P_hat and its inverse (LU with partial pivoting)
        c->opt.restriction = CAMS_R_FV;
        launch_coarse_operator(c);
        launch_coarse_factor(c);
        // one multiscale stage on r0: d = P_hat (R^FV A P_hat)^-1 R^FV r0
        launch_restrict(c, c->a.r0);
        launch_gemv(c, c->a.rc, c->a.xc, nullptr, 0);
        c->opt.restriction = restriction;
        launch_prolong(c, c->a.xc, c->a.d1, nullptr);
        launch_face_flux(c, p_dev, c->a.d1, flux_dev);
        launch_axpy(c, p_dev, c->a.d1, c->g.N);
        CAMS_HIP(hipGetLastError());
        int32_t flags = 0;
        sync_status(c, &flags);
        if (flags & F_SINGULAR_COARSE) {
            c->has_coarse = c->has_system = false;
            return fail(c, CAMS_E_BREAKDOWN, "singular MSFV coarse operator");
        }
    } catch (const HipError &e) {
        c->opt.restriction = restriction;
        c->has_coarse = c->has_system = false;
        return fail(c, CAMS_E_DEVICE, std::string("conservative_sweep: ") + hipGetErrorString(e.code));
    }
    // the coarse factor now holds the MSFV inverse, and p has moved
    c->has_coarse = c->has_system = c->has_cfac = false;
    return CAMS_OK;
}

cams_status cams_newton_history(cams_ctx *c, const double *pn_dev, double *p_dev, double *res_host,
                                double *err_host, int32_t *newton_host, int32_t cap, int32_t *count,
                                cams_stats *stats)
{
    if (!c) return CAMS_E_ARG;
    if (cap < 0 || !count || (cap > 0 && (!res_host || !err_host || !newton_host)))
        return fail(c, CAMS_E_ARG, "history buffers");
    cams_history h;
    h.res = res_host;
    h.err = err_host;
    h.newton = newton_host;
    h.cap = cap;
    h.count = 0;
    h.nu = 0;
    h.p = p_dev;
    h.pn = pn_dev;
    c->hist = &h;
    const cams_status s = cams_newton_step(c, pn_dev, p_dev, stats);
    c->hist = nullptr;
    *count = h.count;
    return s;
}

size_t cams_array_bytes(const cams_ctx *c, cams_array which)
{
    if (!c) return 0;
    const size_t N = c->g.N, Nc = c->g.Nc;
    switch (which) {
    case CAMS_ARR_T: case CAMS_ARR_W: return 3 * N * 8;
    case CAMS_ARR_DIAG: case CAMS_ARR_R0: return N * 8;
    case CAMS_ARR_INVD: return N * 8 * (c->opt.smoother == CAMS_SMOOTH_BLOCK_ALT_ILU0 ? 2 : 1);
    case CAMS_ARR_P: return 8 * N * 8;
    case CAMS_ARR_AC: case CAMS_ARR_AC_INV: return Nc * Nc * 8;
    }
    return 0;
}

cams_status cams_import_basis(cams_ctx *c, const void *src, size_t bytes)
{
    if (!c || !src) return CAMS_E_ARG;
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "import_basis before set_rock");
    if (c->opt.basis_type != CAMS_BASIS_B4 && c->opt.basis_type != CAMS_BASIS_B3)
        return fail(c, CAMS_E_ARG, "only the pressure-independent bases (B3, B4) can be imported");
    if (bytes != cams_array_bytes(c, CAMS_ARR_P)) return fail(c, CAMS_E_ARG, "basis must hold 8 N doubles");
    try {
        CAMS_HIP(hipMemcpyAsync(c->a.P, src, bytes, hipMemcpyDeviceToDevice, c->stream));
        if (c->opt.precision != CAMS_FP64) launch_round_basis(c);
        CAMS_HIP(hipGetLastError());
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("import_basis: ") + hipGetErrorString(e.code));
    }
    c->learned_blocks = c->fallback_blocks = 0;
    c->block_ratio.clear();
    c->has_basis = true;
    c->has_coarse = c->has_cfac = false;
    return CAMS_OK;
}

cams_status cams_export(cams_ctx *c, cams_array which, void *dst, size_t bytes)
{
    if (!c || !dst) return CAMS_E_ARG;
    if (!c->has_ws) return fail(c, CAMS_E_STATE, "no workspace");
    const size_t need = cams_array_bytes(c, which);
    if (need == 0 || bytes < need) return fail(c, CAMS_E_ARG, "bad array or size");
    const void *src = nullptr;
    switch (which) {
    case CAMS_ARR_T: src = c->a.T; break;
    case CAMS_ARR_W: src = c->a.W; break;
    case CAMS_ARR_DIAG: src = c->a.diag; break;
    case CAMS_ARR_R0: src = c->a.r0; break;
    case CAMS_ARR_P: src = c->a.P; break;
    case CAMS_ARR_AC: src = c->a.Ac; break;
    case CAMS_ARR_AC_INV: src = c->a.Ainv; break;
    case CAMS_ARR_INVD: src = c->a.invd; break;
    }
    try {
        CAMS_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, c->stream));
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("export: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

// Test hook of the coarse factorisation's matrix-core GEMM: C -= A B with
// row-major device matrices (C: M x Nn, A: M x K, B: K x Nn, dense).
cams_status cams_debug_gemm_sub(cams_ctx *c, double *C, const double *A, const double *B, int M, int Nn, int K)
{
    if (!c || !C || !A || !B || M <= 0 || Nn <= 0 || K <= 0) return CAMS_E_ARG;
    try {
        launch_gemm_sub(c, C, Nn, A, K, B, Nn, M, Nn, K);
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("gemm: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

cams_status cams_debug_coarse_solve(cams_ctx *c, const double *rc, double *xc)
{
    if (!c || !rc || !xc) return CAMS_E_ARG;
    if (!c->has_coarse) return fail(c, CAMS_E_STATE, "coarse solve before coarse_op");
    try {
        launch_coarse_solve(c, rc, xc);
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("coarse solve: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

int64_t cams_cnn_num_params(void) { return (int64_t)cnn_num_params(); }

size_t cams_cnn_workspace_bytes(int32_t batch) { return batch > 0 ? cnn_workspace_floats(batch) * 4 : 0; }

cams_status cams_cnn_forward(void *stream, const float *params, const float *feat, int32_t batch, void *ws,
                             float *phi)
{
    if (!params || !feat || !ws || !phi || batch <= 0) return CAMS_E_ARG;
    cnn_forward((hipStream_t)stream, params, feat, batch, (float *)ws, phi);
    return hipGetLastError() == hipSuccess ? CAMS_OK : CAMS_E_DEVICE;
}

size_t cams_cnn_bf16_workspace_bytes(void) { return cnn_bf16_bytes(); }

cams_status cams_cnn_forward_bf16(void *stream, const float *params, const float *feat, int32_t batch, void *ws,
                                  float *phi)
{
    if (!params || !feat || !ws || !phi || batch <= 0 || ((uintptr_t)ws & 15)) return CAMS_E_ARG;
    cnn_forward_bf16((hipStream_t)stream, params, feat, batch, ws, phi);
    return hipGetLastError() == hipSuccess ? CAMS_OK : CAMS_E_DEVICE;
}

cams_status cams_cnn_loss_grad(void *stream, const float *params, const float *feat, const float *target,
                               int32_t batch, void *ws, float *grad, double *loss)
{
    if (!params || !feat || !target || !ws || !grad || !loss || batch <= 0) return CAMS_E_ARG;
    cnn_loss_grad((hipStream_t)stream, params, feat, target, batch, (float *)ws, grad, loss);
    return hipGetLastError() == hipSuccess ? CAMS_OK : CAMS_E_DEVICE;
}

cams_status cams_cnn_adam(void *stream, float *params, const float *grad, float *m, float *v, int32_t n,
                          int32_t step, float lr, float beta1, float beta2, float eps)
{
    if (!params || !grad || !m || !v || n <= 0 || step < 1) return CAMS_E_ARG;
    cnn_adam((hipStream_t)stream, params, grad, m, v, n, step, lr, beta1, beta2, eps);
    return hipGetLastError() == hipSuccess ? CAMS_OK : CAMS_E_DEVICE;
}

int32_t cams_cnn_num_blocks(const cams_ctx *c) { return c ? c->nfull : 0; }

cams_status cams_cnn_patches(cams_ctx *c, float *feat, float *target)
{
    if (!c || !feat) return CAMS_E_ARG;
    if (!c->has_rock) return fail(c, CAMS_E_STATE, "patches before set_rock");
    if (target && !c->has_basis) return fail(c, CAMS_E_STATE, "targets need a built basis");
    try {
        const Region *full = c->a.regions + c->regoff[3];
        cnn_features(c, full, c->nfull, feat);
        if (target) cnn_targets(c, full, c->nfull, target);
        CAMS_HIP(hipGetLastError());
        CAMS_HIP(hipStreamSynchronize(c->stream));
    } catch (const HipError &e) {
        return fail(c, CAMS_E_DEVICE, std::string("cnn_patches: ") + hipGetErrorString(e.code));
    }
    return CAMS_OK;
}

size_t cams_learned_scratch_bytes(const cams_ctx *c) { return c ? learned_scratch_need(c) : 0; }

cams_status cams_set_learned(cams_ctx *c, const float *params, void *scratch, size_t bytes, double fallback_tol)
{
    if (!c) return CAMS_E_ARG;
    if (!params) {
        c->learned_params = nullptr;
        c->has_basis = c->has_coarse = false;
        return CAMS_OK;
    }
    if (c->g.dim != 3 || c->g.r[0] != 8 || c->g.r[1] != 8 || c->g.r[2] != 8)
        return fail(c, CAMS_E_ARG, "the learned basis needs coarsening ratio 8 on a 3D grid");
    if (c->opt.basis_type != CAMS_BASIS_B4) return fail(c, CAMS_E_ARG, "the learned basis predicts B4 bases only");
    if (!scratch || ((uintptr_t)scratch) % kAlign || bytes < learned_scratch_need(c) || !(fallback_tol > 0))
        return fail(c, CAMS_E_ARG, "learned basis: scratch missing, misaligned or too small, or bad tolerance");
    c->learned_params = params;
    c->learned_scratch = (char *)scratch;
    c->learned_scratch_bytes = bytes;
    c->fallback_tol = fallback_tol;
    c->learned_suspended = false;
    c->has_basis = c->has_coarse = false;
    return CAMS_OK;
}

cams_status cams_set_learned_guard(cams_ctx *c, int32_t plain_iters)
{
    if (!c) return CAMS_E_ARG;
    if (plain_iters < 0) return fail(c, CAMS_E_ARG, "plain_iters must be >= 0 (0: no global check)");
    c->guard_iters = plain_iters;
    return CAMS_OK;
}

cams_status cams_basis_block_ratios(const cams_ctx *c, double *ratio_host, int32_t n)
{
    if (!c || !ratio_host || n < 0) return CAMS_E_ARG;
    if ((size_t)n > c->block_ratio.size()) return CAMS_E_STATE;
    memcpy(ratio_host, c->block_ratio.data(), (size_t)n * sizeof(double));
    return CAMS_OK;
}

cams_status cams_basis_stats(const cams_ctx *c, int32_t *learned_blocks, int32_t *fallback_blocks)
{
    if (!c || !learned_blocks || !fallback_blocks) return CAMS_E_ARG;
    *learned_blocks = c->learned_blocks;
    *fallback_blocks = c->fallback_blocks;
    return CAMS_OK;
}

cams_status cams_profile(cams_ctx *c, int kernel)
{
    if (!c || (kernel != CAMS_PROF_NONE && kernel != CAMS_PROF_SMOOTH_STEP)) return CAMS_E_ARG;
    c->prof_kernel = kernel;
    c->prof_used = 0;
    c->prof_ms = c->prof_bytes = 0.0;
    c->prof_launches = 0;
    return CAMS_OK;
}

cams_status cams_profile_read(cams_ctx *c, double *total_ms, int64_t *launches, double *bytes)
{
    if (!c || !total_ms || !launches || !bytes) return CAMS_E_ARG;
    *total_ms = c->prof_ms;
    *launches = c->prof_launches;
    *bytes = c->prof_bytes;
    return CAMS_OK;
}

cams_status cams_destroy(cams_ctx *c)
{
    if (!c) return CAMS_E_ARG;
    if (c->host) (void)hipHostFree(c->host);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    for (int e = 0; e < 8; ++e)
        if (c->ev[e]) (void)hipEventDestroy(c->ev[e]);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipEventDestroy(c->fork_ev);
        (void)hipEventDestroy(c->join_ev);
        (void)hipStreamDestroy(c->side);
    }
    delete c;
    return CAMS_OK;
}

}  // extern "C"
