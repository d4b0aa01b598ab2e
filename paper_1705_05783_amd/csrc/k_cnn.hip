// Learned basis (extension of the B4 basis construction, Sec. 3): a 3D CNN
// maps the log-transmissibility patch of a full dual block (9x9x9 cells, the
// block and its bounding vertex planes) to the 8 basis values of its 7x7x7
// interior cells; a softmax over the 8 vertex channels gives a partition of
// unity by construction.  Edges and faces stay exact (cheap 1D/2D solves),
// so neighbouring blocks agree on shared entities; interiors whose
// local-equation residual is too large fall back to the exact solve.
//
// Layout: activations channel-major per patch x[b][c][p], p = x + 9(y + 9z);
// weights W[tap][ci][co], tap = 9(dz+1) + 3(dy+1) + (dx+1); the convolution is
// out[b][co][p] = bias[co] + sum_{tap,ci} W[tap][ci][co] x[b][ci][p + d(tap)]
// with zero padding.  Network: conv 3->32, ReLU, 32->32, ReLU, 32->32, ReLU,
// 32->8, softmax.  FP32 storage and accumulation; training convolutions on
// FP32 matrix cores, inference on BF16 matrix cores.
#include "cams_internal.h"
#include "dev_util.h"

namespace cams {

namespace {

constexpr int PD = 9;                 // patch extent
constexpr int PP = PD * PD * PD;      // 729 positions
constexpr int CT = 256;               // threads per workgroup
constexpr int MAXC = 32;
__constant__ int kLayersDev[4][2] = {{3, 32}, {32, 32}, {32, 32}, {32, 8}};

__device__ __forceinline__ int nb_pos(int p, int tap)
{
    const int x = p % PD, y = (p / PD) % PD, z = p / (PD * PD);
    const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
    const int X = x + dx, Y = y + dy, Z = z + dz;
    if (X < 0 || X >= PD || Y < 0 || Y >= PD || Z < 0 || Z >= PD) return -1;
    return X + PD * (Y + PD * Z);
}

// ---- training convolutions on FP32 matrix cores (v_mfma_f32_16x16x4f32,
// FP32 inputs and accumulation).  Operand lanes: A row = lane % 16, k =
// lane / 16; B column = lane % 16, k = lane / 16; result element v of a lane:
// row 4 (lane / 16) + v, column lane % 16.
typedef float f32x4m __attribute__((ext_vector_type(4)));
constexpr int MT = 512;               // threads of the convolution workgroup (8 waves)
constexpr int MPT = 46;               // 16-position tiles per patch (736 >= 729)
constexpr int XP = 33;                // LDS row pitch of the staged activations (banks)

// out[b][co][p] = bias[co] + conv(x) (then optional ReLU, optional
// multiplication by (mask[b][co][p] > 0)) as an implicit GEMM: one workgroup
// per (patch b, 16 output channels co0..co0+15); the patch's activations are
// staged position-major in LDS (channels padded to a multiple of 4), the
// layer's weights for the 16 channels likewise; wave w takes the position
// tiles w, w + 8, ...; per tile and tap, one MFMA per 4 input channels.
// CP: the input channels rounded up to the MFMA's k of 4 (4, 8 or 32), a
// compile-time count so that a tap's operand reads go out together.
template <int CP>
__global__ __launch_bounds__(MT) void k_conv_mfma(const float *__restrict__ x, int Ci, const float *__restrict__ W,
                                                   const float *__restrict__ bias, int Co, float *__restrict__ out,
                                                   int relu, const float *__restrict__ mask)
{
    static_assert(CP % 4 == 0 && CP <= MAXC, "channel chunks of 4");
    __shared__ float xs[MPT * 16 * XP];
    __shared__ float ws[27 * CP * 16];
    const int b = blockIdx.x, co0 = blockIdx.y * 16;
    const float *xb = x + (size_t)b * Ci * PP;
    for (int t = threadIdx.x; t < MPT * 16 * CP; t += MT) {
        const int c = t / (MPT * 16), q = t % (MPT * 16);   // coalesced along positions
        xs[q * XP + c] = (c < Ci && q < PP) ? xb[(size_t)c * PP + q] : 0.f;
    }
    for (int t = threadIdx.x; t < 27 * CP * 16; t += MT) {
        const int j = t % 16, ci = (t / 16) % CP, tap = t / (16 * CP);
        ws[t] = (ci < Ci && co0 + j < Co) ? W[((size_t)tap * Ci + ci) * Co + co0 + j] : 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int co = co0 + row;
    const float bs = (bias && co < Co) ? bias[co] : 0.f;
    for (int pt = wave; pt < MPT; pt += MT / 64) {
        const int p = pt * 16 + row;
        const int px = p % PD, py = (p / PD) % PD, pz = p / (PD * PD);
        f32x4m acc = {0.f, 0.f, 0.f, 0.f};
        // three taps' operand reads in flight at a time
#pragma unroll 3
        for (int tap = 0; tap < 27; ++tap) {
            const int X = px + tap % 3 - 1, Y = py + (tap / 3) % 3 - 1, Z = pz + tap / 9 - 1;
            const bool ok = p < PP && X >= 0 && X < PD && Y >= 0 && Y < PD && Z >= 0 && Z < PD;
            const float *xa = xs + (ok ? X + PD * (Y + PD * Z) : 0) * XP + kq;
            const float *wb = ws + (tap * CP + kq) * 16 + row;
            float av[CP / 4], bv[CP / 4];
#pragma unroll
            for (int c = 0; c < CP / 4; ++c) {
                av[c] = ok ? xa[4 * c] : 0.f;
                bv[c] = wb[4 * c * 16];
            }
#pragma unroll
            for (int c = 0; c < CP / 4; ++c) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[c], bv[c], acc, 0, 0, 0);
        }
        // element v: position pt * 16 + 4 kq + v, channel co
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int pr = pt * 16 + 4 * kq + v;
            if (pr >= PP || co >= Co) continue;
            float val = acc[v] + bs;
            if (relu) val = fmaxf(val, 0.f);
            const size_t o = ((size_t)b * Co + co) * PP + pr;
            if (mask && !(mask[o] > 0.f)) val = 0.f;
            out[o] = val;
        }
    }
}

// Partial weight gradient as per-tap GEMMs over the positions, on matrix
// cores: part[grp][tap][ci][co] = sum_{b in grp} sum_p x[b][ci][p + d(tap)]
// g[b][co][p].  Workgroup (tap, grp), 4 waves; wave w owns the 16 x 16 block
// (ci tile w / 2, co tile w % 2) of the Ci x Co result; positions are staged
// 64 at a time (x shifted by the tap, zero outside the patch), one MFMA per
// 4 positions.
__global__ __launch_bounds__(CT) void k_conv_wgrad_mfma(const float *__restrict__ x, int Ci,
                                                         const float *__restrict__ g, int Co, int B, int per_group,
                                                         float *__restrict__ part)
{
    constexpr int CH = 64;
    __shared__ float xs[CH][MAXC + 1];
    __shared__ float gs[CH][MAXC + 1];
    const int tap = blockIdx.x, grp = blockIdx.y;
    const int b0 = grp * per_group, b1 = min(B, b0 + per_group);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, kq = lane >> 4;
    const int ci = (wave >> 1) * 16 + row, co = (wave & 1) * 16 + row;   // A row / B column of this lane
    const bool active = (wave >> 1) * 16 < Ci && (wave & 1) * 16 < Co;
    f32x4m acc = {0.f, 0.f, 0.f, 0.f};
    for (int b = b0; b < b1; ++b) {
        for (int p0 = 0; p0 < PP; p0 += CH) {
            for (int t = threadIdx.x; t < MAXC * CH; t += CT) {
                const int c = t / CH, pp = t % CH, p = p0 + pp;
                float xv = 0.f, gv = 0.f;
                if (p < PP) {
                    if (c < Ci) {
                        const int q = nb_pos(p, tap);
                        if (q >= 0) xv = x[((size_t)b * Ci + c) * PP + q];
                    }
                    if (c < Co) gv = g[((size_t)b * Co + c) * PP + p];
                }
                xs[pp][c] = xv;
                gs[pp][c] = gv;
            }
            __syncthreads();
            if (active)
#pragma unroll
                for (int k4 = 0; k4 < CH; k4 += 4)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[k4 + kq][ci], gs[k4 + kq][co], acc, 0, 0, 0);
            __syncthreads();
        }
    }
    // element v: ci row 4 kq + v of the wave's ci tile, co = this lane's column
    if (active) {
        const int cot = (wave & 1) * 16 + row;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int cr = (wave >> 1) * 16 + 4 * kq + v;
            if (cr < Ci && cot < Co) part[((size_t)grp * 27 + tap) * Ci * Co + (size_t)cr * Co + cot] = acc[v];
        }
    }
}

// Weights for the input gradient: Wt[26 - tap][co][ci] = W[tap][ci][co].
__global__ __launch_bounds__(CT) void k_flip_weights(const float *__restrict__ W, int Ci, int Co,
                                                      float *__restrict__ Wt)
{
    const int t = blockIdx.x * CT + threadIdx.x;
    if (t >= 27 * Ci * Co) return;
    const int co = t % Co, ci = (t / Co) % Ci, tap = t / (Co * Ci);
    Wt[((size_t)(26 - tap) * Co + co) * Ci + ci] = W[t];
}

// grad[i] = sum over groups of part[grp][i] (fixed order).
__global__ __launch_bounds__(CT) void k_sum_groups(const float *__restrict__ part, int groups, int n,
                                                    float *__restrict__ grad)
{
    const int i = blockIdx.x * CT + threadIdx.x;
    if (i >= n) return;
    float s = 0.f;
    for (int q = 0; q < groups; ++q) s += part[(size_t)q * n + i];
    grad[i] = s;
}

// Bias gradient: sum over patches and positions, one workgroup per channel.
__global__ __launch_bounds__(CT) void k_bias_grad(const float *__restrict__ g, int Co, int B, float *__restrict__ gb)
{
    __shared__ double sh[CT / 64];
    const int co = blockIdx.x;
    double s = 0.0;
    for (int t = threadIdx.x; t < B * PP; t += CT) {
        const int b = t / PP, p = t % PP;
        s += g[((size_t)b * Co + co) * PP + p];
    }
    const double tot = block_sum<CT>(s, sh);
    if (threadIdx.x == 0) gb[co] = (float)tot;
}

__device__ __forceinline__ bool interior_pos(int p, int &ip)
{
    const int x = p % PD, y = (p / PD) % PD, z = p / (PD * PD);
    if (x < 1 || x > PD - 2 || y < 1 || y > PD - 2 || z < 1 || z > PD - 2) return false;
    ip = (x - 1) + 7 * ((y - 1) + 7 * (z - 1));
    return true;
}

// Softmax over the 8 channels; with a target: MSE over the interior cells,
// its gradient wrt the logits, and per-workgroup loss partials.
__global__ __launch_bounds__(CT) void k_softmax_mse(const float *__restrict__ logits, const float *__restrict__ target,
                                                     int B, float inv_nterm, float *__restrict__ phi,
                                                     float *__restrict__ glog, double *__restrict__ loss_part)
{
    __shared__ double sh[CT / 64];
    const int t = blockIdx.x * CT + threadIdx.x;
    double l2 = 0.0;
    if (t < B * PP) {
        const int b = t / PP, p = t % PP;
        float z[8], m = -3.0e38f;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            z[s] = logits[((size_t)b * 8 + s) * PP + p];
            m = fmaxf(m, z[s]);
        }
        float e[8], se = 0.f;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            e[s] = expf(z[s] - m);
            se += e[s];
        }
        float ph[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            ph[s] = e[s] / se;
            if (phi) phi[((size_t)b * 8 + s) * PP + p] = ph[s];
        }
        if (target && glog) {
            int ip;
            float gz[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (interior_pos(p, ip)) {
                float gp[8], dot = 0.f;
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const float d = ph[s] - target[((size_t)b * 8 + s) * 343 + ip];
                    l2 += (double)d * d;
                    gp[s] = 2.f * d * inv_nterm;
                    dot += ph[s] * gp[s];
                }
#pragma unroll
                for (int s = 0; s < 8; ++s) gz[s] = ph[s] * (gp[s] - dot);
            }
#pragma unroll
            for (int s = 0; s < 8; ++s) glog[((size_t)b * 8 + s) * PP + p] = gz[s];
        }
    }
    const double tot = block_sum<CT>(l2, sh);
    if (threadIdx.x == 0 && loss_part) loss_part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(CT) void k_loss_final(const double *__restrict__ part, int n, double scale,
                                                    double *__restrict__ loss)
{
    __shared__ double sh[CT / 64];
    double s = 0.0;
    for (int t = threadIdx.x; t < n; t += CT) s += part[t];
    const double tot = block_sum<CT>(s, sh);
    if (threadIdx.x == 0) *loss = tot * scale;
}

__global__ __launch_bounds__(CT) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, int n, float lr, float b1, float b2, float eps,
                                              float c1, float c2)
{
    const int i = blockIdx.x * CT + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Features of full dual blocks: ln T on the +x/+y/+z face of every patch cell
// (0 on the patch's last face along that axis).  Region list entries are
// interior boxes of 7x7x7 cells; the patch starts one cell before them.
__global__ __launch_bounds__(CT) void k_cnn_features(GridDev g, const double *__restrict__ T,
                                                      const Region *__restrict__ regs, float *__restrict__ feat)
{
    const int blk = blockIdx.x;
    const Region R = regs[blk];
    const int i0 = R.s[0] - 1, j0 = R.s[1] - 1, k0 = R.s[2] - 1;
    for (int p = threadIdx.x; p < PP; p += CT) {
        const int x = p % PD, y = (p / PD) % PD, z = p / (PD * PD);
        const int n = (i0 + x) + g.nx * ((j0 + y) + g.ny * (k0 + z));
        const double tx = x < PD - 1 ? T[n] : 0.0;
        const double ty = y < PD - 1 ? T[g.N + n] : 0.0;
        const double tz = z < PD - 1 ? T[2 * (size_t)g.N + n] : 0.0;
        float *f = feat + (size_t)blk * 3 * PP;
        f[p] = tx > 0.0 ? (float)log(tx) : 0.f;
        f[PP + p] = ty > 0.0 ? (float)log(ty) : 0.f;
        f[2 * PP + p] = tz > 0.0 ? (float)log(tz) : 0.f;
    }
}

// Targets: the exact basis values of the interior cells (slot s = corner s).
__global__ __launch_bounds__(CT) void k_cnn_targets(GridDev g, const double *__restrict__ P,
                                                     const Region *__restrict__ regs, float *__restrict__ tgt)
{
    const int blk = blockIdx.x;
    const Region R = regs[blk];
    for (int t = threadIdx.x; t < 8 * 343; t += CT) {
        const int s = t / 343, ip = t % 343;
        const int x = ip % 7, y = (ip / 7) % 7, z = ip / 49;
        const int n = (R.s[0] + x) + g.nx * ((R.s[1] + y) + g.ny * (R.s[2] + z));
        tgt[(size_t)blk * 8 * 343 + t] = (float)P[(size_t)s * g.N + n];
    }
}

// Write the predicted interior values into the basis.
__global__ __launch_bounds__(CT) void k_cnn_scatter(GridDev g, const float *__restrict__ phi,
                                                     const Region *__restrict__ regs, double *__restrict__ P)
{
    const int blk = blockIdx.x;
    const Region R = regs[blk];
    for (int t = threadIdx.x; t < 8 * 343; t += CT) {
        const int s = t / 343, ip = t % 343;
        const int x = ip % 7, y = (ip / 7) % 7, z = ip / 49;
        const int p = (x + 1) + PD * ((y + 1) + PD * (z + 1));
        const int n = (R.s[0] + x) + g.nx * ((R.s[1] + y) + g.ny * (R.s[2] + z));
        P[(size_t)s * g.N + n] = (double)phi[((size_t)blk * 8 + s) * PP + p];
    }
}

// Local-equation check of a predicted interior: ||(T Phi)_I|| / ||T_IF Phi_F||
// over the 8 basis functions (T the incompressible two-point operator).
// The basis is stored per cell relative to the cell's lower bracketing
// vertex: interior cells and the lower vertex planes share the block's lower
// vertex, but on an upper vertex plane the lower vertex is the block's upper
// one, so there the block's node s is slot s - bit if s has that axis' bit
// and otherwise a node whose function vanishes on the plane.
__global__ __launch_bounds__(CT) void k_block_residual(GridDev g, const double *__restrict__ T,
                                                        const double *__restrict__ P,
                                                        const Region *__restrict__ regs, double *__restrict__ ratio)
{
    __shared__ double sh[CT / 64];
    const int blk = blockIdx.x;
    const Region R = regs[blk];
    const double *Tx = T, *Ty = T + g.N, *Tz = T + 2 * (size_t)g.N;
    double num = 0.0, den = 0.0;
    for (int t = threadIdx.x; t < 8 * 343; t += CT) {
        const int s = t / 343, ip = t % 343;
        const int x = ip % 7, y = (ip / 7) % 7, z = ip / 49;
        const int i = R.s[0] + x, j = R.s[1] + y, k = R.s[2] + z;
        const int n = i + g.nx * (j + g.ny * k);
        const double *Ps = P + (size_t)s * g.N;
        const double pn = Ps[n];
        double res = 0.0, bnd = 0.0;
        const int nbr[6] = {n - 1, n + 1, n - g.nx, n + g.nx, n - g.sxy, n + g.sxy};
        const double tf[6] = {Tx[n - 1], Tx[n], Ty[n - g.nx], Ty[n], Tz[n - g.sxy], Tz[n]};
        const bool onb[6] = {x == 0, x == 6, y == 0, y == 6, z == 0, z == 6};
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            // f odd: the +x/+y/+z neighbour; on the block boundary it lies on an upper vertex plane
            const int bit = 1 << (f >> 1);
            const bool upper = (f & 1) && onb[f];
            const bool vanish = upper && !(s & bit);
            const int sj = upper && (s & bit) ? s - bit : s;
            const double pv = P[(size_t)sj * g.N + nbr[f]];
            const double pj = vanish ? 0.0 : pv;
            res += tf[f] * (pn - pj);
            if (onb[f]) bnd += tf[f] * pj;
        }
        num += res * res;
        den += bnd * bnd;
    }
    const double sn = block_sum<CT>(num, sh);
    const double sd = block_sum<CT>(den, sh);
    if (threadIdx.x == 0) ratio[blk] = sd > 0.0 ? sqrt(sn / sd) : 0.0;
}

inline unsigned cdiv_u(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- host ----

size_t cnn_num_params()
{
    return 27 * 3 * 32 + 32 + 2 * (27 * 32 * 32 + 32) + 27 * 32 * 8 + 8;
}

static const int kLayers[4][2] = {{3, 32}, {32, 32}, {32, 32}, {32, 8}};

static size_t layer_offset(int l)
{
    size_t o = 0;
    for (int q = 0; q < l; ++q) o += 27 * kLayers[q][0] * kLayers[q][1] + kLayers[q][1];
    return o;
}

// Weight-gradient partials: one group (workgroup per tap) per patch, so the
// matrix-core launch has 27 B workgroups; k_sum_groups adds them up.
static int wgrad_groups(int B) { return B; }

// Workspace (floats) for a batch of B patches: three hidden activations,
// logits, softmax output, two gradient buffers, flipped weights, partial
// weight gradients, loss partials.
size_t cnn_workspace_floats(int B)
{
    const size_t act = (size_t)B * 32 * PP;
    return 3 * act + 2 * (size_t)B * 8 * PP + 2 * act + 27 * 32 * 32 + (size_t)wgrad_groups(B) * 27 * 32 * 32 +
           2 * (size_t)cdiv_u((size_t)B * PP, CT) + 64;
}

struct CnnWs {
    float *a[3], *logits, *phi, *g0, *g1, *wflip, *part;
    double *loss_part;
};

static CnnWs carve(float *ws, int B)
{
    CnnWs w;
    const size_t act = (size_t)B * 32 * PP;
    float *q = ws;
    for (int l = 0; l < 3; ++l) { w.a[l] = q; q += act; }
    w.logits = q; q += (size_t)B * 8 * PP;
    w.phi = q; q += (size_t)B * 8 * PP;
    w.g0 = q; q += act;
    w.g1 = q; q += act;
    w.wflip = q; q += 27 * 32 * 32;
    w.part = q; q += (size_t)wgrad_groups(B) * 27 * 32 * 32;
    w.loss_part = (double *)q;
    return w;
}

// ---- inference on matrix cores (BF16 weights and activations, FP32
// accumulation): one workgroup runs the whole network for one patch with
// both activation buffers in LDS.  Each layer is an implicit GEMM:
// out[p][co] = sum over 27 taps of X[p + d(tap)][0..31] . W[tap][0..31][co],
// one v_mfma_f32_16x16x32_bf16 per (16 positions, 16 channels, tap).
// Activations are position-major with 32 channels (zero padded), so an A
// fragment (8 consecutive channels of one position) is one 16-byte LDS read;
// each wave keeps the B fragments of all 27 taps of its 16 output channels
// in registers and walks its share of the 46 position tiles.

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KC = 32;             // channels per position in the inference buffers
constexpr int NPT = 46;            // 16-position tiles per patch (736 >= 729)
constexpr int IT = 512;            // threads of the inference workgroup (8 waves)
constexpr int kWbLayer = 27 * KC * KC;   // bf16 weights per layer

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// wb[l][tap][co][ci] (co, ci padded to 32, zeros outside) from the FP32
// parameters W[tap][ci][co]; bb[l][co] FP32 biases (zero padded).
__global__ __launch_bounds__(CT) void k_prepare_bf16(const float *__restrict__ params, uint16_t *__restrict__ wb,
                                                      float *__restrict__ bb)
{
    const int t = blockIdx.x * CT + threadIdx.x;
    if (t >= 4 * kWbLayer + 4 * KC) return;
    if (t >= 4 * kWbLayer) {
        const int l = (t - 4 * kWbLayer) / KC, co = (t - 4 * kWbLayer) % KC;
        size_t off = 0;
        for (int q = 0; q < l; ++q) off += 27 * kLayersDev[q][0] * kLayersDev[q][1] + kLayersDev[q][1];
        const int Ci = kLayersDev[l][0], Co = kLayersDev[l][1];
        bb[l * KC + co] = co < Co ? params[off + 27 * Ci * Co + co] : 0.f;
        return;
    }
    const int l = t / kWbLayer, e = t % kWbLayer;
    const int tap = e / (KC * KC), co = (e / KC) % KC, ci = e % KC;
    const int Ci = kLayersDev[l][0], Co = kLayersDev[l][1];
    size_t off = 0;
    for (int q = 0; q < l; ++q) off += 27 * kLayersDev[q][0] * kLayersDev[q][1] + kLayersDev[q][1];
    const float w = (ci < Ci && co < Co) ? params[off + ((size_t)tap * Ci + ci) * Co + co] : 0.f;
    wb[t] = bf16_bits(w);
}

__global__ __launch_bounds__(IT) void k_cnn_infer(const float *__restrict__ feat, const uint16_t *__restrict__ wb,
                                                   const float *__restrict__ bb, float *__restrict__ phi)
{
    __shared__ __attribute__((aligned(16))) uint16_t bufA[NPT * 16 * KC];
    __shared__ __attribute__((aligned(16))) uint16_t bufB[NPT * 16 * KC];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // input: 3 channels of ln T, zero elsewhere (padding channels and rows)
    for (int t = threadIdx.x; t < NPT * 16 * KC; t += IT) {
        const int p = t / KC, c = t % KC;
        bufA[t] = (c < 3 && p < PP) ? bf16_bits(feat[((size_t)b * 3 + c) * PP + p]) : (uint16_t)0;
    }
    __syncthreads();
    const int row = lane & 15, kq = lane >> 4;   // A row / B column, 8-wide k slice
    for (int l = 0; l < 4; ++l) {
        const uint16_t *in = (l & 1) ? bufB : bufA;
        uint16_t *out = (l & 1) ? bufA : bufB;
        const int Co = kLayersDev[l][1];
        const int ntile_c = (Co + 15) / 16;                 // 2 (32 channels) or 1 (8)
        const int cot = wave % ntile_c, pstart = wave / ntile_c, pstep = 8 / ntile_c;
        const int co = cot * 16 + row;
        bf16x8 bw[27];
#pragma unroll
        for (int tap = 0; tap < 27; ++tap)
            bw[tap] = *(const bf16x8 *)(wb + (size_t)l * kWbLayer + ((size_t)tap * KC + co) * KC + 8 * kq);
        const float bias = bb[l * KC + co];
        for (int pt = pstart; pt < NPT; pt += pstep) {
            const int p = pt * 16 + row;
            const int x = p % PD, y = (p / PD) % PD, z = p / (PD * PD);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int tap = 0; tap < 27; ++tap) {
                const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
                const int X = x + dx, Y = y + dy, Z = z + dz;
                const bool ok = p < PP && X >= 0 && X < PD && Y >= 0 && Y < PD && Z >= 0 && Z < PD;
                const int q = ok ? X + PD * (Y + PD * Z) : 0;
                bf16x8 a = *(const bf16x8 *)(in + q * KC + 8 * kq);
                if (!ok) a = bf16x8{};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[tap], acc, 0, 0, 0);
            }
            // D element v of this lane: position pt*16 + 4 kq + v, channel co
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int pr = pt * 16 + 4 * kq + v;
                float val = acc[v] + bias;
                if (l < 3) {
                    out[pr * KC + co] = bf16_bits(fmaxf(val, 0.f));
                } else if (co < 8) {
                    ((float *)out)[pr * 8 + co] = val;   // logits, FP32
                }
            }
        }
        __syncthreads();
    }
    // softmax over the 8 channels (the last layer wrote FP32 logits [p][8] to bufA)
    const float *lg = (const float *)bufA;
    for (int p = threadIdx.x; p < PP; p += IT) {
        float m = lg[p * 8];
#pragma unroll
        for (int s = 1; s < 8; ++s) m = fmaxf(m, lg[p * 8 + s]);
        float e[8], sum = 0.f;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            e[s] = __expf(lg[p * 8 + s] - m);
            sum += e[s];
        }
        const float inv = 1.f / sum;
#pragma unroll
        for (int s = 0; s < 8; ++s) phi[((size_t)b * 8 + s) * PP + p] = e[s] * inv;
    }
}

static void conv_mfma(hipStream_t st, int B, const float *x, int Ci, const float *W, const float *bias, int Co,
                      float *out, int relu, const float *mask)
{
    dim3 grid(B, cdiv_u(Co, 16));
    if (Ci <= 4)
        k_conv_mfma<4><<<grid, MT, 0, st>>>(x, Ci, W, bias, Co, out, relu, mask);
    else if (Ci <= 8)
        k_conv_mfma<8><<<grid, MT, 0, st>>>(x, Ci, W, bias, Co, out, relu, mask);
    else
        k_conv_mfma<MAXC><<<grid, MT, 0, st>>>(x, Ci, W, bias, Co, out, relu, mask);
}

void cnn_forward(hipStream_t st, const float *params, const float *feat, int B, float *ws_f, float *phi_out)
{
    CnnWs w = carve(ws_f, B);
    const float *in = feat;
    for (int l = 0; l < 4; ++l) {
        const int Ci = kLayers[l][0], Co = kLayers[l][1];
        const float *W = params + layer_offset(l);
        const float *bias = W + 27 * Ci * Co;
        float *out = l < 3 ? w.a[l] : w.logits;
        conv_mfma(st, B, in, Ci, W, bias, Co, out, l < 3, nullptr);
        in = out;
    }
    k_softmax_mse<<<cdiv_u((size_t)B * PP, CT), CT, 0, st>>>(w.logits, nullptr, B, 0.f, phi_out ? phi_out : w.phi,
                                                             nullptr, nullptr);
}

void cnn_loss_grad(hipStream_t st, const float *params, const float *feat, const float *target, int B,
                   float *ws_f, float *grad, double *loss_out)
{
    CnnWs w = carve(ws_f, B);
    cnn_forward(st, params, feat, B, ws_f, w.phi);
    const float inv = 1.f / (float)((size_t)B * 8 * 343);
    const unsigned nb = cdiv_u((size_t)B * PP, CT);
    // g0 = d loss / d logits (stored in the logits-sized prefix of g0)
    k_softmax_mse<<<nb, CT, 0, st>>>(w.logits, target, B, inv, w.phi, w.g0, w.loss_part);
    k_loss_final<<<1, CT, 0, st>>>(w.loss_part, (int)nb, (double)inv, loss_out);
    float *gcur = w.g0, *gnext = w.g1;
    const int groups = wgrad_groups(B);
    const int per = (B + groups - 1) / groups;
    for (int l = 3; l >= 0; --l) {
        const int Ci = kLayers[l][0], Co = kLayers[l][1];
        const float *W = params + layer_offset(l);
        const float *xin = l > 0 ? w.a[l - 1] : feat;
        float *gW = grad + layer_offset(l);
        float *gb = gW + 27 * Ci * Co;
        dim3 gw(27, groups);
        k_conv_wgrad_mfma<<<gw, CT, 0, st>>>(xin, Ci, gcur, Co, B, per, w.part);
        k_sum_groups<<<cdiv_u(27 * Ci * Co, CT), CT, 0, st>>>(w.part, groups, 27 * Ci * Co, gW);
        k_bias_grad<<<Co, CT, 0, st>>>(gcur, Co, B, gb);
        if (l > 0) {
            // input gradient through the flipped kernel, masked by ReLU'(a)
            k_flip_weights<<<cdiv_u(27 * Ci * Co, CT), CT, 0, st>>>(W, Ci, Co, w.wflip);
            conv_mfma(st, B, gcur, Co, w.wflip, nullptr, Ci, gnext, 0, w.a[l - 1]);
            float *t = gcur;
            gcur = gnext;
            gnext = t;
        }
    }
}

void cnn_adam(hipStream_t st, float *p, const float *g, float *m, float *v, int n, int t, float lr, float b1,
              float b2, float eps)
{
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_adam<<<cdiv_u(n, CT), CT, 0, st>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

void cnn_features(cams_ctx *c, const Region *regs, int nblk, float *feat)
{
    if (nblk > 0) k_cnn_features<<<nblk, CT, 0, c->stream>>>(c->g, c->a.T, regs, feat);
}

void cnn_targets(cams_ctx *c, const Region *regs, int nblk, float *tgt)
{
    if (nblk > 0) k_cnn_targets<<<nblk, CT, 0, c->stream>>>(c->g, c->a.P, regs, tgt);
}

void cnn_scatter(cams_ctx *c, const Region *regs, int nblk, const float *phi)
{
    if (nblk > 0) k_cnn_scatter<<<nblk, CT, 0, c->stream>>>(c->g, phi, regs, c->a.P);
}

void cnn_block_residual(cams_ctx *c, const Region *regs, int nblk, double *ratio)
{
    if (nblk > 0) k_block_residual<<<nblk, CT, 0, c->stream>>>(c->g, c->a.T, c->a.P, regs, ratio);
}

// Bytes of the inference weights (bf16) and biases prepared by cnn_forward_bf16.
size_t cnn_bf16_bytes() { return 4 * kWbLayer * 2 + 4 * KC * 4; }

// phi_out[b][8][729] from the BF16 matrix-core path; `wb` (cnn_bf16_bytes,
// 16-byte aligned) receives the converted weights first.
void cnn_forward_bf16(hipStream_t st, const float *params, const float *feat, int B, void *wb, float *phi_out)
{
    uint16_t *w16 = (uint16_t *)wb;
    float *bias = (float *)(w16 + 4 * kWbLayer);
    k_prepare_bf16<<<cdiv_u(4 * kWbLayer + 4 * KC, CT), CT, 0, st>>>(params, w16, bias);
    if (B > 0) k_cnn_infer<<<B, IT, 0, st>>>(feat, w16, bias, phi_out);
}

}  // namespace cams
