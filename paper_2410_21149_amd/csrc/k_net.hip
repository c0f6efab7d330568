// Learned pose proposal for submap alignment: a small 3-D convolutional
// network on coarse ESDF summaries, trained and run with hand-written
// kernels.  (Not part of the paper; it proposes the initial pose that the
// correspondence-free ESDF alignment of Sec. III-F then refines.)
//
// Network (input 32^3 x 4 channels, NDHWC):
//   conv 3x3x3, 4 -> 16, stride 1 (32^3), ReLU
//   conv 3x3x3, 16 -> 32, stride 2 (16^3), ReLU
//   conv 3x3x3, 32 -> 64, stride 2 (8^3), ReLU
//   conv 3x3x3, 64 -> 64, stride 2 (4^3), ReLU
//   global mean -> fully connected 64 -> 5 (tx, ty, tz, cos yaw, sin yaw)
// Convolutions (zero padding 1) run as implicit GEMMs on the bf16 matrix
// cores (v_mfma_f32_16x16x16_bf16): bf16 activations and weights, FP32
// accumulation, bias and ReLU in FP32, outputs rounded to bf16 (nearest
// even).  FP32 master weights; the backward pass and Adam run in FP32.
#include "covox_impl.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

namespace covox {

namespace {

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// binary32 -> bfloat16, round to nearest even (NaN kept quiet).
__host__ __device__ inline uint16_t f2bf(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7F800000u) == 0x7F800000u && (x & 0x7FFFFFu)) return (uint16_t)((x >> 16) | 0x40);
    const uint32_t lsb = (x >> 16) & 1u;
    x += 0x7FFFu + lsb;
    return (uint16_t)(x >> 16);
}

__host__ __device__ inline float bf2f(uint16_t h)
{
    const uint32_t x = (uint32_t)h << 16;
    float f;
    memcpy(&f, &x, 4);
    return f;
}

struct ConvShape {
    int cin, cout, din, dout, stride;
    constexpr int K() const { return 27 * cin; }
};

constexpr int kLayers = 4;
constexpr ConvShape kShapes[kLayers] = {{4, 16, 32, 32, 1}, {16, 32, 32, 16, 2}, {32, 64, 16, 8, 2}, {64, 64, 8, 4, 2}};
constexpr int kOut = 5;
constexpr int kFeat = 64;

// ------------------------------------------------------------ forward

__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// One wave computes a tile of 16 positions x 16 CT output channels: per K
// chunk of 16 it loads its A fragment (the im2col row slice) once and runs
// one MFMA per 16 output channels.  With CT = COUT / 16 a workgroup of 4
// waves covers 64 positions; a layer with few positions takes CT = 1, so
// that its waves split the output channels.  The K chunks are summed in
// order for every output, whatever CT.  MFMA operand layout (16x16x16
// bf16): lane l supplies A[m = l % 16][k = 4 (l / 16) + i] and B[k = 4 (l /
// 16) + i][n = l % 16], i = 0..3, and receives D[m = 4 (l / 16) + i][n = l %
// 16].
template <int CIN, int COUT, int DIN, int DOUT, int STRIDE, int CT>
__global__ __launch_bounds__(256) void k_conv_fwd(const uint16_t *__restrict__ x, const uint16_t *__restrict__ w,
                                                  const float *__restrict__ bias, uint16_t *__restrict__ y,
                                                  int64_t n_pos)
{
    constexpr int K = 27 * CIN;
    constexpr int KC = (K + 15) / 16;     // K chunks
    constexpr int NCT = CT;               // output-channel tiles of this wave
    constexpr int NG = COUT / (16 * CT);  // waves per position tile
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int kq = 4 * (lane >> 4);  // first of this lane's 4 k in a chunk
    const int64_t n_items = (n_pos + 15) / 16 * NG;
    for (int64_t item = (int64_t)blockIdx.x * 4 + wid; item < n_items; item += (int64_t)gridDim.x * 4) {
        const int64_t tile = item / NG;
        const int cg = (int)(item % NG);  // output channels cg 16 CT .. (cg + 1) 16 CT - 1
        // A row of this lane: output position tile * 16 + lane % 16
        const int64_t p = tile * 16 + (lane & 15);
        const bool pin = p < n_pos;
        const int64_t pp = pin ? p : 0;
        const int ox = (int)(pp % DOUT), oy = (int)((pp / DOUT) % DOUT), oz = (int)((pp / (DOUT * DOUT)) % DOUT);
        const int64_t nb = pp / ((int64_t)DOUT * DOUT * DOUT);
        v4f32 acc[NCT];
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[t] = (v4f32){0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < KC; ++c) {
            const int k0 = 16 * c + kq;  // 4 consecutive k: same kernel offset, channels ci..ci+3
            v4i16 a = {0, 0, 0, 0};
            v4i16 b[NCT];
#pragma unroll
            for (int t = 0; t < NCT; ++t) b[t] = (v4i16){0, 0, 0, 0};
            if (k0 < K) {
                const int off = k0 / CIN, ci = k0 % CIN;
                const int kd = off / 9, kh = (off / 3) % 3, kw = off % 3;
                const int iz = oz * STRIDE + kd - 1, iy = oy * STRIDE + kh - 1, ix = ox * STRIDE + kw - 1;
                if (pin && iz >= 0 && iy >= 0 && ix >= 0 && iz < DIN && iy < DIN && ix < DIN) {
                    const int64_t src = (((nb * DIN + iz) * DIN + iy) * DIN + ix) * CIN + ci;
                    a = *(const v4i16 *)(x + src);
                }
#pragma unroll
                for (int t = 0; t < NCT; ++t)
                    b[t] = *(const v4i16 *)(w + (int64_t)((cg * NCT + t) * 16 + (lane & 15)) * K + k0);
            }
#pragma unroll
            for (int t = 0; t < NCT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[t], 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int co = (cg * NCT + t) * 16 + (lane & 15);
            const float bv = bias[co];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t q = tile * 16 + 4 * (lane >> 4) + i;
                if (q < n_pos) {
                    const float v = fmaxf(acc[t][i] + bv, 0.0f);
                    y[q * COUT + co] = f2bf(v);
                }
            }
        }
    }
}

// Global mean over the 4^3 positions and the fully connected head.
__global__ void k_pool_fc(const uint16_t *__restrict__ a4, const float *__restrict__ wfc,
                          const float *__restrict__ bfc, float *__restrict__ pooled, float *__restrict__ out, int n)
{
    const int b = blockIdx.x, c = threadIdx.x;  // 64 threads
    if (b >= n) return;
    __shared__ float f[kFeat];
    float s = 0.f;
    for (int p = 0; p < 64; ++p) s += bf2f(a4[((int64_t)b * 64 + p) * kFeat + c]);
    s *= (1.0f / 64.0f);
    f[c] = s;
    pooled[b * kFeat + c] = s;
    __syncthreads();
    if (c < kOut) {
        float o = bfc[c];
        for (int k = 0; k < kFeat; ++k) o += wfc[c * kFeat + k] * f[k];
        out[b * kOut + c] = o;
    }
}

// ------------------------------------------------------------ backward (FP32)

// Loss: sum over the batch of (|t - t*|^2 / s_t^2 + |(c, s) - (c*, s*)|^2),
// divided by n.  d_out = its gradient.
__global__ void k_loss(const float *__restrict__ out, const float *__restrict__ y, float *__restrict__ dout,
                       float *__restrict__ loss, int n, float inv_st2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kOut) return;
    const int k = i % kOut;
    const float wgt = k < 3 ? inv_st2 : 1.0f;
    const float d = out[i] - y[i];
    dout[i] = 2.0f * wgt * d / (float)n;
    atomicAdd(loss, wgt * d * d / (float)n);
}

// FC backward: gradients of the head, then d a4 = (d pooled / 64) masked by
// ReLU (a4 > 0).  Workgroup n (64 threads) sums the head's gradients over the
// batch; workgroup b < n writes d a4 of item b.
__global__ void k_fc_bwd(const float *__restrict__ dout, const float *__restrict__ pooled,
                         const float *__restrict__ wfc, const uint16_t *__restrict__ a4, float *__restrict__ gwfc,
                         float *__restrict__ gbfc, float *__restrict__ da4, int n)
{
    const int t = threadIdx.x, b = blockIdx.x;
    if (b == n) {
        // weight and bias gradients (each thread one feature column)
        for (int o = 0; o < kOut; ++o) {
            float g = 0.f, gb = 0.f;
            for (int bb = 0; bb < n; ++bb) {
                g += dout[bb * kOut + o] * pooled[bb * kFeat + t];
                gb += dout[bb * kOut + o];
            }
            gwfc[o * kFeat + t] += g;
            if (t == 0) gbfc[o] += gb;
        }
        return;
    }
    float dp = 0.f;
    for (int o = 0; o < kOut; ++o) dp += dout[b * kOut + o] * wfc[o * kFeat + t];
    dp *= (1.0f / 64.0f);
    for (int p = 0; p < 64; ++p) {
        const int64_t q = ((int64_t)b * 64 + p) * kFeat + t;
        da4[q] = bf2f(a4[q]) > 0.f ? dp : 0.f;
    }
}

// Weight and bias gradients on the matrix cores (MFMA 16x16x16 bf16, FP32
// accumulation): gw[co][kk] = sum_p dy[p][co] xcol[p][kk], kk = tap CIN +
// ci, xcol the input activation under tap kk of output position p (zero
// outside the grid); column kk = K of xcol is 1, which gives the bias
// gradient sum_p dy[p][co].  One wave per 16 output channels, G tiles of 16
// columns and chunk of positions (16 per MFMA, the reduction dimension):
// dy is read and rounded to bf16 once per step for the G tiles (the
// activations are bf16 already), and each position's coordinates are
// computed once for them; one atomic add per output and chunk.
template <int CIN, int COUT, int DIN, int DOUT, int STRIDE, int G>
__global__ __launch_bounds__(256) void k_conv_wgrad(const uint16_t *__restrict__ x, const float *__restrict__ dy,
                                                    float *__restrict__ gw, float *__restrict__ gb, int64_t n_pos,
                                                    int64_t chunk)
{
    constexpr int K = 27 * CIN;
    constexpr int NCT = COUT / 16;
    constexpr int NKT = (K + 1 + 15) / 16;  // column tiles, the bias column included
    constexpr int NKG = (NKT + G - 1) / G;  // groups of G tiles
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t tile = wave % (NCT * NKG), part = wave / (NCT * NKG);
    const int64_t p0 = part * chunk;
    if (p0 >= n_pos) return;  // uniform across the wave
    const int64_t p1 = min(n_pos, p0 + chunk);
    const int ct = (int)(tile % NCT), kg = (int)(tile / NCT);
    const int co = ct * 16 + (lane & 15);  // this lane's A row
    const int q4 = 4 * (lane >> 4);         // its 4 positions of a step
    int tap[G], ci[G];                      // this lane's B column of each tile: tap and channel
    bool is_w[G], is_b[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int kk = (kg * G + g) * 16 + (lane & 15);
        is_w[g] = kk < K;
        is_b[g] = kk == K;
        tap[g] = is_w[g] ? kk / CIN : 0;
        ci[g] = is_w[g] ? kk % CIN : 0;
    }
    v4f32 acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = (v4f32){0.f, 0.f, 0.f, 0.f};
    for (int64_t pb = p0; pb < p1; pb += 16) {
        v4i16 av = {0, 0, 0, 0};
        int oxs[4], oys[4], ozs[4];
        int64_t nbs[4];
        bool pin[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t p = pb + q4 + i;
            pin[i] = p < p1;
            const int64_t pp = pin[i] ? p : p0;
            av[i] = pin[i] ? (short)f2bf(dy[pp * COUT + co]) : (short)0;
            oxs[i] = (int)(pp % DOUT);
            oys[i] = (int)((pp / DOUT) % DOUT);
            ozs[i] = (int)((pp / (DOUT * DOUT)) % DOUT);
            nbs[i] = pp / ((int64_t)DOUT * DOUT * DOUT);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (kg * G + g >= NKT) break;  // uniform
            const int kd = tap[g] / 9, kh = (tap[g] / 3) % 3, kw = tap[g] % 3;
            v4i16 bv = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (!pin[i]) continue;
                if (is_b[g]) {
                    bv[i] = (short)0x3F80;  // bf16 1.0
                } else if (is_w[g]) {
                    const int iz = ozs[i] * STRIDE + kd - 1, iy = oys[i] * STRIDE + kh - 1, ix = oxs[i] * STRIDE + kw - 1;
                    if (iz >= 0 && iy >= 0 && ix >= 0 && iz < DIN && iy < DIN && ix < DIN)
                        bv[i] = (short)x[(((nbs[i] * DIN + iz) * DIN + iy) * DIN + ix) * CIN + ci[g]];
                }
            }
            acc[g] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[g], 0, 0, 0);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (kg * G + g >= NKT) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int co_o = ct * 16 + q4 + i, kk_o = (kg * G + g) * 16 + (lane & 15);
            if (kk_o < K) atomicAdd(&gw[(int64_t)co_o * K + kk_o], acc[g][i]);
            else if (kk_o == K) atomicAdd(&gb[co_o], acc[g][i]);
        }
    }
}

// Input gradient through the convolution on the matrix cores, masked by the
// ReLU of the layer that produced x (x > 0): dx[p][ci] = sum over (tap, co)
// dy[o][co] w[co][tap CIN + ci], o the output position that tap maps onto
// input position p (none where the stride skips it).  One wave per tile of
// 16 input positions x 16 input channels; the reduction runs over the taps
// that map some position of the tile onto an output and, per tap, over the
// output channels 16 at a time; dy is rounded to bf16 and the bf16 copy of
// the weights is used.
template <int CIN, int COUT, int DIN, int DOUT, int STRIDE>
__global__ __launch_bounds__(256) void k_conv_dgrad(const uint16_t *__restrict__ x, const float *__restrict__ dy,
                                                    const uint16_t *__restrict__ wb, float *__restrict__ dx,
                                                    int64_t n_in)
{
    constexpr int K = 27 * CIN;
    constexpr int NCI = CIN / 16;
    static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel counts in multiples of 16");
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= ((n_in + 15) / 16) * NCI) return;  // uniform across the wave
    const int cit = (int)(wave % NCI);
    const int64_t pt = wave / NCI;
    const int64_t pm = pt * 16 + (lane & 15);  // this lane's A row: an input position
    const bool pin = pm < n_in;
    const int64_t pp = pin ? pm : 0;
    const int ix = (int)(pp % DIN), iy = (int)((pp / DIN) % DIN), iz = (int)((pp / (DIN * DIN)) % DIN);
    const int64_t nb = pp / ((int64_t)DIN * DIN * DIN);
    const int cib = cit * 16 + (lane & 15);  // this lane's B column: an input channel
    const int q4 = 4 * (lane >> 4);
    v4f32 acc = {0.f, 0.f, 0.f, 0.f};
    for (int tap = 0; tap < 27; ++tap) {
        const int kd = tap / 9, kh = (tap / 3) % 3, kw = tap % 3;
        const int tz = iz + 1 - kd, ty = iy + 1 - kh, tx = ix + 1 - kw;
        const bool ok = pin && tz >= 0 && ty >= 0 && tx >= 0 && tz % STRIDE == 0 && ty % STRIDE == 0 &&
                        tx % STRIDE == 0 && tz / STRIDE < DOUT && ty / STRIDE < DOUT && tx / STRIDE < DOUT;
        // a tap that maps no position of the tile onto an output adds only
        // zeros (with stride 2, most taps for a row of input positions)
        if (__ballot(ok) == 0) continue;  // uniform
        const int64_t o = ok ? ((nb * DOUT + tz / STRIDE) * DOUT + ty / STRIDE) * DOUT + tx / STRIDE : 0;
#pragma unroll
        for (int c0 = 0; c0 < COUT; c0 += 16) {
            v4i16 av = {0, 0, 0, 0}, bv;
            if (ok) {
                const float4 g = *(const float4 *)(dy + o * COUT + c0 + q4);
                av[0] = (short)f2bf(g.x);
                av[1] = (short)f2bf(g.y);
                av[2] = (short)f2bf(g.z);
                av[3] = (short)f2bf(g.w);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[i] = (short)wb[(int64_t)(c0 + q4 + i) * K + tap * CIN + cib];
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t p = pt * 16 + q4 + i;
        if (p < n_in) {
            const int64_t id = p * CIN + cit * 16 + (lane & 15);
            dx[id] = bf2f(x[id]) > 0.f ? acc[i] : 0.f;
        }
    }
}

// Adam (Kingma and Ba, 2015) on the FP32 master weights; refreshes the bf16
// copies of the convolution weights.
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_refresh_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

__global__ void k_zero(float *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + t - 1) / t, 1 << 20)); }

}  // namespace

// Parameter layout (FP32 master, in order): for each convolution w[cout][27
// cin], b[cout]; then fc w[5][64], b[5].
struct NetParams {
    int64_t off_w[kLayers], off_b[kLayers], off_fcw, off_fcb, total;
    NetParams()
    {
        int64_t o = 0;
        for (int l = 0; l < kLayers; ++l) {
            off_w[l] = o;
            o += (int64_t)kShapes[l].cout * kShapes[l].K();
            off_b[l] = o;
            o += kShapes[l].cout;
        }
        off_fcw = o;
        o += kOut * kFeat;
        off_fcb = o;
        o += kOut;
        total = o;
    }
};

}  // namespace covox

struct covox_net {
    covox_ctx *ctx = nullptr;
    covox::NetParams P;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // FP32 master, grad, Adam moments
    uint16_t *wb[covox::kLayers] = {nullptr, nullptr, nullptr, nullptr};
    int64_t step = 0;
    // activations for the current batch capacity
    int batch_cap = 0;
    uint16_t *x0 = nullptr, *a[covox::kLayers] = {nullptr, nullptr, nullptr, nullptr};
    float *pooled = nullptr, *out = nullptr, *dout = nullptr, *loss = nullptr;
    float *d[covox::kLayers] = {nullptr, nullptr, nullptr, nullptr};  // gradients of the layer outputs
};

namespace covox {

static int64_t act_elems(int l, int n)
{
    const ConvShape &s = kShapes[l];
    return (int64_t)n * s.dout * s.dout * s.dout * s.cout;
}

static int net_reserve(covox_net *net, int n)
{
    if (n <= net->batch_cap) return COVOX_OK;
    covox_ctx *ctx = net->ctx;
    int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "net reserve sync");  // readers of the old buffers
    if (rc) return rc;
    auto fr = [](void *p) { if (p) (void)hipFree(p); };
    fr(net->x0); fr(net->pooled); fr(net->out); fr(net->dout); fr(net->loss);
    for (int l = 0; l < kLayers; ++l) { fr(net->a[l]); fr(net->d[l]); net->a[l] = nullptr; net->d[l] = nullptr; }
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void **)&net->x0, sizeof(uint16_t) * (int64_t)n * 32768 * 4);
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
        e = hipMalloc((void **)&net->a[l], sizeof(uint16_t) * act_elems(l, n));
        if (e == hipSuccess) e = hipMalloc((void **)&net->d[l], sizeof(float) * act_elems(l, n));
    }
    if (e == hipSuccess) e = hipMalloc((void **)&net->pooled, sizeof(float) * n * kFeat);
    if (e == hipSuccess) e = hipMalloc((void **)&net->out, sizeof(float) * n * kOut);
    if (e == hipSuccess) e = hipMalloc((void **)&net->dout, sizeof(float) * n * kOut);
    if (e == hipSuccess) e = hipMalloc((void **)&net->loss, sizeof(float));
    if (e != hipSuccess) {
        net->batch_cap = 0;
        return fail(ctx, COVOX_EHIP, std::string("net buffers: ") + hipGetErrorString(e));
    }
    net->batch_cap = n;
    return COVOX_OK;
}

template <int L>
static void launch_conv_fwd(covox_net *net, const uint16_t *x, uint16_t *y, int n)
{
    constexpr ConvShape s = kShapes[L];
    // the last layer (4^3 positions per item) splits its output channels over waves
    constexpr int CT = s.dout >= 8 ? s.cout / 16 : 1;
    const int64_t npos = (int64_t)n * s.dout * s.dout * s.dout;
    const int64_t items = (npos + 15) / 16 * (s.cout / (16 * CT));
    const unsigned grid = (unsigned)std::min<int64_t>((items + 3) / 4, 1 << 20);  // 4 waves per workgroup
    hipLaunchKernelGGL((k_conv_fwd<s.cin, s.cout, s.din, s.dout, s.stride, CT>), dim3(grid), dim3(256), 0,
                       net->ctx->stream, x, net->wb[L], net->w + net->P.off_b[L], y, npos);
}

// Buffers of one forward pass: the bf16 input, the four bf16 layer outputs,
// the pooled features and the network outputs.
struct FwdBuffers {
    uint16_t *x0;
    uint16_t *a[kLayers];
    float *pooled, *out;
};

// The forward pass's launches on the context stream, into the given buffers
// (every element of each buffer is written before it is read).
static void forward_launches(covox_net *net, const float *x_dev, int n, const FwdBuffers &b)
{
    covox_ctx *ctx = net->ctx;
    const int64_t nx = (int64_t)n * 32768 * 4;
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(nx, 256)), dim3(256), 0, ctx->stream, x_dev, b.x0, nx);
    launch_conv_fwd<0>(net, b.x0, b.a[0], n);
    launch_conv_fwd<1>(net, b.a[0], b.a[1], n);
    launch_conv_fwd<2>(net, b.a[1], b.a[2], n);
    launch_conv_fwd<3>(net, b.a[2], b.a[3], n);
    hipLaunchKernelGGL(k_pool_fc, dim3(n), dim3(64), 0, ctx->stream, b.a[3], net->w + net->P.off_fcw,
                       net->w + net->P.off_fcb, b.pooled, b.out, n);
}

static int net_forward(covox_net *net, const float *x_dev, int n)
{
    covox_ctx *ctx = net->ctx;
    int rc = net_reserve(net, n);
    if (rc) return rc;
    {
        TimedLaunch tl(ctx, COVOX_K_NET);
        forward_launches(net, x_dev, n, FwdBuffers{net->x0, {net->a[0], net->a[1], net->a[2], net->a[3]},
                                                   net->pooled, net->out});
    }
    return hip_check(ctx, hipGetLastError(), "net forward");
}

template <int L>
static void launch_wgrad(covox_net *net, const uint16_t *x, int n)
{
    constexpr ConvShape s = kShapes[L];
    // One column tile per wave: sharing dy over 4 tiles (fewer, longer waves)
    // measured slower on every layer.
    constexpr int G = 1;
    constexpr int64_t tiles = (int64_t)(s.cout / 16) * (((s.K() + 1 + 15) / 16 + G - 1) / G);
    const int64_t npos = (int64_t)n * s.dout * s.dout * s.dout;
    // positions per wave (a multiple of 16): at most 1024, fewer where the
    // layer has few positions, so that a launch has about 12 k waves
    const int64_t chunk = std::max<int64_t>(64, std::min<int64_t>(1024, npos * tiles / 12288 / 16 * 16));
    const int64_t waves = tiles * ((npos + chunk - 1) / chunk);
    hipLaunchKernelGGL((k_conv_wgrad<s.cin, s.cout, s.din, s.dout, s.stride, G>), dim3(blocks_for(waves * 64, 256)),
                       dim3(256), 0, net->ctx->stream, x, net->d[L], net->g + net->P.off_w[L],
                       net->g + net->P.off_b[L], npos, chunk);
}

template <int L>
static void launch_dgrad(covox_net *net, const uint16_t *x, float *dx, int n)
{
    constexpr ConvShape s = kShapes[L];
    const int64_t nin = (int64_t)n * s.din * s.din * s.din;
    const int64_t waves = ((nin + 15) / 16) * (s.cin / 16);
    hipLaunchKernelGGL((k_conv_dgrad<s.cin, s.cout, s.din, s.dout, s.stride>), dim3(blocks_for(waves * 64, 256)),
                       dim3(256), 0, net->ctx->stream, x, net->d[L], net->wb[L], dx, nin);
}

static int net_backward(covox_net *net, int n)
{
    covox_ctx *ctx = net->ctx;
    const int64_t np = net->P.total;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(np, 256)), dim3(256), 0, ctx->stream, net->g, np);
    hipLaunchKernelGGL(k_fc_bwd, dim3(n + 1), dim3(64), 0, ctx->stream, net->dout, net->pooled, net->w + net->P.off_fcw,
                       net->a[3], net->g + net->P.off_fcw, net->g + net->P.off_fcb, net->d[3], n);
    launch_wgrad<3>(net, net->a[2], n);
    launch_dgrad<3>(net, net->a[2], net->d[2], n);
    launch_wgrad<2>(net, net->a[1], n);
    launch_dgrad<2>(net, net->a[1], net->d[1], n);
    launch_wgrad<1>(net, net->a[0], n);
    launch_dgrad<1>(net, net->a[0], net->d[0], n);
    launch_wgrad<0>(net, net->x0, n);
    return hip_check(ctx, hipGetLastError(), "net backward");
}

static void refresh_bf16(covox_net *net)
{
    for (int l = 0; l < kLayers; ++l) {
        const int64_t nw = (int64_t)kShapes[l].cout * kShapes[l].K();
        hipLaunchKernelGGL(k_refresh_bf16, dim3(blocks_for(nw, 256)), dim3(256), 0, net->ctx->stream,
                           net->w + net->P.off_w[l], net->wb[l], nw);
    }
}

int net_forward_api(covox_net *net, const float *x_dev, int n, float *out_dev)
{
    int rc = net_forward(net, x_dev, n);
    if (rc) return rc;
    return hip_check(net->ctx, hipMemcpyAsync(out_dev, net->out, sizeof(float) * n * kOut, hipMemcpyDeviceToDevice,
                                              net->ctx->stream), "net output copy");
}

const float *net_loss_dev(const covox_net *net) { return net->loss; }

// ------------------------------------------------- forward without allocation
//
// Activations of at most COVOX_NET_NOALLOC_MAX_PAIRS pairs in a file-scope
// device array.  Its address on each device comes from hipGetSymbolAddress,
// taken once per device when a context is created there; host code never
// uses the array's name as a device address.

constexpr int64_t kNoAllocX0 = (int64_t)COVOX_NET_NOALLOC_MAX_PAIRS * 32768 * 4;  // bf16 elements
constexpr int64_t noalloc_act(int l)
{
    return (int64_t)COVOX_NET_NOALLOC_MAX_PAIRS * kShapes[l].dout * kShapes[l].dout * kShapes[l].dout *
           kShapes[l].cout;
}
constexpr int64_t kNoAllocBytes =
    2 * (kNoAllocX0 + noalloc_act(0) + noalloc_act(1) + noalloc_act(2) + noalloc_act(3)) +
    4 * (int64_t)COVOX_NET_NOALLOC_MAX_PAIRS * kFeat;
static_assert(kNoAllocBytes % 256 == 0, "scratch regions stay 256-byte aligned");

}  // namespace covox

static __device__ __align__(256) unsigned char scratch[covox::kNoAllocBytes];

namespace covox {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch_init(covox_ctx *ctx)
{
    const int dev = ctx->device;
    if (dev < 0 || dev >= kMaxDevices) return fail(ctx, COVOX_EHIP, "no-alloc scratch: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return COVOX_OK;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
        return fail(ctx, COVOX_EHIP, std::string("no-alloc scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    return COVOX_OK;
}

int net_forward_noalloc(covox_net *net, const float *x_dev, int n, float *out_dev)
{
    covox_ctx *ctx = net->ctx;
    if (n > COVOX_NET_NOALLOC_MAX_PAIRS)
        return fail(ctx, COVOX_EINVAL, "net_forward_noalloc: more than COVOX_NET_NOALLOC_MAX_PAIRS pairs");
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) base = (unsigned char *)g_scratch_ptr[ctx->device];
    }
    if (!base) return fail(ctx, COVOX_EHIP, "net_forward_noalloc: scratch address not set up on this device");
    // Regions sized for the maximum batch; n pairs use the front of each.
    FwdBuffers b;
    b.x0 = (uint16_t *)base;
    base += 2 * kNoAllocX0;
    for (int l = 0; l < kLayers; ++l) {
        b.a[l] = (uint16_t *)base;
        base += 2 * noalloc_act(l);
    }
    b.pooled = (float *)base;
    b.out = out_dev;
    forward_launches(net, x_dev, n, b);
    return hip_check(ctx, hipGetLastError(), "net forward (no allocation)");
}

int net_train_step(covox_net *net, const float *x_dev, const float *y_dev, int n, float lr, float trans_scale,
                   float *loss_host)
{
    int rc = net_train_async(net, x_dev, y_dev, n, lr, trans_scale);
    if (rc) return rc;
    if (loss_host) {
        covox_ctx *ctx = net->ctx;
        if ((rc = hip_check(ctx, hipMemcpyAsync(loss_host, net->loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
                            "loss copy")))
            return rc;
        return hip_check(ctx, hipStreamSynchronize(ctx->stream), "train sync");
    }
    return COVOX_OK;
}

int net_train_async(covox_net *net, const float *x_dev, const float *y_dev, int n, float lr, float trans_scale)
{
    covox_ctx *ctx = net->ctx;
    int rc = net_forward(net, x_dev, n);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, ctx->stream, net->loss, (int64_t)1);
    hipLaunchKernelGGL(k_loss, dim3(blocks_for((int64_t)n * kOut, 64)), dim3(64), 0, ctx->stream, net->out, y_dev,
                       net->dout, net->loss, n, 1.0f / (trans_scale * trans_scale));
    {
        TimedLaunch tl(ctx, COVOX_K_NET);
        if ((rc = net_backward(net, n))) return rc;
    }
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)net->step), c2 = 1.f - powf(b2, (float)net->step);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(net->P.total, 256)), dim3(256), 0, ctx->stream, net->w, net->g, net->m,
                       net->v, net->P.total, lr, b1, b2, 1e-8f, c1, c2);
    refresh_bf16(net);
    return hip_check(ctx, hipGetLastError(), "net train step");
}

int net_grads(covox_net *net, const float *x_dev, const float *y_dev, int n, float trans_scale, float *grad_host,
              float *loss_host)
{
    covox_ctx *ctx = net->ctx;
    int rc = net_forward(net, x_dev, n);
    if (rc) return rc;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, ctx->stream, net->loss, (int64_t)1);
    hipLaunchKernelGGL(k_loss, dim3(blocks_for((int64_t)n * kOut, 64)), dim3(64), 0, ctx->stream, net->out, y_dev,
                       net->dout, net->loss, n, 1.0f / (trans_scale * trans_scale));
    if ((rc = net_backward(net, n))) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(grad_host, net->g, sizeof(float) * net->P.total, hipMemcpyDeviceToHost,
                                            ctx->stream), "grad copy")))
        return rc;
    if (loss_host &&
        (rc = hip_check(ctx, hipMemcpyAsync(loss_host, net->loss, sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
                        "loss copy")))
        return rc;
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "grad sync");
}

int net_create(covox_ctx *ctx, uint64_t seed, covox_net **out)
{
    covox_net *net = new covox_net();
    net->ctx = ctx;
    const int64_t np = net->P.total;
    hipError_t e = hipSuccess;
    for (float **p : {&net->w, &net->g, &net->m, &net->v})
        if (e == hipSuccess) e = hipMalloc((void **)p, sizeof(float) * np);
    for (int l = 0; l < kLayers && e == hipSuccess; ++l)
        e = hipMalloc((void **)&net->wb[l], sizeof(uint16_t) * (int64_t)kShapes[l].cout * kShapes[l].K());
    if (e != hipSuccess) {
        net_destroy(net);
        return fail(ctx, COVOX_EHIP, std::string("net_create: ") + hipGetErrorString(e));
    }
    // He-uniform initialisation from SplitMix64 (zero biases)
    std::vector<float> h(np, 0.f);
    uint64_t state = seed;
    auto uni = [&]() {
        state += 0x9e3779b97f4a7c15ull;
        return (double)(mix64(state) >> 11) * (1.0 / 9007199254740992.0);
    };
    for (int l = 0; l < kLayers; ++l) {
        const double lim = sqrt(6.0 / (double)kShapes[l].K());
        for (int64_t i = 0; i < (int64_t)kShapes[l].cout * kShapes[l].K(); ++i)
            h[net->P.off_w[l] + i] = (float)((2.0 * uni() - 1.0) * lim);
    }
    const double lim = sqrt(6.0 / (double)kFeat);
    for (int i = 0; i < kOut * kFeat; ++i) h[net->P.off_fcw + i] = (float)((2.0 * uni() - 1.0) * lim) * 0.1f;
    std::vector<float> zeros(np, 0.f);
    e = hipMemcpy(net->w, h.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net->m, zeros.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(net->v, zeros.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        net_destroy(net);
        return fail(ctx, COVOX_EHIP, std::string("net_create upload: ") + hipGetErrorString(e));
    }
    refresh_bf16(net);
    int rc = hip_check(ctx, hipGetLastError(), "net init");
    if (rc) {
        net_destroy(net);
        return rc;
    }
    ctx->nets.push_back(net);
    *out = net;
    return COVOX_OK;
}

static void net_free_device(covox_net *net)
{
    for (float **p : {&net->w, &net->g, &net->m, &net->v, &net->pooled, &net->out, &net->dout, &net->loss}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    if (net->x0) (void)hipFree(net->x0);
    net->x0 = nullptr;
    for (int l = 0; l < kLayers; ++l) {
        for (void **p : {(void **)&net->wb[l], (void **)&net->a[l], (void **)&net->d[l]}) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
    }
    net->batch_cap = 0;
}

void net_detach(covox_net *net)
{
    if (!net) return;
    net_free_device(net);
    net->ctx = nullptr;
}

void net_destroy(covox_net *net)
{
    if (!net) return;
    if (covox_ctx *ctx = net->ctx) {
        (void)hipStreamSynchronize(ctx->stream);
        ctx->nets.erase(std::remove(ctx->nets.begin(), ctx->nets.end(), net), ctx->nets.end());
    }
    net_free_device(net);
    delete net;
}

int64_t net_num_params(const covox_net *net) { return net->P.total; }

covox_ctx *net_ctx(const covox_net *net) { return net->ctx; }

int net_get_params(covox_net *net, float *host, int64_t n)
{
    if (n != net->P.total) return fail(net->ctx, COVOX_EINVAL, "net params: wrong count");
    int rc = hip_check(net->ctx, hipStreamSynchronize(net->ctx->stream), "params sync");  // pending training steps
    if (rc) return rc;
    return hip_check(net->ctx, hipMemcpy(host, net->w, sizeof(float) * n, hipMemcpyDeviceToHost), "params copy");
}

int net_set_params(covox_net *net, const float *host, int64_t n)
{
    if (n != net->P.total) return fail(net->ctx, COVOX_EINVAL, "net params: wrong count");
    int rc = hip_check(net->ctx, hipStreamSynchronize(net->ctx->stream), "params sync");  // readers in flight
    if (rc) return rc;
    rc = hip_check(net->ctx, hipMemcpy(net->w, host, sizeof(float) * n, hipMemcpyHostToDevice), "params upload");
    if (rc) return rc;
    refresh_bf16(net);
    return hip_check(net->ctx, hipStreamSynchronize(net->ctx->stream), "params sync");
}

}  // namespace covox
