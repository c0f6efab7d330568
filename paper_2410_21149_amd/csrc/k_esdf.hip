// Exact truncated ESDF from the TSDF (paper Sec. I: distance to the nearest
// obstacle built from the TSDF, reusing the in-band distances; Sec. III-E:
// an exact Euclidean distance transform in the PBA lineage, organised per
// block).
//
// The squared distance k(i) = min over sites s of |i - s|^2 is separable:
//   g1(x,y,z) = min_x' (x - x')^2 over sites on the x line    (k_edt_x)
//   g2(x,y,z) = min_y' g1(x,y',z) + (y - y')^2                 (k_edt_y)
//   k(x,y,z)  = min_z' g2(x,y,z') + (z - z')^2                 (k_edt_z)
// Only k <= R^2 (R = round(d_max / vs)) matters, so every pass looks at most
// R voxels (HB = ceil(R / 8) blocks) to each side and stores larger values as
// "infinite"; in each pass the search from the centre stops once d^2 reaches
// the best value, which makes the min exact.  The passes run over the dense
// block box of the allocated blocks: intermediate values are needed in
// unallocated blocks between allocated ones.
//
// Layout: every dense block keeps its 512 voxels contiguous (l = x + 8y +
// 64z), like the TSDF pool, so one wave64 owns one block with lane = (x, y)
// and z in registers; neighbours along an axis are whole blocks, staged in
// LDS per wave.  Site masks are 8 64-bit words per block (word z, bit x+8y).
#include "covox_impl.h"
#include "edt_envelope.h"

#include <algorithm>

namespace covox {

namespace {

constexpr int kBig = 1 << 24;

template <typename S> __device__ __forceinline__ float ldv(const S *p);
template <> __device__ __forceinline__ float ldv<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldv<__half>(const __half *p) { return __half2float(*p); }

struct Dom {
    int32_t lo[3], dim[3];
    int64_t n;
};

__device__ __forceinline__ Dom read_dom(const SubmapMeta *m)
{
    Dom d;
    if (m->n_blocks <= 0) {
        d.n = 0;
        for (int a = 0; a < 3; ++a) { d.lo[a] = 0; d.dim[a] = 0; }
        return d;
    }
    d.n = 1;
    for (int a = 0; a < 3; ++a) {
        d.lo[a] = m->bmin[a];
        d.dim[a] = m->bmax[a] - m->bmin[a] + 1;
        d.n *= d.dim[a];
    }
    return d;
}

__device__ __forceinline__ void dom_coords(const Dom &d, int64_t db, int &x, int &y, int &z)
{
    x = (int)(db % d.dim[0]);
    y = (int)((db / d.dim[0]) % d.dim[1]);
    z = (int)(db / ((int64_t)d.dim[0] * d.dim[1]));
}

__device__ __forceinline__ int64_t dom_index(const Dom &d, int x, int y, int z)
{
    return ((int64_t)z * d.dim[1] + y) * d.dim[0] + x;
}

// Page (dense block -> buffer index, -1 if unallocated) and site masks.
template <typename S>
__global__ __launch_bounds__(256) void k_page_sites(SubmapMeta *meta, const uint64_t *__restrict__ tkeys,
                                                    const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                    const S *__restrict__ D, const S *__restrict__ W,
                                                    float vs, int32_t *__restrict__ page,
                                                    uint64_t *__restrict__ sites)
{
    const Dom d = read_dom(meta);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    if (wave == 0 && lane == 0) {
        for (int a = 0; a < 3; ++a) { meta->dom_min[a] = d.lo[a]; meta->dom_dim[a] = d.dim[a]; }
        meta->dom_valid = 1;
    }
    for (int64_t db = wave; db < d.n; db += nwaves) {
        int x, y, z;
        dom_coords(d, db, x, y, z);
        int64_t idx = -1;
        if (lane == 0) idx = hash_find(tkeys, tvals, tmask, pack_key(d.lo[0] + x, d.lo[1] + y, d.lo[2] + z));
        idx = __shfl(idx, 0, 64);
        if (lane == 0) page[db] = (int32_t)idx;
        uint64_t w = 0;
        if (idx >= 0) {
            const S *Db = D + idx * 512 + lane;
            const S *Wb = W + idx * 512 + lane;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float Dv = ldv(Db + 64 * k), Wv = ldv(Wb + 64 * k);
                const uint64_t m = __ballot(Wv > 0.0f && fabsf(Dv) <= vs);
                if (lane == k) w = m;
            }
        }
        if (lane < 8) sites[db * 8 + lane] = w;
    }
}

// Distance to the nearest set bit of the 128-bit mask (lo, hi) from bit p.
__device__ __forceinline__ int nearest_bit(uint64_t lo, uint64_t hi, int p)
{
    uint64_t rlo, rhi;
    if (p == 0) { rlo = lo; rhi = hi; }
    else if (p < 64) { rlo = (lo >> p) | (hi << (64 - p)); rhi = hi >> p; }
    else { rlo = hi >> (p - 64); rhi = 0; }
    const int dr = rlo ? __ffsll((long long)rlo) - 1 : (rhi ? 63 + __ffsll((long long)rhi) : 1000);
    const int s = 127 - p;
    uint64_t llo, lhi;
    if (s == 0) { llo = lo; lhi = hi; }
    else if (s < 64) { lhi = (hi << s) | (lo >> (64 - s)); llo = lo << s; }
    else { lhi = lo << (s - 64); llo = 0; }
    const int dl = lhi ? __clzll((long long)lhi) : (llo ? 64 + __clzll((long long)llo) : 1000);
    return min(dl, dr);
}

// ------------------------------------------------------------------------
// y and z passes: lower envelope of parabolas per line (Felzenszwalb and
// Huttenlocher).  One wave per block column; lane = one line.  A line longer
// than kWin voxels is cut into output segments that each carry C = 8 HB >= R
// voxels of context on both sides, which is exact because only k <= R^2 is
// kept.  Breakpoints s(p, q) = ((f_q - f_p) + (q - p)(q + p)) / (2 (q - p))
// are compared by integer cross-multiplication (|N| < 2^18, D <= 2 kWin), so
// the envelope is exact.

constexpr int kWin = 256;  // window positions (u8 stack entries)

__device__ __forceinline__ void segment(int L, int C, int seg, int S, int &y0, int &y1, int &w0, int &w1)
{
    y0 = seg * S;
    y1 = min(y0 + S, L);
    w0 = max(0, y0 - C);
    w1 = min(L, y1 + C);
}

// g2(x, y, z) = min_y' g1(x, y', z)^2 + (y - y')^2, kept when <= R^2.
// Lane = x + 8 z within the block column (bx, *, bz).
__global__ __launch_bounds__(64) void k_edt_y_env(const SubmapMeta *meta, const uint8_t *__restrict__ g1,
                                              uint16_t *__restrict__ g2, int R, int HB)
{
    __shared__ __align__(16) uint8_t col[kWin * 64];   // [position][lane]
    __shared__ __align__(16) uint8_t stk[kWin * 64];   // [entry][lane]
    __shared__ __align__(16) uint16_t ost[8 * 64];     // one block of outputs [y][lane]
    const Dom d = read_dom(meta);
    const int lane = threadIdx.x;
    const int C = 8 * HB;
    const int S = kWin - 2 * C;
    const int L = 8 * d.dim[1];
    const int nseg = L > 0 ? (L + S - 1) / S : 0;
    const int64_t ncol = (int64_t)d.dim[0] * d.dim[2] * nseg;
    const int R2 = R * R;
    auto getf = [&](int q) {
        const int a = col[q * 64 + lane];
        return a * a;
    };
    for (int64_t c = blockIdx.x; c < ncol; c += gridDim.x) {
        const int seg = (int)(c % nseg);
        const int64_t cc = c / nseg;
        const int bx = (int)(cc % d.dim[0]), bz = (int)(cc / d.dim[0]);
        int y0, y1, w0, w1;
        segment(L, C, seg, S, y0, y1, w0, w1);
        // stage the window: block j holds bytes (x = 0..7) for (y = lane & 7, z = lane >> 3)
        for (int j = w0 / 8; j < w1 / 8; ++j) {
            const int64_t db = dom_index(d, bx, j, bz);
            const uint64_t v = ((const uint64_t *)(g1 + db * 512))[lane];
            *(uint64_t *)&col[(8 * (j - w0 / 8) + (lane & 7)) * 64 + 8 * (lane >> 3)] = v;
        }
        wave_sync();
        Envelope e;
        e.k = -1;
        e.p = e.fp = e.pp = e.fpp = 0;
        const int W = w1 - w0;
        for (int q = 0; q < W; ++q) {
            const int a = col[q * 64 + lane];
            if (a == 255) continue;
            env_push(e, stk, 64, lane, q, a * a, getf);
        }
        Walker wk;
        if (e.k >= 0) walk_init(wk, e, stk, 64, lane, getf);
        for (int yb = y0; yb < y1; yb += 8) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                int v = 0xFFFF;
                if (e.k >= 0) {
                    const int val = walk_at(wk, e, stk, 64, lane, yb + t - w0, getf);
                    if (val <= R2) v = val;
                }
                ost[t * 64 + lane] = (uint16_t)v;
            }
            wave_sync();
            const int64_t db = dom_index(d, bx, yb / 8, bz);
            const uint4 o = *(const uint4 *)&ost[(lane & 7) * 64 + 8 * (lane >> 3)];
            *(uint4 *)(g2 + db * 512 + 8 * lane) = o;
            wave_sync();
        }
    }
}

// k(x, y, z) = min_z' g2(x, y, z')  + (z - z')^2 and phi for the allocated
// blocks of the column (bx, by, *).  Lane = x + 8 y, the in-block layout.
template <typename S>
__global__ __launch_bounds__(64) void k_edt_z_env(const SubmapMeta *meta, const int32_t *__restrict__ page,
                                              const uint16_t *__restrict__ g2, const S *__restrict__ D,
                                              const S *__restrict__ W, float *__restrict__ phi, int R, int HB,
                                              float vs, float tau, float dmax)
{
    __shared__ __align__(16) uint16_t col[kWin * 64];  // [position][lane]
    __shared__ __align__(16) uint8_t stk[kWin * 64];
    const Dom d = read_dom(meta);
    const int lane = threadIdx.x;
    const int C = 8 * HB;
    const int Sg = kWin - 2 * C;
    const int L = 8 * d.dim[2];
    const int nseg = L > 0 ? (L + Sg - 1) / Sg : 0;
    const int64_t ncol = (int64_t)d.dim[0] * d.dim[1] * nseg;
    const int R2 = R * R;
    auto getf = [&](int q) { return (int)col[q * 64 + lane]; };
    for (int64_t c = blockIdx.x; c < ncol; c += gridDim.x) {
        const int seg = (int)(c % nseg);
        const int64_t cc = c / nseg;
        const int bx = (int)(cc % d.dim[0]), by = (int)(cc / d.dim[0]);
        int z0, z1, w0, w1;
        segment(L, C, seg, Sg, z0, z1, w0, w1);
        for (int j = w0 / 8; j < w1 / 8; ++j) {
            const uint16_t *src = g2 + dom_index(d, bx, by, j) * 512 + lane;
#pragma unroll
            for (int t = 0; t < 8; ++t) col[(8 * (j - w0 / 8) + t) * 64 + lane] = src[64 * t];
        }
        wave_sync();
        Envelope e;
        e.k = -1;
        e.p = e.fp = e.pp = e.fpp = 0;
        const int Wn = w1 - w0;
        for (int q = 0; q < Wn; ++q) {
            const int a = col[q * 64 + lane];
            if (a == 0xFFFF) continue;
            env_push(e, stk, 64, lane, q, a, getf);
        }
        Walker wk;
        if (e.k >= 0) walk_init(wk, e, stk, 64, lane, getf);
        for (int zb = z0; zb < z1; zb += 8) {
            const int64_t idx = page[dom_index(d, bx, by, zb / 8)];
            if (idx < 0) continue;
            const S *Db = D + idx * 512 + lane;
            const S *Wb = W + idx * 512 + lane;
            float *Pb = phi + idx * 512 + lane;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float Dv = ldv(Db + 64 * t), Wv = ldv(Wb + 64 * t);
                float out;
                if (!(Wv > 0.0f)) {
                    out = __builtin_nanf("");
                } else if (fabsf(Dv) < tau) {
                    out = Dv;
                } else {
                    int best = kBig;
                    if (e.k >= 0) best = walk_at(wk, e, stk, 64, lane, zb + t - w0, getf);
                    const float sg = Dv > 0.0f ? 1.0f : -1.0f;
                    if (best > R2) out = sg * dmax;
                    else out = sg * fminf(dmax, vs * sqrtf((float)best));
                }
                Pb[64 * t] = out;
            }
        }
        wave_sync();
    }
}

// ------------------------------------------------------------------------
// Voxel-parallel passes: one 512-lane workgroup per block, one lane per
// voxel (l = x + 8y + 64z), the 2 HB + 1 neighbour blocks along the pass axis
// staged in LDS.  The min-plus search walks outward from the voxel and stops
// once d^2 reaches the best value, so it is exact; its cost follows the
// distance to the nearest site rather than the line length, which suits
// small domains where per-line envelopes leave the GPU idle.

__device__ __forceinline__ int sq8(uint8_t v) { return v == 255 ? kBig : (int)v * (int)v; }
__device__ __forceinline__ int inf16(uint16_t v) { return v == 0xFFFF ? kBig : (int)v; }

__global__ __launch_bounds__(512) void k_edt_x_vox(const SubmapMeta *meta, const uint64_t *__restrict__ sites,
                                                   uint8_t *__restrict__ g1, int R, int HB)
{
    __shared__ uint64_t wl[(2 * kMaxHalo + 1) * 8];
    const Dom d = read_dom(meta);
    const int tid = threadIdx.x;
    const int x = tid & 7, y = (tid >> 3) & 7, z = tid >> 6;
    const int nb = 2 * HB + 1;
    for (int64_t db = blockIdx.x; db < d.n; db += gridDim.x) {
        int bx, by, bz;
        dom_coords(d, db, bx, by, bz);
        if (tid < nb * 8) {
            const int i = tid >> 3, k = tid & 7;
            const int nx = bx + i - HB;
            wl[tid] = (nx >= 0 && nx < d.dim[0]) ? sites[(db + (i - HB)) * 8 + k] : 0ull;
        }
        __syncthreads();
        uint64_t lo = 0, hi = 0;
        for (int i = 0; i < nb; ++i) {
            const uint64_t byte = (wl[i * 8 + z] >> (8 * y)) & 0xFFull;
            const int pos = 8 * i;
            if (pos < 64) lo |= byte << pos;
            else hi |= byte << (pos - 64);
        }
        const int dist = nearest_bit(lo, hi, 8 * HB + x);
        g1[db * 512 + tid] = dist <= R ? (uint8_t)dist : (uint8_t)255;
        __syncthreads();
    }
}

__global__ __launch_bounds__(512) void k_edt_y_vox(const SubmapMeta *meta, const uint8_t *__restrict__ g1,
                                                   uint16_t *__restrict__ g2, int R, int HB)
{
    __shared__ __align__(16) uint32_t colw[(2 * kMaxHalo + 1) * 128];
    const uint8_t *col = (const uint8_t *)colw;
    const Dom d = read_dom(meta);
    const int tid = threadIdx.x;
    const int x = tid & 7, y = (tid >> 3) & 7, z = tid >> 6;
    const int nb = 2 * HB + 1;
    const int R2 = R * R;
    const int Y = 8 * HB + y;
    for (int64_t db = blockIdx.x; db < d.n; db += gridDim.x) {
        int bx, by, bz;
        dom_coords(d, db, bx, by, bz);
        for (int e = tid; e < nb * 128; e += 512) {
            const int i = e >> 7, w = e & 127;
            const int ny = by + i - HB;
            colw[e] = (ny >= 0 && ny < d.dim[1]) ? ((const uint32_t *)(g1 + (db + (int64_t)(i - HB) * d.dim[0]) * 512))[w]
                                                 : 0xFFFFFFFFu;
        }
        __syncthreads();
        auto at = [&](int yy) { return col[(yy >> 3) * 512 + x + 8 * (yy & 7) + 64 * z]; };
        int best = sq8(at(Y));
        for (int dd = 1; dd <= R; ++dd) {
            const int d2 = dd * dd;
            if (d2 >= best) break;
            best = min(best, min(sq8(at(Y - dd)), sq8(at(Y + dd))) + d2);
        }
        g2[db * 512 + tid] = best <= R2 ? (uint16_t)best : (uint16_t)0xFFFF;
        __syncthreads();
    }
}

template <typename S>
__global__ __launch_bounds__(512) void k_edt_z_vox(const SubmapMeta *meta, const uint64_t *__restrict__ keys,
                                                   const uint16_t *__restrict__ g2, const S *__restrict__ D,
                                                   const S *__restrict__ W, float *__restrict__ phi, int R, int HB,
                                                   float vs, float tau, float dmax)
{
    __shared__ __align__(16) uint32_t colw[(2 * kMaxHalo + 1) * 256];
    const uint16_t *col = (const uint16_t *)colw;
    const Dom d = read_dom(meta);
    const int64_t nbk = meta->n_blocks;
    const int tid = threadIdx.x;
    const int z = tid >> 6;
    const int nb = 2 * HB + 1;
    const int R2 = R * R;
    const int Z = 8 * HB + z;
    const int64_t stride_z = (int64_t)d.dim[0] * d.dim[1];
    for (int64_t j = blockIdx.x; j < nbk; j += gridDim.x) {
        int bx, by, bz;
        unpack_key(keys[j], bx, by, bz);
        bx -= d.lo[0]; by -= d.lo[1]; bz -= d.lo[2];
        const int64_t db = dom_index(d, bx, by, bz);
        for (int e = tid; e < nb * 256; e += 512) {
            const int i = e >> 8, w = e & 255;
            const int nz = bz + i - HB;
            colw[e] = (nz >= 0 && nz < d.dim[2]) ? ((const uint32_t *)(g2 + (db + (int64_t)(i - HB) * stride_z) * 512))[w]
                                                 : 0xFFFFFFFFu;
        }
        const float Dv = ldv(D + j * 512 + tid), Wv = ldv(W + j * 512 + tid);
        __syncthreads();
        float out;
        if (!(Wv > 0.0f)) {
            out = __builtin_nanf("");
        } else if (fabsf(Dv) < tau) {
            out = Dv;
        } else {
            const int base = tid & 63;
            auto at = [&](int zz) { return col[(zz >> 3) * 512 + base + 64 * (zz & 7)]; };
            int best = inf16(at(Z));
            for (int dd = 1; dd <= R; ++dd) {
                const int d2 = dd * dd;
                if (d2 >= best) break;
                best = min(best, min(inf16(at(Z - dd)), inf16(at(Z + dd))) + d2);
            }
            const float sg = Dv > 0.0f ? 1.0f : -1.0f;
            if (best > R2) out = sg * dmax;
            else out = sg * fminf(dmax, vs * sqrtf((float)best));
        }
        phi[j * 512 + tid] = out;
        __syncthreads();
    }
}

unsigned grid_for(int64_t waves)
{
    const int64_t g = (waves + 3) / 4;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

// Workgroups for a line pass: the columns (block extents along axes a and b
// of the host-side bound box) times the segments along the third axis.
static unsigned grid_cols(const covox_submap *s, int a, int b, int HB)
{
    if (!s->bound_valid) return 1;
    const int c = 3 - a - b;
    const int64_t L = 8 * (int64_t)(s->bound_hi[c] - s->bound_lo[c] + 1);
    const int64_t S = kWin - 16 * HB;
    const int64_t nseg = (L + S - 1) / S;
    const int64_t n = (int64_t)(s->bound_hi[a] - s->bound_lo[a] + 1) * (s->bound_hi[b] - s->bound_lo[b] + 1) * nseg;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 65536));
}

static int64_t bound_blocks(const covox_submap *s)
{
    if (!s->bound_valid) return 0;
    int64_t n = 1;
    for (int a = 0; a < 3; ++a) n *= (int64_t)(s->bound_hi[a] - s->bound_lo[a] + 1);
    return n;
}

int build_page(covox_ctx *ctx, covox_submap *s)
{
    if (s->page_version == s->version) return COVOX_OK;
    const int64_t nd = std::max<int64_t>(bound_blocks(s), 1);
    int rc;
    if ((rc = ensure_buffer(ctx, (void **)&s->page, &s->page_cap, nd, sizeof(int32_t), "page"))) return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->sites, &ctx->sites_cap, nd, 8 * sizeof(uint64_t), "site masks")))
        return rc;
    const float vs = (float)ctx->p.voxel_size;
    const uint64_t tmask = (uint64_t)s->tcap - 1;
    {
        TimedLaunch tl(ctx, COVOX_K_ESDF_PAGE);
        if (ctx->p.precision == COVOX_FP16)
            hipLaunchKernelGGL(k_page_sites<__half>, dim3(grid_for(nd)), dim3(256), 0, ctx->stream, s->meta,
                               s->tkeys, s->tvals, tmask, (const __half *)s->D, (const __half *)s->W, vs, s->page,
                               ctx->sites);
        else
            hipLaunchKernelGGL(k_page_sites<float>, dim3(grid_for(nd)), dim3(256), 0, ctx->stream, s->meta,
                               s->tkeys, s->tvals, tmask, (const float *)s->D, (const float *)s->W, vs, s->page,
                               ctx->sites);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "page launch"))) return rc;
    s->page_version = s->version;
    return COVOX_OK;
}

int update_esdf(covox_ctx *ctx, covox_submap *s)
{
    if (s->esdf_version == s->version) return COVOX_OK;
    const covox_params &p = ctx->p;
    const int R = (int)std::llround(p.d_max / p.voxel_size);
    const int HB = (R + 7) / 8;
    // the site masks of the page build are consumed here: rebuild them
    s->page_version = 0;
    int rc;
    if ((rc = build_page(ctx, s))) return rc;
    const int64_t nd = std::max<int64_t>(bound_blocks(s), 1);
    if ((rc = ensure_buffer(ctx, (void **)&ctx->g1, &ctx->g1_cap, nd, 512, "edt g1"))) return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->g2, &ctx->g2_cap, nd, 1024, "edt g2"))) return rc;
    const float vs = (float)p.voxel_size, tau = (float)(p.trunc_vox * p.voxel_size), dmax = (float)p.d_max;
    // Pass shape: per-line envelopes when there are enough lines to fill the
    // GPU, voxel-parallel windowed search otherwise (or as forced by
    // COVOX_EDT_MODE = window | envelope).
    const unsigned cols_y = grid_cols(s, 0, 2, HB), cols_z = grid_cols(s, 0, 1, HB);
    bool envelope = std::min(cols_y, cols_z) >= (unsigned)ctx->edt_env_min_cols;
    if (ctx->edt_mode == 1) envelope = false;
    if (ctx->edt_mode == 2) envelope = true;
    const unsigned gd = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nd, 65536));
    const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(std::min(s->nb_upper, s->cap), 65536));
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_X);
        hipLaunchKernelGGL(k_edt_x_vox, dim3(gd), dim3(512), 0, ctx->stream, s->meta, ctx->sites, ctx->g1, R, HB);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Y);
        if (envelope)
            hipLaunchKernelGGL(k_edt_y_env, dim3(cols_y), dim3(64), 0, ctx->stream, s->meta, ctx->g1, ctx->g2, R, HB);
        else
            hipLaunchKernelGGL(k_edt_y_vox, dim3(gd), dim3(512), 0, ctx->stream, s->meta, ctx->g1, ctx->g2, R, HB);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Z);
        const bool h = p.precision == COVOX_FP16;
        if (envelope && h)
            hipLaunchKernelGGL(k_edt_z_env<__half>, dim3(cols_z), dim3(64), 0, ctx->stream, s->meta, s->page, ctx->g2,
                               (const __half *)s->D, (const __half *)s->W, s->phi, R, HB, vs, tau, dmax);
        else if (envelope)
            hipLaunchKernelGGL(k_edt_z_env<float>, dim3(cols_z), dim3(64), 0, ctx->stream, s->meta, s->page, ctx->g2,
                               (const float *)s->D, (const float *)s->W, s->phi, R, HB, vs, tau, dmax);
        else if (h)
            hipLaunchKernelGGL(k_edt_z_vox<__half>, dim3(gb), dim3(512), 0, ctx->stream, s->meta, s->keys, ctx->g2,
                               (const __half *)s->D, (const __half *)s->W, s->phi, R, HB, vs, tau, dmax);
        else
            hipLaunchKernelGGL(k_edt_z_vox<float>, dim3(gb), dim3(512), 0, ctx->stream, s->meta, s->keys, ctx->g2,
                               (const float *)s->D, (const float *)s->W, s->phi, R, HB, vs, tau, dmax);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "esdf launch"))) return rc;
    s->esdf_version = s->version;
    return COVOX_OK;
}

}  // namespace covox
