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

__global__ __launch_bounds__(256) void k_edt_x(const SubmapMeta *meta, const uint64_t *__restrict__ sites,
                                               uint8_t *__restrict__ g1, int R, int HB)
{
    __shared__ uint64_t wl[4][(2 * kMaxHalo + 1) * 8];
    const Dom d = read_dom(meta);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nb = 2 * HB + 1;
    const int x = lane & 7, y = lane >> 3;
    uint64_t *w = wl[wid];
    for (int64_t db = wave; db < d.n; db += nwaves) {
        int bx, by, bz;
        dom_coords(d, db, bx, by, bz);
        for (int e = lane; e < nb * 8; e += 64) {
            const int i = e >> 3, z = e & 7;
            const int nx = bx + i - HB;
            w[e] = (nx >= 0 && nx < d.dim[0]) ? sites[(db + (i - HB)) * 8 + z] : 0ull;
        }
        wave_sync();
        uint8_t out[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            uint64_t lo = 0, hi = 0;
            for (int i = 0; i < nb; ++i) {
                const uint64_t byte = (w[i * 8 + z] >> (8 * y)) & 0xFFull;
                const int pos = 8 * i;
                if (pos < 64) lo |= byte << pos;
                else hi |= byte << (pos - 64);
            }
            const int dist = nearest_bit(lo, hi, 8 * HB + x);
            out[z] = dist <= R ? (uint8_t)dist : (uint8_t)255;
        }
        wave_sync();
#pragma unroll
        for (int z = 0; z < 8; ++z) g1[db * 512 + lane + 64 * z] = out[z];
    }
}

__device__ __forceinline__ int sq8(uint8_t v) { return v == 255 ? kBig : (int)v * (int)v; }
__device__ __forceinline__ int inf16(uint16_t v) { return v == 0xFFFF ? kBig : (int)v; }

__global__ __launch_bounds__(256) void k_edt_y(const SubmapMeta *meta, const uint8_t *__restrict__ g1,
                                               uint16_t *__restrict__ g2, int R, int HB)
{
    __shared__ uint64_t col[4][(2 * kMaxHalo + 1) * 64];  // (2HB+1) blocks x 512 bytes per wave
    const Dom d = read_dom(meta);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nb = 2 * HB + 1;
    const int x = lane & 7, y = lane >> 3;
    const int R2 = R * R;
    uint8_t *c8 = (uint8_t *)col[wid];
    const int64_t stride_y = d.dim[0];
    for (int64_t db = wave; db < d.n; db += nwaves) {
        int bx, by, bz;
        dom_coords(d, db, bx, by, bz);
        for (int i = 0; i < nb; ++i) {
            const int ny = by + i - HB;
            uint64_t v = ~0ull;
            if (ny >= 0 && ny < d.dim[1])
                v = ((const uint64_t *)(g1 + (db + (int64_t)(i - HB) * stride_y) * 512))[lane];
            col[wid][i * 64 + lane] = v;
        }
        wave_sync();
        uint16_t out[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const int Y = 8 * HB + y;
            auto at = [&](int yy) { return c8[(yy >> 3) * 512 + x + 8 * (yy & 7) + 64 * z]; };
            int best = sq8(at(Y));
            for (int dd = 1; dd <= R; ++dd) {
                const int d2 = dd * dd;
                if (d2 >= best) break;
                const int a = sq8(at(Y - dd)), b = sq8(at(Y + dd));
                best = min(best, min(a, b) + d2);
            }
            out[z] = best <= R2 ? (uint16_t)best : (uint16_t)0xFFFF;
        }
        wave_sync();
#pragma unroll
        for (int z = 0; z < 8; ++z) g2[db * 512 + lane + 64 * z] = out[z];
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_edt_z(const SubmapMeta *meta, const uint64_t *__restrict__ keys,
                                               const uint16_t *__restrict__ g2, const S *__restrict__ D,
                                               const S *__restrict__ W, float *__restrict__ phi, int R, int HB,
                                               float vs, float tau, float dmax)
{
    __shared__ uint64_t col[4][(2 * kMaxHalo + 1) * 128];  // (2HB+1) blocks x 512 u16 per wave
    const Dom d = read_dom(meta);
    const int64_t nbk = meta->n_blocks;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nb = 2 * HB + 1;
    const int R2 = R * R;
    const uint16_t *c16 = (const uint16_t *)col[wid];
    const int64_t stride_z = (int64_t)d.dim[0] * d.dim[1];
    for (int64_t j = wave; j < nbk; j += nwaves) {
        int bx, by, bz;
        unpack_key(keys[j], bx, by, bz);
        bx -= d.lo[0]; by -= d.lo[1]; bz -= d.lo[2];
        const int64_t db = dom_index(d, bx, by, bz);
        for (int i = 0; i < nb; ++i) {
            const int nz = bz + i - HB;
            uint64_t v0 = ~0ull, v1 = ~0ull;
            if (nz >= 0 && nz < d.dim[2]) {
                const uint64_t *src = (const uint64_t *)(g2 + (db + (int64_t)(i - HB) * stride_z) * 512);
                v0 = src[2 * lane];
                v1 = src[2 * lane + 1];
            }
            col[wid][i * 128 + 2 * lane] = v0;
            col[wid][i * 128 + 2 * lane + 1] = v1;
        }
        wave_sync();
        const S *Db = D + j * 512 + lane;
        const S *Wb = W + j * 512 + lane;
        float *Pb = phi + j * 512 + lane;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const float Dv = ldv(Db + 64 * z), Wv = ldv(Wb + 64 * z);
            float out;
            if (!(Wv > 0.0f)) {
                out = __builtin_nanf("");
            } else if (fabsf(Dv) < tau) {
                out = Dv;
            } else {
                const int Z = 8 * HB + z;
                auto at = [&](int zz) { return c16[(zz >> 3) * 512 + lane + 64 * (zz & 7)]; };
                int best = inf16(at(Z));
                for (int dd = 1; dd <= R; ++dd) {
                    const int d2 = dd * dd;
                    if (d2 >= best) break;
                    const int a = inf16(at(Z - dd)), b = inf16(at(Z + dd));
                    best = min(best, min(a, b) + d2);
                }
                const float sg = Dv > 0.0f ? 1.0f : -1.0f;
                if (best > R2) out = sg * dmax;
                else out = sg * fminf(dmax, vs * sqrtf((float)best));
            }
            Pb[64 * z] = out;
        }
        wave_sync();
    }
}

unsigned grid_for(int64_t waves)
{
    const int64_t g = (waves + 3) / 4;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

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
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_X);
        hipLaunchKernelGGL(k_edt_x, dim3(grid_for(nd)), dim3(256), 0, ctx->stream, s->meta, ctx->sites, ctx->g1, R,
                           HB);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Y);
        hipLaunchKernelGGL(k_edt_y, dim3(grid_for(nd)), dim3(256), 0, ctx->stream, s->meta, ctx->g1, ctx->g2, R,
                           HB);
    }
    const int64_t nbk = std::max<int64_t>(1, std::min(s->nb_upper, s->cap));
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Z);
        if (p.precision == COVOX_FP16)
            hipLaunchKernelGGL(k_edt_z<__half>, dim3(grid_for(nbk)), dim3(256), 0, ctx->stream, s->meta, s->keys,
                               ctx->g2, (const __half *)s->D, (const __half *)s->W, s->phi, R, HB, vs, tau, dmax);
        else
            hipLaunchKernelGGL(k_edt_z<float>, dim3(grid_for(nbk)), dim3(256), 0, ctx->stream, s->meta, s->keys,
                               ctx->g2, (const float *)s->D, (const float *)s->W, s->phi, R, HB, vs, tau, dmax);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "esdf launch"))) return rc;
    s->esdf_version = s->version;
    return COVOX_OK;
}

}  // namespace covox
