// Raycast TSDF integration (paper Sec. III-C: a ray from the optical centre
// through every observed point updates each voxel it crosses up to the
// truncation distance behind the point; Sec. III-D: count and allocate the
// new blocks, then merge the frame's contributions per voxel).
//
// One frame is seven launches on the context stream:
//   fill_u32        clears the block flags of the frustum's block box;
//   k_ray_mark      one lane per pixel walks its ray and flags each box block
//                   that receives a contribution (in an LDS bitmap per
//                   workgroup, written out once per flagged block);
//   k_ray_resolve   one lane per box block: a flagged block that exists gets
//                   its buffer index, the others stay NEW;
//   k_scan          (shared with projection mapping) compacts the flags in
//                   key order, checks capacity, numbers the new blocks;
//   k_ray_activate  one wave per new block: key, hash insert, zeroed voxels;
//   k_ray_accum     one lane per pixel walks its ray again and adds w and t w
//                   of each contribution to binary64 accumulators of the
//                   voxel: lanes of a wave that reach the same voxel in the
//                   same step are summed in registers, the workgroup's
//                   16 x 16 pixel tile sums its voxels in an LDS table, and
//                   the table is flushed with global FP64 atomics; with
//                   constant weights, contributions clamped to tau travel as
//                   integer counts;
//   k_ray_apply     one wave per touched block: W' = W + sw, D' = (D W + stw)
//                   / W' where sw > 0, and the accumulators are cleared.
// The paper orders the merge by sorting the contributions by voxel address;
// here the sums are formed by hardware FP64 atomics instead, in any order.
// The walk takes each crossing parameter as ((i + [u > 0]) vs - o) * (1 / u)
// with the reciprocal rounded once per ray: a multiply per step instead of a
// division, and faithful to 2^-22 relative of the exact crossing.  A walk
// with correctly rounded crossings can therefore take another step only where
// two crossing parameters (or the nearest one and the segment end) lie within
// that margin of each other; elsewhere block keys, buffer indices and the set
// of contributions are those of the exact traversal.  The binary64 sums of
// binary32 products depend on their order only at rare rounding ties.
#include "covox_impl.h"

#include <math.h>

#include <algorithm>

namespace covox {

namespace {

constexpr uint32_t kNewFlag = 0xFFFFFFFFu;  // the compaction's NEW marker

// A ray and the state of its grid walk (Amanatides and Woo, Eurographics
// 1987).  Voxel i spans [i vs, (i + 1) vs) per axis; sn[a] is the ray
// parameter of the next boundary along axis a, computed from the index.
struct Ray {
    float o[3], u[3], iu[3], r, s1, w;
    int32_t i[3];
    int32_t step[3];
    float sn[3];
    int32_t left;  // voxels the walk may still visit
};

__device__ __forceinline__ float next_boundary(const Ray &R, int a, float vs)
{
    return (((float)(R.i[a] + (R.step[a] > 0 ? 1 : 0)) * vs) - R.o[a]) * R.iu[a];
}

// Sets up the ray of pixel (col, row); false when its depth is invalid.
__device__ __forceinline__ bool ray_setup(const FrameArgs &f, float vs, float tau, float maxr, int col, int row,
                                          Ray &R)
{
    const float z = f.depth[(int64_t)row * f.W + col];
    if (!(z > 0.0f && z <= maxr)) return false;
    const float xc = (((float)col - f.K[2]) * z) / f.K[0];
    const float yc = (((float)row - f.K[3]) * z) / f.K[1];
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (f.Rs[3 * k] * xc + f.Rs[3 * k + 1] * yc) + f.Rs[3 * k + 2] * z;
    R.r = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    R.s1 = R.r + tau;
    const float s0 = f.ray_carve ? 0.0f : fmaxf(R.r - tau, 0.0f);
    R.left = 3 * (int32_t)ceilf((R.s1 - s0) / vs) + 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.u[a] = d[a] / R.r;
        R.o[a] = f.o[a];
        const float e = R.o[a] + s0 * R.u[a];
        R.i[a] = (int32_t)floorf(e / vs);
        R.step[a] = R.u[a] > 0.0f ? 1 : (R.u[a] < 0.0f ? -1 : 0);
        R.iu[a] = R.step[a] ? 1.0f / R.u[a] : 0.0f;
        R.sn[a] = R.step[a] ? next_boundary(R, a, vs) : INFINITY;
    }
    R.w = f.weight_mode == COVOX_WEIGHT_INV_DEPTH2 ? 1.0f / (z * z) : 1.0f;
    return true;
}

// Moves to the next voxel; false when the walk has ended (the nearest
// boundary lies at or beyond s1, or the step bound is reached).
// The axis is chosen and applied with selects only (constant indices), so
// that the ray stays in registers.
__device__ __forceinline__ bool ray_next(Ray &R, float vs)
{
    const bool y_first = R.sn[1] < R.sn[0];
    const float m01 = y_first ? R.sn[1] : R.sn[0];
    const bool z_first = R.sn[2] < m01;
    const float smin = z_first ? R.sn[2] : m01;
    if (!(smin < R.s1)) return false;
    if (--R.left <= 0) return false;
    const bool pick[3] = {!z_first && !y_first, !z_first && y_first, z_first};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R.i[a] += pick[a] ? R.step[a] : 0;
        const float nb = next_boundary(R, a, vs);
        R.sn[a] = pick[a] ? nb : R.sn[a];
    }
    return true;
}

// Contribution of the current voxel: t = min(sdf, tau) when sdf >= -tau.
__device__ __forceinline__ bool ray_contrib(const Ray &R, float vs, float tau, float &t)
{
    float c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = ((float)R.i[a] + 0.5f) * vs;
    const float proj = ((c[0] - R.o[0]) * R.u[0] + (c[1] - R.o[1]) * R.u[1]) + (c[2] - R.o[2]) * R.u[2];
    const float sdf = R.r - proj;
    if (!(sdf >= -tau)) return false;
    t = fminf(sdf, tau);
    return true;
}

// Pixel of a lane: workgroups of 256 lanes cover 16 x 16 pixel tiles, each
// wave an 8 x 8 quarter, so that the rays of a wave stay close together.
__device__ __forceinline__ void lane_pixel(int &col, int &row)
{
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    col = (int)blockIdx.x * 16 + (wv & 1) * 8 + (lane & 7);
    row = (int)blockIdx.y * 16 + (wv >> 1) * 8 + (lane >> 3);
}

// Block flags of a workgroup are first set in an LDS bitmap over the box
// (boxes of up to kMarkBits blocks) and then written out once each.
constexpr int kMarkWords = 2048;
constexpr int64_t kMarkBits = 32 * kMarkWords;

__global__ __launch_bounds__(256) void k_ray_mark(FrameArgs f, float vs, float tau, float maxr,
                                                  uint32_t *__restrict__ cand, int64_t n_box)
{
    __shared__ uint32_t s_bits[kMarkWords];
    const bool local = n_box <= kMarkBits;  // uniform
    const int nw = (int)((n_box + 31) / 32);
    if (local) {
        for (int k = threadIdx.x; k < nw; k += blockDim.x) s_bits[k] = 0u;
        __syncthreads();
    }
    int col, row;
    lane_pixel(col, row);
    Ray R;
    if (col < f.W && row < f.H && ray_setup(f, vs, tau, maxr, col, row, R)) {
        int64_t last = -1;
        do {
            float t;
            if (ray_contrib(R, vs, tau, t)) {
                // the box holds every voxel a ray can cross (host-side construction)
                const int jx = (R.i[0] >> 3) - f.blo[0], jy = (R.i[1] >> 3) - f.blo[1], jz = (R.i[2] >> 3) - f.blo[2];
                if (jx >= 0 && jx < f.bdim[0] && jy >= 0 && jy < f.bdim[1] && jz >= 0 && jz < f.bdim[2]) {
                    const int64_t j = ((int64_t)jx * f.bdim[1] + jy) * f.bdim[2] + jz;
                    if (j != last) {
                        const uint32_t bit = 1u << (j & 31);
                        if (!local) cand[j] = kNewFlag;
                        else if (!(s_bits[j >> 5] & bit)) atomicOr(&s_bits[j >> 5], bit);  // set once
                        last = j;
                    }
                }
            }
        } while (ray_next(R, vs));
    }
    if (local) {
        __syncthreads();
        for (int k = threadIdx.x; k < nw; k += blockDim.x) {
            uint32_t bits = s_bits[k];
            while (bits) {
                const int b = __ffs(bits) - 1;
                cand[32 * (int64_t)k + b] = kNewFlag;
                bits &= bits - 1u;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_ray_resolve(FrameArgs f, const uint64_t *__restrict__ tkeys,
                                                     const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                     uint32_t *__restrict__ cand, int64_t n_box)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_box || cand[j] != kNewFlag) return;
    const int64_t nz = f.bdim[2], ny = f.bdim[1];
    const int32_t bz = f.blo[2] + (int32_t)(j % nz);
    const int32_t by = f.blo[1] + (int32_t)((j / nz) % ny);
    const int32_t bx = f.blo[0] + (int32_t)(j / (nz * ny));
    const int64_t idx = hash_find(tkeys, tvals, tmask, pack_key(bx, by, bz));
    if (idx >= 0) cand[j] = (uint32_t)idx + 1u;
}

__global__ __launch_bounds__(256) void k_ray_activate(const SubmapMeta *__restrict__ meta,
                                                      const uint64_t *__restrict__ t_key,
                                                      const uint32_t *__restrict__ t_idx, uint64_t *keys, float *D,
                                                      float *W, uint64_t *tkeys, uint32_t *tvals, uint64_t tmask)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n_t = meta->n_touched;
    for (int64_t t = wave; t < n_t; t += nwaves) {
        const uint32_t v = t_idx[t];
        if (!(v >> 31)) continue;  // uniform across the wave
        const int64_t idx = v & 0x7FFFFFFFu;
        if (lane == 0) {
            keys[idx] = t_key[t];
            hash_insert(tkeys, tvals, tmask, t_key[t], (uint32_t)idx);
        }
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            D[idx * 512 + lane + 64 * z] = 0.0f;
            W[idx * 512 + lane + 64 * z] = 0.0f;
        }
    }
}

// Per-workgroup accumulation table in LDS: the 256 rays of a 16 x 16 pixel
// tile run inside a narrow cone and cross mostly the same voxels, so their
// contributions are summed here and each voxel costs the workgroup one pair
// of global atomics when the table is flushed.  Open addressing with linear
// probing; a contribution that finds no slot within kAccProbe probes goes
// to the global accumulators directly.
constexpr int kAccSlots = 1024;
constexpr int kAccProbe = 16;
constexpr unsigned long long kAccEmpty = ~0ull;

__device__ __forceinline__ void add_global(double *acc, int64_t addr, double vw, double vtw)
{
    unsafeAtomicAdd(acc + 2 * addr, vw);
    unsafeAtomicAdd(acc + 2 * addr + 1, vtw);
}

// With constant weights, a contribution clamped to tau (free space: most of
// them) is (w, t w) = (1, tau), so it is counted instead: an integer per LDS
// slot, ballot popcounts for a wave's group.  The count c enters the binary64
// sums as c and c tau, both exact.
__global__ __launch_bounds__(256) void k_ray_accum(FrameArgs f, float vs, float tau, float maxr,
                                                   const SubmapMeta *__restrict__ meta,
                                                   const uint64_t *__restrict__ tkeys,
                                                   const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                   double *__restrict__ acc)
{
    __shared__ unsigned long long s_key[kAccSlots];
    __shared__ double s_w[kAccSlots], s_tw[kAccSlots];
    __shared__ uint32_t s_cnt[kAccSlots];
    if (meta->n_touched == 0) return;  // uniform: nothing committed (capacity failure, or no contribution)
    for (int k = threadIdx.x; k < kAccSlots; k += blockDim.x) {
        s_key[k] = kAccEmpty;
        s_w[k] = 0.0;
        s_tw[k] = 0.0;
        s_cnt[k] = 0u;
    }
    __syncthreads();
    const bool counted = f.weight_mode == COVOX_WEIGHT_CONSTANT;  // uniform
    const double tau_d = (double)tau;
    const int lane = threadIdx.x & 63;
    int col, row;
    lane_pixel(col, row);
    Ray R;
    bool active = col < f.W && row < f.H && ray_setup(f, vs, tau, maxr, col, row, R);
    int32_t cb[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    int64_t base = -1;
    // The loop runs while any lane of the wave walks, so that every lane
    // takes part in the ballots and shuffles below.
    while (__ballot(active)) {
        bool has = false;
        int64_t addr = -1;
        double vw = 0.0, vtw = 0.0;
        uint32_t cnt = 0;  // clamped contributions carried as a count
        if (active) {
            float t;
            if (ray_contrib(R, vs, tau, t)) {
                const int32_t bx = R.i[0] >> 3, by = R.i[1] >> 3, bz = R.i[2] >> 3;
                if (bx != cb[0] || by != cb[1] || bz != cb[2]) {
                    cb[0] = bx; cb[1] = by; cb[2] = bz;
                    base = hash_find(tkeys, tvals, tmask, pack_key(bx, by, bz));
                }
                if (base >= 0) {
                    has = true;
                    addr = base * 512 + (R.i[0] & 7) + 8 * (R.i[1] & 7) + 64 * (R.i[2] & 7);
                    if (counted && t == tau) {
                        cnt = 1u;
                    } else {
                        vw = (double)R.w;
                        vtw = (double)t * (double)R.w;  // exact in binary64
                    }
                }
            }
            active = ray_next(R, vs);
        }
        // lanes that reached the first contributing lane's voxel: summed in
        // registers, the leader carries the sum
        const uint64_t m = __ballot(has);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            const int64_t la = __shfl(addr, leader, 64);
            const bool in = has && addr == la;
            const uint64_t g = __ballot(in);
            if (__popcll(g) > 1) {
                const uint32_t gc = (uint32_t)__popcll(__ballot(in && cnt != 0u));
                double a = 0.0, b = 0.0;
                if (__ballot(in && cnt == 0u)) {  // some member carries a value
                    a = in ? vw : 0.0;
                    b = in ? vtw : 0.0;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        a += __shfl_xor(a, off, 64);
                        b += __shfl_xor(b, off, 64);
                    }
                }
                if (in) {
                    has = lane == leader;
                    vw = a;
                    vtw = b;
                    cnt = gc;
                }
            }
        }
        if (has) {
            const unsigned long long key = (unsigned long long)addr;
            uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 54);  // 10 bits
            bool done = false;
            for (int p = 0; p < kAccProbe && !done; ++p, h = (h + 1) & (kAccSlots - 1)) {
                unsigned long long k = s_key[h];
                if (k == kAccEmpty) {
                    k = atomicCAS(&s_key[h], kAccEmpty, key);  // the old value: empty, or the winner's key
                    if (k == kAccEmpty) k = key;
                }
                if (k == key) {
                    if (cnt) atomicAdd(&s_cnt[h], cnt);
                    if (vw != 0.0) {
                        __hip_atomic_fetch_add(&s_w[h], vw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        __hip_atomic_fetch_add(&s_tw[h], vtw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    done = true;
                }
            }
            if (!done) add_global(acc, addr, (double)cnt + vw, (double)cnt * tau_d + vtw);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kAccSlots; k += blockDim.x)
        if (s_key[k] != kAccEmpty) {
            const double c = (double)s_cnt[k];
            add_global(acc, (int64_t)s_key[k], c + s_w[k], c * tau_d + s_tw[k]);
        }
}

__global__ __launch_bounds__(256) void k_ray_apply(SubmapMeta *__restrict__ meta, const uint32_t *__restrict__ t_idx,
                                                   float *D, float *W, double *__restrict__ acc,
                                                   uint8_t *__restrict__ dirty)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n_t = meta->n_touched;
    for (int64_t t = wave; t < n_t; t += nwaves) {
        const int64_t idx = t_idx[t] & 0x7FFFFFFFu;
        int n_ok = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const int64_t o = idx * 512 + lane + 64 * z;
            double2 *a2 = reinterpret_cast<double2 *>(acc) + o;
            const double2 sum = *a2;
            const bool ok = sum.x > 0.0;
            n_ok += __popcll(__ballot(ok));
            if (ok) {
                const float Wold = W[o], Dold = D[o];
                const float Wn = Wold + (float)sum.x;
                const float Dn = ((Dold * Wold) + (float)sum.y) / Wn;
                D[o] = Dn;
                W[o] = Wn;
                *a2 = make_double2(0.0, 0.0);
            }
        }
        if (lane == 0) {
            atomicAdd(&meta->n_updates, (unsigned long long)n_ok);
            dirty[idx] = 1;
        }
    }
}

}  // namespace

int ensure_ray_acc(covox_ctx *ctx)
{
    const int64_t need = ctx->p.block_capacity;
    if (ctx->ray_acc && ctx->ray_acc_blocks >= need) return COVOX_OK;
    if (ctx->capturing) return fail(ctx, COVOX_EINVAL, "raycast accumulators cannot be allocated under capture");
    int rc;
    if (ctx->ray_acc) {
        if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "raycast accumulator sync"))) return rc;
        (void)hipFree(ctx->ray_acc);
        ctx->ray_acc = nullptr;
        ctx->ray_acc_blocks = 0;
    }
    const size_t bytes = (size_t)need * 512 * 2 * sizeof(double);
    if ((rc = hip_check(ctx, hipMalloc((void **)&ctx->ray_acc, bytes), "raycast accumulators"))) return rc;
    if ((rc = hip_check(ctx, hipMemset(ctx->ray_acc, 0, bytes), "raycast accumulator clear"))) return rc;
    ctx->ray_acc_blocks = need;
    return COVOX_OK;
}

int raycast_frame(covox_ctx *ctx, covox_submap *s, const float *depth, int32_t H, int32_t W, const float K[4],
                  const double T_wc[16], bool *maybe_full)
{
    const covox_params &p = ctx->p;
    FrameArgs f;
    int64_t n_box = 0;
    int rc = prepare_frame(ctx, s, depth, H, W, K, T_wc, f, n_box);
    if (rc) return rc;
    if (p.precision != COVOX_FP32) return fail(ctx, COVOX_EINVAL, "integrate: raycasting needs FP32 storage");
    {
        // Longest ray: to depth max_range + tau through the outermost pixel
        // edge.  Walks are bounded by 3 x its length in voxels + 6 steps.
        const double zf = p.max_range + p.trunc_vox * p.voxel_size;
        const double ax = std::max(std::fabs(-0.5 - K[2]), std::fabs(W - 0.5 - K[2])) / K[0];
        const double ay = std::max(std::fabs(-0.5 - K[3]), std::fabs(H - 0.5 - K[3])) / K[1];
        if (zf * std::sqrt(1.0 + ax * ax + ay * ay) / p.voxel_size > 65536.0)
            return fail(ctx, COVOX_EINVAL, "integrate: rays longer than 65536 voxels (check K and max_range)");
    }
    if ((rc = ensure_ray_acc(ctx))) return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->cand, &ctx->cand_cap, n_box, sizeof(uint32_t), "candidates")))
        return rc;
    // touched keys, then (from n_box on) the new blocks' keys (k_scan)
    if ((rc = ensure_buffer(ctx, (void **)&ctx->t_key, &ctx->t_key_cap, 2 * n_box, sizeof(uint64_t), "touched keys")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->t_idx, &ctx->t_idx_cap, n_box, sizeof(uint32_t), "touched index")))
        return rc;

    const float vs = (float)p.voxel_size, tau = (float)(p.trunc_vox * p.voxel_size), maxr = (float)p.max_range;
    const uint64_t tmask = (uint64_t)s->tcap - 1;
    const int64_t table_limit = (int64_t)(0.85 * (double)s->tcap);
    const dim3 pix_grid((unsigned)((W + 15) / 16), (unsigned)((H + 15) / 16));
    const unsigned box_grid = (unsigned)((n_box + 255) / 256);
    const unsigned wave_grid = (unsigned)std::min<int64_t>((n_box + 3) / 4, 65536);
    float *Dp = (float *)s->D, *Wp = (float *)s->W;
    refresh_block_bound(s, n_box);
    {
        TimedLaunch tl(ctx, COVOX_K_RAY_MARK);
        fill_u32(ctx->stream, ctx->cand, 0u, n_box);
        hipLaunchKernelGGL(k_ray_mark, pix_grid, dim3(256), 0, ctx->stream, f, vs, tau, maxr, ctx->cand, n_box);
        hipLaunchKernelGGL(k_ray_resolve, dim3(box_grid), dim3(256), 0, ctx->stream, f, s->tkeys, s->tvals, tmask,
                           ctx->cand, n_box);
    }
    launch_block_scan(ctx, s, f, n_box, table_limit);
    {
        TimedLaunch tl(ctx, COVOX_K_RAY_ACCUM);
        hipLaunchKernelGGL(k_ray_activate, dim3(wave_grid), dim3(256), 0, ctx->stream, s->meta, ctx->t_key, ctx->t_idx,
                           s->keys, Dp, Wp, s->tkeys, s->tvals, tmask);
        hipLaunchKernelGGL(k_ray_accum, pix_grid, dim3(256), 0, ctx->stream, f, vs, tau, maxr, s->meta, s->tkeys,
                           s->tvals, tmask, ctx->ray_acc);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_RAY_APPLY);
        hipLaunchKernelGGL(k_ray_apply, dim3(wave_grid), dim3(256), 0, ctx->stream, s->meta, ctx->t_idx, Dp, Wp,
                           ctx->ray_acc, s->dirty);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "raycast launch"))) return rc;
    s->nb_upper += n_box;
    grow_bounds(s, f);
    s->version++;
    *maybe_full = s->nb_upper > s->cap || s->nb_upper > table_limit;
    return COVOX_OK;
}

}  // namespace covox
