// Incremental ESDF by wavefront propagation (paper Sec. III-E: voxels that
// become occupied or free seed work in per-block queues, a wave processes a
// block, every axis of the block is swept, block faces hand better
// distances to the neighbours, repeated until nothing changes).
//
// Each voxel of an allocated block keeps its nearest known site (a packed
// offset) and the squared distance k to it in voxels^2, k <= R^2.  One
// update:
//   k_wf_sites    one wave per block: site masks (observed, |D| <= vs);
//   k_wf_seed     one wave per block: blocks allocated since the last update
//                 start empty, sites take themselves (k = 0), voxels whose
//                 parent is no longer a site lose it; changed blocks are
//                 queued;
//   rounds, until the queue is empty (three launches each):
//     k_wf_list   one workgroup: compacts and clears the queue flags;
//     k_wf_round  one wave per queued block, state in LDS: the six faces
//                 take the parents of the neighbours' face voxels from the
//                 previous round's state, then forward and backward sweeps
//                 along x, y, z (one lane per line); the block is written to
//                 the second buffer and, if it changed, it and its six
//                 neighbours are flagged for the next round;
//     k_wf_commit one wave per queued block: second buffer -> state;
//   k_wf_phi      one wave per block: phi as for the exact EDT, from k.
// Rounds read only the previous round's state (double buffering), so the
// result does not depend on scheduling; all of it is integer arithmetic.
#include "covox_impl.h"

#include <math.h>

#include <algorithm>

namespace covox {

namespace {

constexpr int32_t kWfInf = INT32_MAX;
constexpr int32_t kWfNone = -1;

__device__ __forceinline__ int32_t wf_pack(int dx, int dy, int dz)
{
    return (dx + 128) | ((dy + 128) << 8) | ((dz + 128) << 16);
}

// v takes the parent of its neighbour u (k_u, p_u; e = u - v) when nearer
// and within R.
__device__ __forceinline__ void wf_offer(int32_t &kv, int32_t &pv, int32_t ku, int32_t pu, int ex, int ey, int ez,
                                         int R2)
{
    if (ku == kWfInf) return;
    const int ox = (pu & 255) - 128 + ex, oy = ((pu >> 8) & 255) - 128 + ey, oz = ((pu >> 16) & 255) - 128 + ez;
    const int k = ox * ox + oy * oy + oz * oz;
    if (k > R2 || k >= kv) return;
    kv = k;
    pv = wf_pack(ox, oy, oz);
}

template <typename S> __device__ __forceinline__ float ldw(const S *p);
template <> __device__ __forceinline__ float ldw<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldw<__half>(const __half *p) { return __half2float(*p); }

template <typename S>
__global__ __launch_bounds__(256) void k_wf_sites(const SubmapMeta *__restrict__ meta, const S *__restrict__ D,
                                                  const S *__restrict__ W, float vs, uint64_t *__restrict__ sites)
{
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= meta->n_blocks) return;  // uniform across the wave
    uint64_t w = 0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const float Dv = ldw(D + j * 512 + lane + 64 * z), Wv = ldw(W + j * 512 + lane + 64 * z);
        const uint64_t m = __ballot(Wv > 0.0f && fabsf(Dv) <= vs);
        if (lane == z) w = m;
    }
    if (lane < 8) sites[j * 8 + lane] = w;
}

__global__ __launch_bounds__(256) void k_wf_seed(const SubmapMeta *__restrict__ meta, const int64_t *__restrict__ wn,
                                                 const uint64_t *__restrict__ keys, const uint64_t *__restrict__ tkeys,
                                                 const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                 const uint64_t *__restrict__ sites, int32_t *__restrict__ wk,
                                                 int32_t *__restrict__ wp, uint32_t *__restrict__ flag)
{
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (j >= meta->n_blocks) return;  // uniform across the wave
    const bool fresh = j >= *wn;
    int bx, by, bz;
    unpack_key(keys[j], bx, by, bz);
    const int x = 8 * bx + (lane & 7), y = 8 * by + (lane >> 3);
    bool dirty = fresh;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int64_t o = j * 512 + lane + 64 * z;
        int32_t k = fresh ? kWfInf : wk[o], p = fresh ? kWfNone : wp[o];
        if ((sites[j * 8 + z] >> lane) & 1ull) {
            if (k != 0) { k = 0; p = wf_pack(0, 0, 0); dirty = true; }
        } else if (k != kWfInf) {
            const int sx = x + (p & 255) - 128, sy = y + ((p >> 8) & 255) - 128, sz = 8 * bz + z + ((p >> 16) & 255) - 128;
            const int64_t sb = hash_find(tkeys, tvals, tmask, pack_key(sx >> 3, sy >> 3, sz >> 3));
            const int sl = (sx & 7) + 8 * (sy & 7);
            if (sb < 0 || !((sites[sb * 8 + (sz & 7)] >> sl) & 1ull)) {
                k = kWfInf;
                p = kWfNone;
                dirty = true;
            }
        }
        wk[o] = k;
        wp[o] = p;
    }
    if (__ballot(dirty) && lane == 0) flag[j] = 1u;
}

// Compacts the flagged blocks j < n_blocks into list[0 .. *count) in
// ascending order and clears the flags.
__global__ __launch_bounds__(1024) void k_wf_list(const SubmapMeta *__restrict__ meta, uint32_t *__restrict__ flag,
                                                  int32_t *__restrict__ list, int32_t *__restrict__ count,
                                                  int64_t *__restrict__ total)
{
    __shared__ int32_t wsum[16];
    const int64_t n = meta->n_blocks;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int32_t base = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t j = c0 + tid;
        const bool f = j < n && flag[j] != 0u;
        if (j < n && f) flag[j] = 0u;
        const uint64_t m = __ballot(f);
        if (lane == 0) wsum[wid] = __popcll(m);
        __syncthreads();
        int32_t before = 0, all = 0;
        for (int w = 0; w < 16; ++w) {
            if (w < wid) before += wsum[w];
            all += wsum[w];
        }
        if (f) list[base + before + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)j;
        base += all;
        __syncthreads();
    }
    if (tid == 0) {
        *count = base;
        *total += base;
    }
}

__device__ __forceinline__ int lin3(int x, int y, int z) { return x + 8 * y + 64 * z; }

__global__ __launch_bounds__(256) void k_wf_round(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                                                  const uint64_t *__restrict__ keys, const uint64_t *__restrict__ tkeys,
                                                  const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                  const int32_t *__restrict__ wk, const int32_t *__restrict__ wp,
                                                  int32_t *__restrict__ nk, int32_t *__restrict__ np,
                                                  uint32_t *__restrict__ flag, int R2)
{
    __shared__ int32_t sk[4][512], sp[4][512];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t t = blockIdx.x * 4 + wid;
    if (t >= *count) return;  // uniform across the wave
    const int64_t j = list[t];
    int32_t *K = sk[wid], *P = sp[wid];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        K[lane + 64 * z] = wk[j * 512 + lane + 64 * z];
        P[lane + 64 * z] = wp[j * 512 + lane + 64 * z];
    }
    int bx, by, bz;
    unpack_key(keys[j], bx, by, bz);
    int64_t nb = -1;  // lane d < 6 holds the neighbour in direction d
    if (lane < 6) {
        int c[3] = {bx, by, bz};
        c[lane >> 1] += (lane & 1) ? 1 : -1;
        nb = hash_find(tkeys, tvals, tmask, pack_key(c[0], c[1], c[2]));
    }
    wave_sync();
    // faces -x, +x, -y, +y, -z, +z in turn; lane = (u1, u2) on the face
    for (int d = 0; d < 6; ++d) {
        const int64_t n = __shfl(nb, d, 64);
        if (n >= 0) {  // uniform across the wave
            const int a = d >> 1, side = (d & 1) ? 7 : 0;
            const int u1 = lane & 7, u2 = lane >> 3;
            int c[3];
            c[a] = side;
            c[a == 0 ? 1 : 0] = u1;
            c[a == 2 ? 1 : 2] = u2;
            const int lv = lin3(c[0], c[1], c[2]);
            c[a] = 7 - side;
            const int lu = lin3(c[0], c[1], c[2]);
            const int e = (d & 1) ? 1 : -1;
            int32_t kv = K[lv], pv = P[lv];
            wf_offer(kv, pv, wk[n * 512 + lu], wp[n * 512 + lu], a == 0 ? e : 0, a == 1 ? e : 0, a == 2 ? e : 0, R2);
            K[lv] = kv;
            P[lv] = pv;
        }
        wave_sync();
    }
    // sweeps: one lane per line along axis a
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int u1 = lane & 7, u2 = lane >> 3;
        int c[3];
        c[a == 0 ? 1 : 0] = u1;
        c[a == 2 ? 1 : 2] = u2;
        for (int x = 1; x < 8; ++x) {
            c[a] = x;
            const int lv = lin3(c[0], c[1], c[2]);
            c[a] = x - 1;
            const int lu = lin3(c[0], c[1], c[2]);
            int32_t kv = K[lv], pv = P[lv];
            wf_offer(kv, pv, K[lu], P[lu], a == 0 ? -1 : 0, a == 1 ? -1 : 0, a == 2 ? -1 : 0, R2);
            K[lv] = kv;
            P[lv] = pv;
        }
        for (int x = 6; x >= 0; --x) {
            c[a] = x;
            const int lv = lin3(c[0], c[1], c[2]);
            c[a] = x + 1;
            const int lu = lin3(c[0], c[1], c[2]);
            int32_t kv = K[lv], pv = P[lv];
            wf_offer(kv, pv, K[lu], P[lu], a == 0 ? 1 : 0, a == 1 ? 1 : 0, a == 2 ? 1 : 0, R2);
            K[lv] = kv;
            P[lv] = pv;
        }
        wave_sync();
    }
    bool ch = false;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int l = lane + 64 * z;
        ch |= K[l] != wk[j * 512 + l] || P[l] != wp[j * 512 + l];
        nk[j * 512 + l] = K[l];
        np[j * 512 + l] = P[l];
    }
    if (__ballot(ch)) {
        if (lane == 0) flag[j] = 1u;
        if (lane < 6 && nb >= 0) flag[nb] = 1u;
    }
}

__global__ __launch_bounds__(256) void k_wf_commit(const int32_t *__restrict__ list, const int32_t *__restrict__ count,
                                                   const int32_t *__restrict__ nk, const int32_t *__restrict__ np,
                                                   int32_t *__restrict__ wk, int32_t *__restrict__ wp)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t t = blockIdx.x * 4 + wid;
    if (t >= *count) return;
    const int64_t j = list[t];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        wk[j * 512 + lane + 64 * z] = nk[j * 512 + lane + 64 * z];
        wp[j * 512 + lane + 64 * z] = np[j * 512 + lane + 64 * z];
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_wf_phi(SubmapMeta *__restrict__ meta, const S *__restrict__ D,
                                                const S *__restrict__ W, const int32_t *__restrict__ wk, float vs,
                                                float tau, float dmax, float *__restrict__ phi,
                                                int64_t *__restrict__ wn)
{
    const int64_t j = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n = meta->n_blocks;
    if (j == 0 && lane == 0) *wn = n;
    if (j >= n) return;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int64_t o = j * 512 + lane + 64 * z;
        const float Dv = ldw(D + o), Wv = ldw(W + o);
        const int32_t k = wk[o];
        float out;
        if (!(Wv > 0.0f)) out = __builtin_nanf("");
        else if (fabsf(Dv) < tau) out = Dv;
        else {
            const float sg = Dv > 0.0f ? 1.0f : -1.0f;
            out = k == kWfInf ? sg * dmax : sg * fminf(dmax, vs * sqrtf((float)k));
        }
        phi[o] = out;
    }
}

__global__ void k_wf_zero(int64_t *p) { *p = 0; }

}  // namespace

int wavefront_reset(covox_ctx *ctx, covox_submap *s)
{
    if (!s->wf_wn) return COVOX_OK;
    hipLaunchKernelGGL(k_wf_zero, dim3(1), dim3(1), 0, ctx->stream, s->wf_wn);
    return hip_check(ctx, hipGetLastError(), "wavefront reset");
}

int update_esdf_wavefront(covox_ctx *ctx, covox_submap *s)
{
    if (ctx->capturing) return fail(ctx, COVOX_EINVAL, "update_esdf: the wavefront ESDF cannot be captured");
    const covox_params &p = ctx->p;
    int rc;
    const int64_t cap = s->cap;
    if (!s->wf_k) {
        if ((rc = hip_check(ctx, hipMalloc((void **)&s->wf_k, sizeof(int32_t) * 512 * cap), "wavefront state")) ||
            (rc = hip_check(ctx, hipMalloc((void **)&s->wf_p, sizeof(int32_t) * 512 * cap), "wavefront state")) ||
            (rc = hip_check(ctx, hipMalloc((void **)&s->wf_wn, sizeof(int64_t)), "wavefront state")))
            return rc;
        hipLaunchKernelGGL(k_wf_zero, dim3(1), dim3(1), 0, ctx->stream, s->wf_wn);
    }
    if ((rc = ensure_buffer(ctx, (void **)&ctx->wf_nk, &ctx->wf_nk_cap, 512 * cap, sizeof(int32_t), "wavefront")) ||
        (rc = ensure_buffer(ctx, (void **)&ctx->wf_np, &ctx->wf_np_cap, 512 * cap, sizeof(int32_t), "wavefront")) ||
        (rc = ensure_buffer(ctx, (void **)&ctx->wf_sites, &ctx->wf_sites_cap, 8 * cap, sizeof(uint64_t), "wavefront")) ||
        (rc = ensure_buffer(ctx, (void **)&ctx->wf_flag, &ctx->wf_flag_cap, cap, sizeof(uint32_t), "wavefront")) ||
        (rc = ensure_buffer(ctx, (void **)&ctx->wf_list, &ctx->wf_list_cap, cap, sizeof(int32_t), "wavefront")) ||
        (rc = ensure_buffer(ctx, (void **)&ctx->wf_cnt, &ctx->wf_cnt_cap, 4, sizeof(int64_t), "wavefront")))
        return rc;
    if (!ctx->wf_pin) {
        if ((rc = hip_check(ctx, hipHostMalloc((void **)&ctx->wf_pin, 2 * sizeof(int64_t), hipHostMallocDefault),
                            "wavefront counter")))
            return rc;
    }
    // the page (dense block index) serves the alignment and the summaries
    if ((rc = build_page(ctx, s))) return rc;
    const int R = (int)std::llround(p.d_max / p.voxel_size);
    const int64_t nbu = std::max<int64_t>(std::min(s->nb_upper, cap), 1);
    const unsigned gw = (unsigned)((nbu + 3) / 4);
    const uint64_t tmask = (uint64_t)s->tcap - 1;
    const float vs = (float)p.voxel_size;
    int32_t *count = (int32_t *)ctx->wf_cnt;
    int64_t *total = ctx->wf_cnt + 1;
    fill_u32(ctx->stream, ctx->wf_flag, 0u, nbu);
    fill_u64(ctx->stream, (uint64_t *)ctx->wf_cnt, 0ull, 2);
    {
        TimedLaunch tl(ctx, COVOX_K_WAVEFRONT);
        if (p.precision == COVOX_FP16)
            hipLaunchKernelGGL(k_wf_sites<__half>, dim3(gw), dim3(256), 0, ctx->stream, s->meta, (const __half *)s->D,
                               (const __half *)s->W, vs, ctx->wf_sites);
        else
            hipLaunchKernelGGL(k_wf_sites<float>, dim3(gw), dim3(256), 0, ctx->stream, s->meta, (const float *)s->D,
                               (const float *)s->W, vs, ctx->wf_sites);
        hipLaunchKernelGGL(k_wf_seed, dim3(gw), dim3(256), 0, ctx->stream, s->meta, s->wf_wn, s->keys, s->tkeys,
                           s->tvals, tmask, ctx->wf_sites, s->wf_k, s->wf_p, ctx->wf_flag);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "wavefront seed"))) return rc;
    // rounds in groups of four between reads of the queue size
    int64_t rounds = 0;
    for (;;) {
        for (int r = 0; r < 4; ++r) {
            TimedLaunch tl(ctx, COVOX_K_WAVEFRONT);
            hipLaunchKernelGGL(k_wf_list, dim3(1), dim3(1024), 0, ctx->stream, s->meta, ctx->wf_flag, ctx->wf_list,
                               count, total);
            hipLaunchKernelGGL(k_wf_round, dim3(gw), dim3(256), 0, ctx->stream, ctx->wf_list, count, s->keys,
                               s->tkeys, s->tvals, tmask, s->wf_k, s->wf_p, ctx->wf_nk, ctx->wf_np, ctx->wf_flag,
                               R * R);
            hipLaunchKernelGGL(k_wf_commit, dim3(gw), dim3(256), 0, ctx->stream, ctx->wf_list, count, ctx->wf_nk,
                               ctx->wf_np, s->wf_k, s->wf_p);
            ++rounds;
        }
        if ((rc = hip_check(ctx, hipGetLastError(), "wavefront round"))) return rc;
        // the queue size of the last list: zero means the last round did nothing
        if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->wf_pin, ctx->wf_cnt, 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                                                ctx->stream), "wavefront count")) ||
            (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "wavefront sync")))
            return rc;
        if ((int32_t)(ctx->wf_pin[0] & 0xFFFFFFFF) == 0) break;
        if (rounds > 4 * (cap + 8)) return fail(ctx, COVOX_EHIP, "update_esdf: the wavefront did not settle");
    }
    ctx->wf_last_block_rounds = ctx->wf_pin[1];
    {
        TimedLaunch tl(ctx, COVOX_K_WAVEFRONT);
        const float tau = (float)band_limit(p), dmax = (float)p.d_max;
        if (p.precision == COVOX_FP16)
            hipLaunchKernelGGL(k_wf_phi<__half>, dim3(gw), dim3(256), 0, ctx->stream, s->meta, (const __half *)s->D,
                               (const __half *)s->W, s->wf_k, vs, tau, dmax, s->phi, s->wf_wn);
        else
            hipLaunchKernelGGL(k_wf_phi<float>, dim3(gw), dim3(256), 0, ctx->stream, s->meta, (const float *)s->D,
                               (const float *)s->W, s->wf_k, vs, tau, dmax, s->phi, s->wf_wn);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "wavefront phi"))) return rc;
    s->esdf_version = s->version;
    s->esdf_exact = false;  // phi is the wavefront's, not the exact transform
    return COVOX_OK;
}

}  // namespace covox
