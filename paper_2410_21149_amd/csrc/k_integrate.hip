// Projective TSDF integration (paper Sec. III-C projection mapping; the
// count / allocate / update phases of Sec. III-D).
//
// One frame is three launches on the context stream:
//   k_probe      one wave64 per block of the frustum's block box: the 512
//                voxels are tested for validity (lane = (x, y), z in a loop),
//                a ballot gives "any valid", lane 0 looks the key up in the
//                hash table (existing buffer index, or NEW);
//   k_scan       one 1024-lane workgroup compacts the probe results in box
//                order -- which is ascending packed-key order -- so new
//                blocks receive n_blocks + rank deterministically; it checks
//                capacity before anything is committed;
//   k_integrate  one wave64 per touched block: activates new blocks (key
//                store + hash insert, zero-initialised voxels) and applies
//                the running-average update to every valid voxel.
// Parity-relevant arithmetic is binary32 in a fixed operation order (the
// library is built with -ffp-contract=off; division is correctly rounded).
#include "covox_impl.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace covox {

namespace {

constexpr uint32_t kNew = 0xFFFFFFFFu;

template <typename S> __device__ __forceinline__ float ld(const S *p);
template <> __device__ __forceinline__ float ld<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ld<__half>(const __half *p) { return __half2float(*p); }
template <typename S> __device__ __forceinline__ void st(S *p, float v);
template <> __device__ __forceinline__ void st<float>(float *p, float v) { *p = v; }
template <> __device__ __forceinline__ void st<__half>(__half *p, float v) { *p = __float2half_rn(v); }

// Validity of the 8 voxels (ix, iy, iz0 + z), z = 0..7, of one lane under
// the frame's projection: the voxel centre lies in front of the camera, its
// nearest pixel is inside the image, the pixel's depth d is in (0, max
// range], and the signed distance sdf = d - (voxel depth) is at least -tau.
// Sets sdf and the observation weight w (1, or 1 / d^2) of each valid voxel
// and returns the mask of valid voxels.  The steps run in three passes (the
// pixel of every voxel, the 8 depth reads, the tests) so that the reads are
// in flight together; the arithmetic of each voxel is unchanged.
__device__ __forceinline__ uint32_t proj_column(const FrameArgs &f, float vs, float tau, float maxr, int ix, int iy,
                                                int iz0, float sdf[8], float w[8])
{
    const float cx = ((float)ix + 0.5f) * vs;
    const float cy = ((float)iy + 0.5f) * vs;
    float pzv[8];
    int64_t pix[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const float cz = ((float)(iz0 + z) + 0.5f) * vs;
        const float px = ((f.R[0] * cx + f.R[1] * cy) + f.R[2] * cz) + f.t[0];
        const float py = ((f.R[3] * cx + f.R[4] * cy) + f.R[5] * cz) + f.t[1];
        const float pz = ((f.R[6] * cx + f.R[7] * cy) + f.R[8] * cz) + f.t[2];
        pzv[z] = pz;
        pix[z] = -1;
        if (pz > 0.0f) {
            const float u = ((f.K[0] * px) / pz) + f.K[2];
            const float v = ((f.K[1] * py) / pz) + f.K[3];
            const float uf = floorf(u + 0.5f);
            const float vf = floorf(v + 0.5f);
            if (uf >= 0.0f && uf < (float)f.W && vf >= 0.0f && vf < (float)f.H)
                pix[z] = (int64_t)(int)vf * f.W + (int)uf;
        }
    }
    float d[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) d[z] = f.depth[pix[z] >= 0 ? pix[z] : 0];  // pixel 0 stands in, unused
    uint32_t okm = 0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        sdf[z] = 0.0f;
        w[z] = 0.0f;
        if (pix[z] < 0 || !(d[z] > 0.0f && d[z] <= maxr)) continue;
        sdf[z] = d[z] - pzv[z];
        w[z] = f.weight_mode == COVOX_WEIGHT_INV_DEPTH2 ? 1.0f / (d[z] * d[z]) : 1.0f;
        okm |= (uint32_t)(sdf[z] >= -tau) << z;
    }
    return okm;
}

// The nearest pixel of the voxel centre (cx, cy, cz) and its camera depth
// pz, by the arithmetic of proj_column (kept written out there, where the
// compiler schedules the eight voxels of a lane together); -1 when the
// centre is behind the camera or projects outside the image.
__device__ __forceinline__ int64_t proj_pixel(const FrameArgs &f, float cx, float cy, float cz, float &pz)
{
    const float px = ((f.R[0] * cx + f.R[1] * cy) + f.R[2] * cz) + f.t[0];
    const float py = ((f.R[3] * cx + f.R[4] * cy) + f.R[5] * cz) + f.t[1];
    pz = ((f.R[6] * cx + f.R[7] * cy) + f.R[8] * cz) + f.t[2];
    if (pz > 0.0f) {
        const float u = ((f.K[0] * px) / pz) + f.K[2];
        const float v = ((f.K[1] * py) / pz) + f.K[3];
        const float uf = floorf(u + 0.5f);
        const float vf = floorf(v + 0.5f);
        if (uf >= 0.0f && uf < (float)f.W && vf >= 0.0f && vf < (float)f.H) return (int64_t)(int)vf * f.W + (int)uf;
    }
    return -1;
}

// Whether some voxel (ix, iy, iz0 + z), Z0 <= z < Z1, of the lane passes the
// validity test of proj_column (same arithmetic; the weights are not needed).
template <int Z0, int Z1>
__device__ __forceinline__ bool proj_any(const FrameArgs &f, float vs, float tau, float maxr, int ix, int iy, int iz0)
{
    const float cx = ((float)ix + 0.5f) * vs;
    const float cy = ((float)iy + 0.5f) * vs;
    float pzv[Z1 - Z0];
    int64_t pix[Z1 - Z0];
#pragma unroll
    for (int z = Z0; z < Z1; ++z) pix[z - Z0] = proj_pixel(f, cx, cy, ((float)(iz0 + z) + 0.5f) * vs, pzv[z - Z0]);
    float d[Z1 - Z0];
#pragma unroll
    for (int k = 0; k < Z1 - Z0; ++k) d[k] = f.depth[pix[k] >= 0 ? pix[k] : 0];  // pixel 0 stands in, unused
    bool any = false;
#pragma unroll
    for (int k = 0; k < Z1 - Z0; ++k) any |= pix[k] >= 0 && d[k] > 0.0f && d[k] <= maxr && d[k] - pzv[k] >= -tau;
    return any;
}

// False only if no voxel centre of block (bx, by, bz) can pass the validity
// test in this frame: the sphere holding the centres lies behind the
// camera, beyond the far limit, or outside a side plane of the image.
__device__ __forceinline__ bool block_may_be_visible(const FrameArgs &f, float vs, int bx, int by, int bz)
{
    const float cx = (float)(8 * bx + 4) * vs, cy = (float)(8 * by + 4) * vs, cz = (float)(8 * bz + 4) * vs;
    const float px = ((f.R[0] * cx + f.R[1] * cy) + f.R[2] * cz) + f.t[0];
    const float py = ((f.R[3] * cx + f.R[4] * cy) + f.R[5] * cz) + f.t[1];
    const float pz = ((f.R[6] * cx + f.R[7] * cy) + f.R[8] * cz) + f.t[2];
    const float r = f.cull_r;
    if (pz < -r || pz > f.zfar + r) return false;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (f.plane[k][0] * px + f.plane[k][1] * py + f.plane[k][2] * pz < -r) return false;
    return true;
}

__device__ __forceinline__ void box_block(const FrameArgs &f, int64_t j, int &bx, int &by, int &bz)
{
    const int64_t nz = f.bdim[2], ny = f.bdim[1];
    bz = f.blo[2] + (int)(j % nz);
    by = f.blo[1] + (int)((j / nz) % ny);
    bx = f.blo[0] + (int)(j / (nz * ny));
}

// The running-average update of one voxel column (8 z values of a lane) of
// an allocated block; returns the number of updated voxels of the wave.
template <typename S>
__device__ __forceinline__ int update_column(S *Db, S *Wb, const float sdf[8], const float wt[8], uint32_t okm, float tau,
                                             bool is_new)
{
    // Every read is issued in straight-line code, so that the eight are in
    // flight together (a conditional read would make the compiler wait for
    // each one in turn), but a voxel that is not updated reads its lane's
    // z = 0 voxel instead: rows of the block that no lane updates are not
    // fetched.  Only updated voxels are written, and every voxel of a new
    // block (zero where not updated).
    float Dp[8], Wp[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const int o = ((okm >> z) & 1u) ? 64 * z : 0;
        Dp[z] = ld(Db + o);
        Wp[z] = ld(Wb + o);
    }
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        Dp[z] = is_new ? 0.0f : Dp[z];
        Wp[z] = is_new ? 0.0f : Wp[z];
    }
    int n_ok = 0;
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        const bool ok = (okm >> z) & 1u;
        n_ok += __popcll(__ballot(ok));
        const float tr = fminf(sdf[z], tau);
        const float Wn = Wp[z] + wt[z];
        const float Dn = ((Dp[z] * Wp[z]) + (tr * wt[z])) / Wn;
        Dp[z] = ok ? Dn : Dp[z];
        Wp[z] = ok ? Wn : Wp[z];
    }
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        if (((okm >> z) & 1u) || is_new) {
            st(Db + 64 * z, Dp[z]);
            st(Wb + 64 * z, Wp[z]);
        }
    }
    return n_ok;
}

// Work item of workgroup w in a grid of n_wg = 8 C workgroups: with XCD
// order, item (w mod 8) C + floor(w / 8), so that the workgroups the
// dispatcher deals to one XCD cover one contiguous eighth of the items;
// otherwise w.
__device__ __forceinline__ int64_t work_item(int64_t w, int64_t n_wg, bool xcd)
{
    return xcd ? (w & 7) * (n_wg >> 3) + (w >> 3) : w;
}

// FUSED: blocks that already exist are updated here (their buffer index is
// known), so only new blocks are left to k_integrate.  Used only when the
// host bound proves that this frame cannot overflow the pool or the table,
// so that no capacity failure can follow a partial update.
template <typename S, bool FUSED>
__global__ __launch_bounds__(256) void k_probe(FrameArgs f, float vs, float tau, float maxr,
                                               const uint64_t *__restrict__ tkeys,
                                               const uint32_t *__restrict__ tvals, uint64_t tmask,
                                               uint32_t *__restrict__ cand, int64_t n_box, S *D, S *W,
                                               SubmapMeta *meta, uint8_t *__restrict__ dirty, int xcd)
{
    const int64_t j = work_item(blockIdx.x, gridDim.x, xcd) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= n_box) return;  // uniform across the wave
    int bx, by, bz;
    box_block(f, j, bx, by, bz);
    if (!block_may_be_visible(f, vs, bx, by, bz)) {  // uniform across the wave
        if (lane == 0) cand[j] = 0;
        return;
    }
    // the home slot of the block's key is read before the validity test, so
    // that its latency overlaps the depth reads
    // (every lane reads the same slot: one request, no branch)
    const uint64_t key = pack_key(bx, by, bz);
    const HashProbe hp = hash_first(tkeys, tvals, tmask, key);
    const int ix = 8 * bx + (lane & 7);
    const int iy = 8 * by + (lane >> 3);
    float sdf[8], wt[8];
    const uint32_t okm = proj_column(f, vs, tau, maxr, ix, iy, 8 * bz, sdf, wt);
    const uint64_t m = __ballot(okm != 0);
    uint32_t out = 0;
    if (m) {
        int64_t idx = -1;
        if (lane == 0) idx = hash_resolve(hp, tkeys, tvals, tmask, key);
        idx = __shfl(idx, 0, 64);
        out = idx >= 0 ? (uint32_t)idx + 1u : kNew;
        if (FUSED && idx >= 0) {
            const int n_ok = update_column(D + idx * 512 + lane, W + idx * 512 + lane, sdf, wt, okm, tau, false);
            if (lane == 0) {
                atomicAdd(&meta->n_updates, (unsigned long long)n_ok);
                dirty[idx] = 1;
            }
        }
    }
    if (lane == 0) cand[j] = out;
}

// Exclusive scan of one int64 per thread over a 1024-thread workgroup.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *lds, int64_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int64_t w = lane < nw ? lds[lane] : 0;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int64_t y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < nw) lds[lane] = w;  // inclusive wave totals
    }
    __syncthreads();
    const int64_t before = (wid > 0 ? lds[wid - 1] : 0) + x - v;
    *total = lds[nw - 1];
    __syncthreads();
    return before;
}

// Block count and call sequence for the host's bound (pinned host memory).
__device__ __forceinline__ void publish_count(uint64_t *host_nb, uint64_t seq, int64_t n_blocks)
{
    *(volatile uint64_t *)host_nb = ((seq & 0xFFFFFFull) << 40) | (uint64_t)n_blocks;
}

__global__ __launch_bounds__(1024) void k_scan(const uint32_t *__restrict__ cand, int64_t n_box, FrameArgs f,
                                               SubmapMeta *meta, int64_t cap, int64_t table_limit,
                                               uint64_t *__restrict__ t_key, uint32_t *__restrict__ t_idx,
                                               uint64_t *__restrict__ t_new, uint64_t *host_nb, uint64_t seq)
{
    __shared__ int64_t lds[16];
    __shared__ int32_t red[6][16];
    const int tid = threadIdx.x;
    const int64_t C = (n_box + blockDim.x - 1) / blockDim.x;
    const int64_t beg = std::min<int64_t>((int64_t)tid * C, n_box);
    const int64_t end = std::min<int64_t>(beg + C, n_box);
    // the first kCache entries of the thread's range stay in registers for
    // the second pass; their reads are issued together
    constexpr int kCache = 8;
    uint32_t cv[kCache];
#pragma unroll
    for (int q = 0; q < kCache; ++q) cv[q] = beg + q < end ? cand[beg + q] : 0u;
    int64_t nt = 0, nn = 0;
#pragma unroll
    for (int q = 0; q < kCache; ++q) {
        nt += cv[q] != 0;
        nn += cv[q] == kNew;
    }
    for (int64_t j = beg + kCache; j < end; ++j) {
        const uint32_t v = cand[j];
        nt += v != 0;
        nn += v == kNew;
    }
    // one scan of both counts (touched in the low, new in the high 32 bits:
    // each is at most n_box < 2^32, so the fields never carry into each other)
    int64_t tot;
    const int64_t off = block_exclusive_scan(nt | (nn << 32), lds, &tot);
    int64_t off_t = off & 0xFFFFFFFFll, off_n = off >> 32;
    const int64_t tot_t = tot & 0xFFFFFFFFll, tot_n = tot >> 32;
    const int64_t n0 = meta->n_blocks;
    __syncthreads();  // every thread has read n_blocks before it changes
    const bool pool_full = n0 + tot_n > cap;
    const bool table_full = n0 + tot_n > table_limit;
    if (pool_full || table_full) {
        if (tid == 0) {
            meta->status = pool_full ? COVOX_EPOOL_FULL : COVOX_ETABLE_FULL;
            meta->n_new = 0;
            meta->n_touched = 0;
            publish_count(host_nb, seq, n0);
        }
        return;
    }
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    auto emit = [&](int64_t j, uint32_t v) {
        if (!v) return;
        int bx, by, bz;
        box_block(f, j, bx, by, bz);
        uint32_t idx;
        if (v == kNew) {
            t_new[off_n] = pack_key(bx, by, bz);  // the new blocks alone, in index order
            idx = (uint32_t)(n0 + off_n++) | 0x80000000u;
            lo[0] = min(lo[0], bx); lo[1] = min(lo[1], by); lo[2] = min(lo[2], bz);
            hi[0] = max(hi[0], bx); hi[1] = max(hi[1], by); hi[2] = max(hi[2], bz);
        } else {
            idx = v - 1u;
        }
        t_key[off_t] = pack_key(bx, by, bz);
        t_idx[off_t] = idx;
        ++off_t;
    };
#pragma unroll
    for (int q = 0; q < kCache; ++q)
        if (beg + q < end) emit(beg + q, cv[q]);
    for (int64_t j = beg + kCache; j < end; ++j) emit(j, cand[j]);
    // box of the new blocks: wave reduction, then across waves
    const int lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        for (int o = 32; o > 0; o >>= 1) {
            lo[a] = min(lo[a], __shfl_xor(lo[a], o, 64));
            hi[a] = max(hi[a], __shfl_xor(hi[a], o, 64));
        }
        if (lane == 0) { red[a][wid] = lo[a]; red[3 + a][wid] = hi[a]; }
    }
    __syncthreads();
    if (tid == 0) {
        int32_t L[3], Hh[3];
        for (int a = 0; a < 3; ++a) {
            L[a] = INT32_MAX; Hh[a] = INT32_MIN;
            for (int w = 0; w < nw; ++w) { L[a] = min(L[a], red[a][w]); Hh[a] = max(Hh[a], red[3 + a][w]); }
        }
        if (tot_n > 0) {
            for (int a = 0; a < 3; ++a) {
                if (n0 == 0) { meta->bmin[a] = L[a]; meta->bmax[a] = Hh[a]; }
                else { meta->bmin[a] = min(meta->bmin[a], L[a]); meta->bmax[a] = max(meta->bmax[a], Hh[a]); }
            }
        }
        meta->n_blocks = n0 + tot_n;
        meta->n_new = (int32_t)tot_n;
        meta->n_touched = (int32_t)tot_t;
        publish_count(host_nb, seq, n0 + tot_n);
    }
}

// NEW_ONLY: the probe has already updated the existing blocks (fused path),
// and the waves walk the scan's list of the new blocks alone (t_new; block
// index n_blocks - n_new + position), so that a small grid suffices.
template <typename S, bool NEW_ONLY>
__global__ __launch_bounds__(256) void k_integrate(FrameArgs f, float vs, float tau, float maxr,
                                                   SubmapMeta *__restrict__ meta,
                                                   const uint64_t *__restrict__ t_key,
                                                   const uint32_t *__restrict__ t_idx,
                                                   const uint64_t *__restrict__ t_new, uint64_t *keys, S *D, S *W,
                                                   uint64_t *tkeys, uint32_t *tvals, uint64_t tmask,
                                                   uint8_t *__restrict__ dirty)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t n_t = NEW_ONLY ? (int64_t)meta->n_new : (int64_t)meta->n_touched;
    const int64_t n0 = NEW_ONLY ? meta->n_blocks - n_t : 0;
    for (int64_t t = wave; t < n_t; t += nwaves) {
        const uint32_t v = NEW_ONLY ? 0x80000000u | (uint32_t)(n0 + t) : t_idx[t];
        const bool is_new = (v >> 31) != 0;
        const uint64_t key = NEW_ONLY ? t_new[t] : t_key[t];
        const int64_t idx = v & 0x7FFFFFFFu;
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        if (is_new && lane == 0) {
            keys[idx] = key;
            hash_insert(tkeys, tvals, tmask, key, (uint32_t)idx);
        }
        const int ix = 8 * bx + (lane & 7);
        const int iy = 8 * by + (lane >> 3);
        float sdf[8], wt[8];
        const uint32_t okm = proj_column(f, vs, tau, maxr, ix, iy, 8 * bz, sdf, wt);
        const int n_ok = update_column(D + idx * 512 + lane, W + idx * 512 + lane, sdf, wt, okm, tau, is_new);
        if (lane == 0) {
            atomicAdd(&meta->n_updates, (unsigned long long)n_ok);
            dirty[idx] = 1;
        }
    }
}

// ------------------------------------------------------- frame batches
// A batch of F frames takes three launches.  k_probe_batch tests every
// frame's box blocks against the table as it was before the batch.
// k_scan_batch walks the frames in order in one workgroup: a candidate
// marked new that an earlier frame of the batch has created becomes
// existing; the remaining new blocks of the frame get n_blocks + rank in
// key order (so indices follow (first frame, key), as with per-frame calls)
// and are activated at once; every block touched by some frame is listed
// once.  k_integrate_batch gives each listed block one wave that applies the
// frames in order in registers and writes D and W once.

__global__ __launch_bounds__(256) void k_probe_batch(const FrameArgs *__restrict__ frames, float vs, float tau,
                                                     float maxr, const uint64_t *__restrict__ tkeys,
                                                     const uint32_t *__restrict__ tvals, uint64_t tmask,
                                                     uint32_t *__restrict__ cand, int64_t stride, int F, int xcd)
{
    // work items: (frame, group of 4 box blocks), frame-major, in a grid
    // stride; with XCD order the workgroups on XCD r (w mod 8 = r) stride
    // over the r-th eighth of the items
    const int64_t per_frame = (stride + 3) / 4, n_items = per_frame * F;
    int64_t first, end, step;
    if (xcd) {
        const int64_t per = (n_items + 7) / 8, r = blockIdx.x & 7;
        first = r * per + (blockIdx.x >> 3);
        end = min(n_items, (r + 1) * per);
        step = gridDim.x >> 3;
    } else {
        first = blockIdx.x;
        end = n_items;
        step = gridDim.x;
    }
    const int lane = threadIdx.x & 63;
    for (int64_t item = first; item < end; item += step) {
        const int fi = (int)(item / per_frame);
        const FrameArgs f = frames[fi];
        const int64_t n_box = (int64_t)f.bdim[0] * f.bdim[1] * f.bdim[2];
        // the wave index is read through the scalar unit, so that the box
        // coordinates of the wave's block are scalar arithmetic
        const int64_t j = (item % per_frame) * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (j >= n_box) continue;  // uniform across the wave
        int bx, by, bz;
        box_block(f, j, bx, by, bz);
        uint32_t out = 0;
        if (block_may_be_visible(f, vs, bx, by, bz)) {  // uniform across the wave
            const int ix = 8 * bx + (lane & 7);
            const int iy = 8 * by + (lane >> 3);
            // only whether some voxel is valid matters here: the bottom row
            // of 64 voxels first, which decides a block of free space or at
            // the surface; the other seven rows only when it has none
            uint64_t m = __ballot(proj_any<0, 1>(f, vs, tau, maxr, ix, iy, 8 * bz));
            if (m == 0) m = __ballot(proj_any<1, 8>(f, vs, tau, maxr, ix, iy, 8 * bz));
            if (lane == 0 && m) {
                const int64_t idx = hash_find(tkeys, tvals, tmask, pack_key(bx, by, bz));
                out = idx >= 0 ? (uint32_t)idx + 1u : kNew;
            }
        }
        if (lane == 0) cand[(int64_t)fi * stride + j] = out;
    }
}

// The allocation of a batch in four parallel steps, equal to per-frame
// calls: a block is new in the first frame of the batch that touches it and
// not before the batch; new blocks take n_blocks + rank in (first frame, key)
// order; the frames up to the first one that would overflow the pool or the
// table are committed, the rest dropped.
//   k_batch_first     first frame of every new key (temporary table, min)
//   k_batch_rank      one workgroup per frame: the frame's first-time new
//                     blocks ranked in box order (= key order)
//   k_batch_commit    offsets of the frames, capacity check, counts
//   k_batch_activate  keys, table entries and the list of distinct touched
//                     blocks of the committed frames

constexpr uint32_t kFirstNew = 0x80000000u;  // candidate: first-time new, low bits = rank in its frame

__global__ __launch_bounds__(256) void k_batch_first(const FrameArgs *__restrict__ frames,
                                                     const uint32_t *__restrict__ cand, int64_t stride,
                                                     uint64_t *fkeys, uint32_t *ffirst, uint64_t fmask)
{
    const int fi = blockIdx.y;
    const FrameArgs &f = frames[fi];
    const int64_t n_box = (int64_t)f.bdim[0] * f.bdim[1] * f.bdim[2];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_box; j += (int64_t)gridDim.x * blockDim.x) {
        if (cand[(int64_t)fi * stride + j] != kNew) continue;
        int bx, by, bz;
        box_block(f, j, bx, by, bz);
        const uint64_t key = pack_key(bx, by, bz);
        // the table holds at least twice as many slots as candidates
        for (uint64_t h = mix64(key) & fmask;; h = (h + 1) & fmask) {
            const unsigned long long prev =
                atomicCAS((unsigned long long *)&fkeys[h], (unsigned long long)kEmpty, (unsigned long long)key);
            if (prev == kEmpty || prev == key) {
                atomicMin(&ffirst[h], (uint32_t)fi);
                break;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_batch_rank(const FrameArgs *__restrict__ frames, uint32_t *cand,
                                                     int64_t stride, const uint64_t *__restrict__ fkeys,
                                                     const uint32_t *__restrict__ ffirst, uint64_t fmask,
                                                     int64_t *fcount)
{
    __shared__ int64_t lds[16];
    const int fi = blockIdx.x;
    const FrameArgs &f = frames[fi];
    const int64_t n_box = (int64_t)f.bdim[0] * f.bdim[1] * f.bdim[2];
    uint32_t *cf = cand + (int64_t)fi * stride;
    const int tid = threadIdx.x;
    const int64_t C = (n_box + blockDim.x - 1) / blockDim.x;
    const int64_t beg = std::min<int64_t>((int64_t)tid * C, n_box);
    const int64_t end = std::min<int64_t>(beg + C, n_box);
    int64_t nn = 0;
    for (int64_t j = beg; j < end; ++j) {
        if (cf[j] != kNew) continue;
        int bx, by, bz;
        box_block(f, j, bx, by, bz);
        const uint64_t key = pack_key(bx, by, bz);
        uint64_t h = mix64(key) & fmask;
        while (fkeys[h] != key) h = (h + 1) & fmask;  // present: inserted by this candidate
        if (ffirst[h] == (uint32_t)fi) ++nn;
        else cf[j] = 0;  // created by an earlier frame of the batch
    }
    int64_t tot;
    int64_t off = block_exclusive_scan(nn, lds, &tot);
    for (int64_t j = beg; j < end; ++j)
        if (cf[j] == kNew) cf[j] = kFirstNew | (uint32_t)(off++);
    if (tid == 0) fcount[fi] = tot;
}

// One wave: F <= 64 frames.
__global__ __launch_bounds__(64) void k_batch_commit(int F, const int64_t *__restrict__ fcount, int64_t *foff,
                                                     SubmapMeta *meta, int64_t cap, int64_t table_limit,
                                                     uint64_t *host_nb, uint64_t seq)
{
    const int lane = threadIdx.x;
    const int64_t n0 = meta->n_blocks;
    const int64_t c = lane < F ? fcount[lane] : 0;
    int64_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    const bool over = lane < F && (n0 + incl > cap || n0 + incl > table_limit);
    const uint64_t m = __ballot(over);
    const int committed = m ? __ffsll((long long)m) - 1 : F;
    if (lane < F) foff[lane] = n0 + incl - c;
    // (all lanes take part in the shuffles)
    const int src = committed < F ? committed : 0;
    const int64_t before_fail = __shfl(incl - c, src, 64);
    const int64_t at_fail = __shfl(incl, src, 64);
    const int64_t total_all = __shfl(incl, 63, 64);
    if (lane == 0) {
        const int64_t n_new = committed < F ? before_fail : total_all;
        if (committed < F) meta->status = n0 + at_fail > cap ? COVOX_EPOOL_FULL : COVOX_ETABLE_FULL;
        if (n0 == 0 && n_new > 0)
            for (int a = 0; a < 3; ++a) { meta->bmin[a] = INT32_MAX; meta->bmax[a] = INT32_MIN; }
        meta->n_blocks = n0 + n_new;
        meta->n_new = (int32_t)n_new;
        meta->n_touched = 0;
        meta->batch_n0 = n0;
        meta->batch_frames = committed;
        publish_count(host_nb, seq, n0 + n_new);
    }
}

__global__ __launch_bounds__(256) void k_batch_activate(const FrameArgs *__restrict__ frames,
                                                        const uint32_t *__restrict__ cand, int64_t stride,
                                                        const int64_t *__restrict__ foff, SubmapMeta *meta,
                                                        uint64_t *keys, uint64_t *tkeys, uint32_t *tvals,
                                                        uint64_t tmask, uint32_t *stamp, uint32_t batch_id,
                                                        uint32_t *list)
{
    const int fi = blockIdx.y;
    if (fi >= meta->batch_frames) return;  // uniform: frame not committed
    const FrameArgs &f = frames[fi];
    const int64_t n_box = (int64_t)f.bdim[0] * f.bdim[1] * f.bdim[2];
    const int64_t base = foff[fi];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_box; j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = cand[(int64_t)fi * stride + j];
        if (!v) continue;
        uint32_t idx;
        bool listed;
        if (v & kFirstNew) {
            int bx, by, bz;
            box_block(f, j, bx, by, bz);
            const uint64_t key = pack_key(bx, by, bz);
            idx = (uint32_t)(base + (v & ~kFirstNew));
            keys[idx] = key;
            hash_insert(tkeys, tvals, tmask, key, idx);
            stamp[idx] = batch_id;
            listed = true;
            atomicMin(&meta->bmin[0], bx); atomicMin(&meta->bmin[1], by); atomicMin(&meta->bmin[2], bz);
            atomicMax(&meta->bmax[0], bx); atomicMax(&meta->bmax[1], by); atomicMax(&meta->bmax[2], bz);
        } else {
            idx = v - 1u;  // existed before the batch
            listed = atomicExch(&stamp[idx], batch_id) != batch_id;
        }
        if (listed) list[atomicAdd(&meta->n_touched, 1)] = idx;
    }
}

// Storage rounding of a value kept in registers across frames, so that the
// batch matches per-frame calls that store after every frame.
template <typename S> __device__ __forceinline__ float stored(float v);
template <> __device__ __forceinline__ float stored<float>(float v) { return v; }
template <> __device__ __forceinline__ float stored<__half>(float v) { return __half2float(__float2half_rn(v)); }

template <typename S>
__global__ __launch_bounds__(256) void k_integrate_batch(const FrameArgs *__restrict__ frames,
                                                         SubmapMeta *__restrict__ meta,
                                                         const uint32_t *__restrict__ list,
                                                         const uint64_t *__restrict__ keys, S *D, S *W, float vs,
                                                         float tau, float maxr, uint8_t *__restrict__ dirty, int xcd)
{
    const int lane = threadIdx.x & 63;
    const int64_t n_t = meta->n_touched, n0 = meta->batch_n0;
    const int F = meta->batch_frames;
    // the listed blocks in a grid stride; with XCD order, the workgroups on
    // XCD r (w mod 8 = r) stride over the r-th eighth of the list
    const int64_t wpg = blockDim.x >> 6;
    int64_t t0, t1, step, first;
    if (xcd) {
        const int r = blockIdx.x & 7;
        t0 = n_t * r / 8;
        t1 = n_t * (r + 1) / 8;
        step = (int64_t)(gridDim.x >> 3) * wpg;
        first = (int64_t)(blockIdx.x >> 3) * wpg + (threadIdx.x >> 6);
    } else {
        t0 = 0;
        t1 = n_t;
        step = (int64_t)gridDim.x * wpg;
        first = (int64_t)blockIdx.x * wpg + (threadIdx.x >> 6);
    }
    for (int64_t t = t0 + first; t < t1; t += step) {
        const int64_t idx = list[t];
        const bool is_new = idx >= n0;
        int bx, by, bz;
        unpack_key(keys[idx], bx, by, bz);
        const int ix = 8 * bx + (lane & 7);
        const int iy = 8 * by + (lane >> 3);
        S *Db = D + idx * 512 + lane;
        S *Wb = W + idx * 512 + lane;
        float dv[8], wv[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            dv[z] = is_new ? 0.0f : ld(Db + 64 * z);
            wv[z] = is_new ? 0.0f : ld(Wb + 64 * z);
        }
        int n_ok = 0;
        for (int fi = 0; fi < F; ++fi) {
            const FrameArgs &f = frames[fi];
            if (bx < f.blo[0] || bx >= f.blo[0] + f.bdim[0] || by < f.blo[1] || by >= f.blo[1] + f.bdim[1] ||
                bz < f.blo[2] || bz >= f.blo[2] + f.bdim[2] || !block_may_be_visible(f, vs, bx, by, bz))
                continue;  // no valid voxel in this frame
            float sdf[8], w[8];
            const uint32_t okm = proj_column(f, vs, tau, maxr, ix, iy, 8 * bz, sdf, w);
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const bool ok = (okm >> z) & 1u;
                n_ok += __popcll(__ballot(ok));
                if (ok) {
                    const float tr = fminf(sdf[z], tau);
                    const float Wn = wv[z] + w[z];
                    const float Dn = ((dv[z] * wv[z]) + (tr * w[z])) / Wn;
                    dv[z] = stored<S>(Dn);
                    wv[z] = stored<S>(Wn);
                }
            }
        }
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            st(Db + 64 * z, dv[z]);
            st(Wb + 64 * z, wv[z]);
        }
        if (lane == 0) {
            atomicAdd(&meta->n_updates, (unsigned long long)n_ok);
            dirty[idx] = 1;
        }
    }
}

// ---------------------------------------------------------------- host

void rigid_inverse(const double *T, double *O)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) O[4 * r + c] = T[4 * c + r];
    for (int r = 0; r < 3; ++r)
        O[4 * r + 3] = -((O[4 * r + 0] * T[3] + O[4 * r + 1] * T[7]) + O[4 * r + 2] * T[11]);
    O[12] = 0; O[13] = 0; O[14] = 0; O[15] = 1;
}

void rigid_mul(const double *A, const double *B, double *O)
{
    double t[16];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            t[4 * r + c] = (A[4 * r + 0] * B[c] + A[4 * r + 1] * B[4 + c]) + A[4 * r + 2] * B[8 + c];
        t[4 * r + 3] = ((A[4 * r + 0] * B[3] + A[4 * r + 1] * B[7]) + A[4 * r + 2] * B[11]) + A[4 * r + 3];
    }
    t[12] = 0; t[13] = 0; t[14] = 0; t[15] = 1;
    for (int k = 0; k < 16; ++k) O[k] = t[k];
}

bool is_rigid(const double *T)
{
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(T[k])) return false;
    if (T[12] != 0 || T[13] != 0 || T[14] != 0 || T[15] != 1) return false;
    double e = 0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + r] * T[4 * k + c];
            e = std::max(e, std::fabs(s - (r == c ? 1.0 : 0.0)));
        }
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    return e <= 1e-6 && det > 0;
}

// Workgroups of the new-block integration after a fused probe: a frame adds a
// few new blocks, except the first ones; the waves walk the list with a
// stride.
constexpr unsigned kNewGrid = 64;

template <typename S>
void launch_frame(covox_ctx *ctx, covox_submap *s, const FrameArgs &f, float vs, float tau, float maxr, uint64_t tmask,
                  int64_t table_limit, int64_t n_box, unsigned grid, bool fused)
{
    S *D = (S *)s->D, *W = (S *)s->W;
    const int xcd = ctx->tune.mapping_xcd_order != 0;
    const unsigned grid8 = (grid + 7) / 8 * 8;  // a multiple of 8 for the XCD order
    {
        TimedLaunch tl(ctx, COVOX_K_PROBE);
        if (fused)
            hipLaunchKernelGGL((k_probe<S, true>), dim3(grid8), dim3(256), 0, ctx->stream, f, vs, tau, maxr, s->tkeys,
                               s->tvals, tmask, ctx->cand, n_box, D, W, s->meta, s->dirty, xcd);
        else
            hipLaunchKernelGGL((k_probe<S, false>), dim3(grid8), dim3(256), 0, ctx->stream, f, vs, tau, maxr, s->tkeys,
                               s->tvals, tmask, ctx->cand, n_box, D, W, s->meta, s->dirty, xcd);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_SCAN);
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, ctx->cand, n_box, f, s->meta, s->cap,
                           table_limit, ctx->t_key, ctx->t_idx, ctx->t_key + n_box, s->pin_nb_dev, s->seq);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_INTEGRATE);
        if (fused)
            hipLaunchKernelGGL((k_integrate<S, true>), dim3(std::min(grid, kNewGrid)), dim3(256), 0, ctx->stream, f, vs,
                               tau, maxr, s->meta, ctx->t_key, ctx->t_idx, ctx->t_key + n_box, s->keys, D, W,
                               s->tkeys, s->tvals, tmask, s->dirty);
        else
            hipLaunchKernelGGL((k_integrate<S, false>), dim3(grid), dim3(256), 0, ctx->stream, f, vs, tau, maxr,
                               s->meta, ctx->t_key, ctx->t_idx, ctx->t_key + n_box, s->keys, D, W, s->tkeys,
                               s->tvals, tmask, s->dirty);
    }
}

}  // namespace

// Tightens the host's upper bound on the block count without stalling: the
// count the scan kernel of call q last published, plus the box sizes of the
// calls enqueued after q.  Then registers the next call with its box size.
void refresh_block_bound(covox_submap *s, int64_t next_box)
{
    const uint64_t v = *s->pin_nb;
    const uint64_t q = v >> 40, cnt = v & ((1ull << 40) - 1);
    const uint64_t behind = (s->seq - q) & 0xFFFFFFull;  // calls enqueued after q
    if (behind < (uint64_t)covox_submap::kSeqRing && behind <= s->seq) {
        int64_t b = (int64_t)cnt;
        for (uint64_t k = s->seq - behind + 1; k <= s->seq; ++k) b += s->box_ring[k % covox_submap::kSeqRing];
        s->nb_upper = std::min(s->nb_upper, b);
    }
    s->seq++;
    s->box_ring[s->seq % covox_submap::kSeqRing] = next_box;
}

// The compaction launch shared by both integrators (one workgroup).
void launch_block_scan(covox_ctx *ctx, covox_submap *s, const FrameArgs &f, int64_t n_box, int64_t table_limit)
{
    TimedLaunch tl(ctx, COVOX_K_SCAN);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, ctx->stream, ctx->cand, n_box, f, s->meta, s->cap,
                       table_limit, ctx->t_key, ctx->t_idx, ctx->t_key + n_box, s->pin_nb_dev, s->seq);
}

// Frame parameters (pose rounded once from binary64) and the block box of
// the frustum.
int prepare_frame(covox_ctx *ctx, const covox_submap *s, const float *depth, int32_t H, int32_t W, const float K[4],
                  const double T_wc[16], FrameArgs &f, int64_t &n_box)
{
    const covox_params &p = ctx->p;
    if (!depth || H <= 0 || W <= 0 || !K || !T_wc) return fail(ctx, COVOX_EINVAL, "integrate: bad argument");
    if (!(K[0] > 0) || !(K[1] > 0) || !std::isfinite(K[2]) || !std::isfinite(K[3]))
        return fail(ctx, COVOX_EINVAL, "integrate: fx and fy must be positive");
    if (!is_rigid(T_wc)) return fail(ctx, COVOX_EINVAL, "integrate: T_world_cam is not a rigid transform");

    // camera <- submap, binary64, rounded once to binary32
    double inv_wc[16], T_cs[16];
    rigid_inverse(T_wc, inv_wc);
    rigid_mul(inv_wc, s->T_ws, T_cs);
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) f.R[3 * r + c] = (float)T_cs[4 * r + c];
        f.t[r] = (float)T_cs[4 * r + 3];
    }
    for (int k = 0; k < 4; ++k) f.K[k] = K[k];
    f.H = H;
    f.W = W;
    f.depth = depth;
    f.weight_mode = p.weight_mode;
    {
        // side planes through the camera centre for u in [-1.5, W + 0.5]
        // and v in [-1.5, H + 0.5] (one pixel beyond the pixel-centre test)
        const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
        const double n[4][3] = {{fx, 0, cx + 1.5}, {-fx, 0, W + 0.5 - cx}, {0, fy, cy + 1.5}, {0, -fy, H + 0.5 - cy}};
        for (int k = 0; k < 4; ++k) {
            const double len = std::sqrt(n[k][0] * n[k][0] + n[k][1] * n[k][1] + n[k][2] * n[k][2]);
            for (int a = 0; a < 3; ++a) f.plane[k][a] = (float)(n[k][a] / len);
        }
        f.zfar = (float)(p.max_range + p.trunc_vox * p.voxel_size);
        f.cull_r = (float)(1.01 * std::sqrt(3.0) * 3.5 * p.voxel_size + 1e-4);
    }

    // Block box containing every voxel centre of the frustum cut at
    // max_range + tau (conservative; validity decides exactly).
    double inv_ws[16], T_sc[16];
    rigid_inverse(s->T_ws, inv_ws);
    rigid_mul(inv_ws, T_wc, T_sc);
    // submap <- camera, rounded once, for raycasting
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) f.Rs[3 * r + c] = (float)T_sc[4 * r + c];
        f.o[r] = (float)T_sc[4 * r + 3];
    }
    f.ray_carve = p.ray_carve;
    const double tau = p.trunc_vox * p.voxel_size;
    const double zf = p.max_range + tau;
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) mn[a] = mx[a] = T_sc[4 * a + 3];
    const double us[2] = {-0.5, W - 0.5}, vv[2] = {-0.5, H - 0.5};
    for (double u : us)
        for (double v : vv) {
            const double pc[3] = {(u - K[2]) / K[0] * zf, (v - K[3]) / K[1] * zf, zf};
            for (int a = 0; a < 3; ++a) {
                const double w = T_sc[4 * a] * pc[0] + T_sc[4 * a + 1] * pc[1] + T_sc[4 * a + 2] * pc[2] + T_sc[4 * a + 3];
                mn[a] = std::min(mn[a], w);
                mx[a] = std::max(mx[a], w);
            }
        }
    n_box = 1;
    for (int a = 0; a < 3; ++a) {
        const int64_t ilo = (int64_t)std::floor(mn[a] / p.voxel_size - 0.5) - 1;
        const int64_t ihi = (int64_t)std::ceil(mx[a] / p.voxel_size - 0.5) + 1;
        const int64_t blo = ilo >= 0 ? ilo / 8 : -((-ilo + 7) / 8);
        const int64_t bhi = ihi >= 0 ? ihi / 8 : -((-ihi + 7) / 8);
        if (blo < -kKeyOff + 1 || bhi > kKeyOff - 2)
            return fail(ctx, COVOX_EINVAL, "integrate: frustum outside the addressable block range");
        f.blo[a] = (int32_t)blo;
        f.bdim[a] = (int32_t)(bhi - blo + 1);
        n_box *= f.bdim[a];
    }
    return COVOX_OK;
}

namespace {

// Batch id reserved for batches captured in a graph.
constexpr uint32_t kCapturedBatch = 0xFFFFFFFFu;

// Uploads the frame parameters of a batch through pinned staging: slot k is
// reused only once its previous upload has completed.
int stage_frames(covox_ctx *ctx, const FrameArgs *fr, int32_t F)
{
    int rc;
    const int slot = ctx->frames_slot;
    ctx->frames_slot ^= 1;
    if (!ctx->frames_pin[slot]) {
        if ((rc = hip_check(ctx, hipHostMalloc((void **)&ctx->frames_pin[slot], sizeof(FrameArgs) * kMaxBatch,
                                               hipHostMallocDefault), "frame staging")))
            return rc;
        if ((rc = hip_check(ctx, hipEventCreateWithFlags(&ctx->frames_ev[slot], hipEventDisableTiming),
                            "frame staging event")))
            return rc;
    } else if ((rc = hip_check(ctx, hipEventSynchronize(ctx->frames_ev[slot]), "frame staging wait"))) {
        return rc;
    }
    ::memcpy(ctx->frames_pin[slot], fr, sizeof(FrameArgs) * F);
    if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->frames_dev, ctx->frames_pin[slot], sizeof(FrameArgs) * F,
                                            hipMemcpyHostToDevice, ctx->stream), "frame batch upload")))
        return rc;
    return hip_check(ctx, hipEventRecord(ctx->frames_ev[slot], ctx->stream), "frame staging record");
}

}  // namespace

// Host bounds after frames with the given boxes were enqueued.
void grow_bounds(covox_submap *s, const FrameArgs &f)
{
    for (int a = 0; a < 3; ++a) {
        const int32_t lo = f.blo[a], hi = f.blo[a] + f.bdim[a] - 1;
        if (!s->bound_valid) { s->bound_lo[a] = lo; s->bound_hi[a] = hi; }
        else { s->bound_lo[a] = std::min(s->bound_lo[a], lo); s->bound_hi[a] = std::max(s->bound_hi[a], hi); }
    }
    s->bound_valid = true;
}

int integrate_frame(covox_ctx *ctx, covox_submap *s, const float *depth, int32_t H, int32_t W,
                    const float K[4], const double T_wc[16], bool *maybe_full)
{
    const covox_params &p = ctx->p;
    if (p.integrator == COVOX_RAYCAST) return raycast_frame(ctx, s, depth, H, W, K, T_wc, maybe_full);
    FrameArgs f;
    int64_t n_box = 0;
    int rc = prepare_frame(ctx, s, depth, H, W, K, T_wc, f, n_box);
    if (rc) return rc;
    const double tau = p.trunc_vox * p.voxel_size;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->cand, &ctx->cand_cap, n_box, sizeof(uint32_t), "candidates")))
        return rc;
    // touched keys, then (from n_box on) the new blocks' keys
    if ((rc = ensure_buffer(ctx, (void **)&ctx->t_key, &ctx->t_key_cap, 2 * n_box, sizeof(uint64_t), "touched keys")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->t_idx, &ctx->t_idx_cap, n_box, sizeof(uint32_t), "touched index")))
        return rc;

    const float vs = (float)p.voxel_size, tau_f = (float)tau, maxr = (float)p.max_range;
    const uint64_t tmask = (uint64_t)s->tcap - 1;
    const int64_t table_limit = (int64_t)(0.85 * (double)s->tcap);
    const unsigned grid = (unsigned)((n_box + 3) / 4);
    refresh_block_bound(s, n_box);  // s->seq is now this frame's sequence number
    // Existing blocks are updated by the probe when no capacity failure is
    // possible for this frame (every box block new would still fit).
    const bool fused = s->nb_upper + n_box <= std::min<int64_t>(s->cap, table_limit);
    if (p.precision == COVOX_FP16)
        launch_frame<__half>(ctx, s, f, vs, tau_f, maxr, tmask, table_limit, n_box, grid, fused);
    else
        launch_frame<float>(ctx, s, f, vs, tau_f, maxr, tmask, table_limit, n_box, grid, fused);
    if ((rc = hip_check(ctx, hipGetLastError(), "integrate launch"))) return rc;

    // host-side bounds
    s->nb_upper += n_box;
    grow_bounds(s, f);
    s->version++;
    *maybe_full = s->nb_upper > s->cap || s->nb_upper > table_limit;
    return COVOX_OK;
}

int integrate_batch(covox_ctx *ctx, covox_submap *s, const float *depths, int32_t F, int32_t H, int32_t W,
                    const float K[4], const double *T_wc, bool *maybe_full)
{
    if (F <= 0) return COVOX_OK;
    if (F > kMaxBatch) return fail(ctx, COVOX_EINVAL, "integrate_batch: too many frames in one batch");
    const covox_params &p = ctx->p;
    std::vector<FrameArgs> fr(F);
    int64_t box_max = 0, box_sum = 0;
    for (int32_t i = 0; i < F; ++i) {
        int64_t n_box = 0;
        int rc = prepare_frame(ctx, s, depths + (size_t)i * H * W, H, W, K, T_wc + 16 * i, fr[i], n_box);
        if (rc) return rc;
        box_max = std::max(box_max, n_box);
        box_sum += n_box;
    }
    int rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->frames_dev, &ctx->frames_cap, kMaxBatch, sizeof(FrameArgs),
                            "frame batch")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->cand, &ctx->cand_cap, box_max * F, sizeof(uint32_t), "candidates")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->blist, &ctx->blist_cap, std::max<int64_t>(1, s->cap),
                            sizeof(uint32_t), "batch block list")))
        return rc;
    // first-frame table: a power of two holding every candidate twice over
    int64_t fslots = 1;
    while (fslots < 2 * box_sum) fslots <<= 1;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->fkeys, &ctx->fkeys_cap, fslots, sizeof(uint64_t), "first-frame keys")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->ffirst, &ctx->ffirst_cap, fslots, sizeof(uint32_t),
                            "first-frame values")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->fcount, &ctx->fcount_cap, 2 * kMaxBatch, sizeof(int64_t),
                            "frame counts")))
        return rc;
    const bool capture = ctx->capturing;
    uint32_t batch_id;
    if (capture) {
        // A graph replays its batch ids: clear the stamps inside the graph
        // and use an id that uncaptured batches never take.
        fill_u32(ctx->stream, s->stamp, 0u, std::max<int64_t>(1, s->cap));
        batch_id = kCapturedBatch;
    } else {
        if (++s->batch_id == kCapturedBatch) {  // wrapped: clear the stamps
            fill_u32(ctx->stream, s->stamp, 0u, std::max<int64_t>(1, s->cap));
            s->batch_id = 1;
        }
        batch_id = s->batch_id;
    }
    if (capture) {
        // the graph keeps its own copy of the frame parameters
        void *h = nullptr;
        if ((rc = hip_check(ctx, hipHostMalloc(&h, sizeof(FrameArgs) * F, hipHostMallocDefault), "frame staging")))
            return rc;
        ctx->cap_host.push_back(h);
        ::memcpy(h, fr.data(), sizeof(FrameArgs) * F);
        if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->frames_dev, h, sizeof(FrameArgs) * F, hipMemcpyHostToDevice,
                                                ctx->stream), "frame batch upload")))
            return rc;
    } else if ((rc = stage_frames(ctx, fr.data(), F))) {
        return rc;
    }
    const float vs = (float)p.voxel_size, tau_f = (float)(p.trunc_vox * p.voxel_size), maxr = (float)p.max_range;
    const uint64_t tmask = (uint64_t)s->tcap - 1;
    const int64_t table_limit = (int64_t)(0.85 * (double)s->tcap);
    refresh_block_bound(s, box_sum);
    {
        TimedLaunch tl(ctx, COVOX_K_PROBE);
        const int64_t items = (box_max + 3) / 4 * F;
        const unsigned pgrid = (unsigned)((std::min<int64_t>(items, 1 << 20) + 7) / 8 * 8);
        hipLaunchKernelGGL(k_probe_batch, dim3(pgrid), dim3(256), 0, ctx->stream,
                           ctx->frames_dev, vs, tau_f, maxr, s->tkeys, s->tvals, tmask, ctx->cand, box_max, F,
                           (int)(ctx->tune.mapping_xcd_order != 0));
    }
    {
        TimedLaunch tl(ctx, COVOX_K_SCAN);
        const unsigned gx = (unsigned)std::min<int64_t>((box_max + 255) / 256, 256);
        fill_u64(ctx->stream, ctx->fkeys, kEmpty, fslots);
        fill_u32(ctx->stream, ctx->ffirst, 0xFFFFFFFFu, fslots);
        hipLaunchKernelGGL(k_batch_first, dim3(gx, (unsigned)F), dim3(256), 0, ctx->stream, ctx->frames_dev, ctx->cand,
                           box_max, ctx->fkeys, ctx->ffirst, (uint64_t)fslots - 1);
        hipLaunchKernelGGL(k_batch_rank, dim3((unsigned)F), dim3(1024), 0, ctx->stream, ctx->frames_dev, ctx->cand,
                           box_max, ctx->fkeys, ctx->ffirst, (uint64_t)fslots - 1, ctx->fcount);
        hipLaunchKernelGGL(k_batch_commit, dim3(1), dim3(64), 0, ctx->stream, F, ctx->fcount, ctx->fcount + kMaxBatch,
                           s->meta, s->cap, table_limit, s->pin_nb_dev, s->seq);
        hipLaunchKernelGGL(k_batch_activate, dim3(gx, (unsigned)F), dim3(256), 0, ctx->stream, ctx->frames_dev,
                           ctx->cand, box_max, ctx->fcount + kMaxBatch, s->meta, s->keys, s->tkeys, s->tvals, tmask,
                           s->stamp, batch_id, ctx->blist);
    }
    {
        // one wave per listed block (at most min(capacity, sum of the boxes))
        const int64_t waves = std::max<int64_t>(1, std::min(s->cap, s->nb_upper + box_sum));
        const unsigned grid = (unsigned)std::min<int64_t>((waves + 3) / 4 + 7, 1 << 20) / 8 * 8;
        const int xcd = ctx->tune.mapping_xcd_order != 0;
        TimedLaunch tl(ctx, COVOX_K_INTEGRATE);
        if (p.precision == COVOX_FP16)
            hipLaunchKernelGGL(k_integrate_batch<__half>, dim3(grid), dim3(256), 0, ctx->stream, ctx->frames_dev,
                               s->meta, ctx->blist, s->keys, (__half *)s->D, (__half *)s->W, vs, tau_f, maxr,
                               s->dirty, xcd);
        else
            hipLaunchKernelGGL(k_integrate_batch<float>, dim3(grid), dim3(256), 0, ctx->stream, ctx->frames_dev,
                               s->meta, ctx->blist, s->keys, (float *)s->D, (float *)s->W, vs, tau_f, maxr,
                               s->dirty, xcd);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "integrate batch launch"))) return rc;
    s->nb_upper += box_sum;
    for (int32_t i = 0; i < F; ++i) grow_bounds(s, fr[i]);
    s->version++;
    *maybe_full = s->nb_upper > s->cap || s->nb_upper > table_limit;
    return COVOX_OK;
}

}  // namespace covox
