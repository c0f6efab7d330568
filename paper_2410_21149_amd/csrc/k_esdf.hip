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

#include <string.h>

#include <algorithm>
#include <vector>

namespace covox {

namespace {

constexpr int kBig = 1 << 24;
constexpr int kWin = 256;     // envelope window positions (u8 stack entries)
constexpr int kMaxJobs = kEsdfMaxJobs;  // submaps per launch (the job list is a kernel argument)

template <typename S> __device__ __forceinline__ float ldv(const S *p);
template <> __device__ __forceinline__ float ldv<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldv<__half>(const __half *p) { return __half2float(*p); }

// One submap of an ESDF launch.
struct EsdfJob {
    SubmapMeta *meta;
    EsdfSnap *snap;     // the update's domain (written by the page kernel)
    const uint64_t *keys;
    const uint64_t *tkeys;
    const uint32_t *tvals;
    uint64_t tmask;
    const void *D;
    const void *W;
    float *phi;
    int32_t *page;
    float *seeds;       // phi seed per voxel, by dense block index of the launch
    uint8_t *dirty;     // the submap's per-block change flags (cleared by the page kernel with SEEDS)
    int32_t full;       // every allocated block gets a new phi (else only those near a changed block)
};

template <int NJ>
struct JobList {
    EsdfJob j[NJ];
    int n;
};

// Per-workgroup view of a launch, derived from the submaps' device
// bookkeeping: each submap's domain (its allocated block box) and exclusive
// prefix sums of the work items of every pass over the submaps.  The dense
// prefix is also the offset of the submap's blocks in the shared scratch.
struct JobInfo {
    int32_t lo[3], dim[3];
    int64_t nd, nb;           // dense blocks of the box, allocated blocks
    int64_t od, ob, oy, oz;   // prefixes: dense, allocated, y columns, z columns
    int64_t oxy, ozc;         // prefixes: y and z column segments of the column passes
};

struct Plan {
    JobInfo info[kMaxJobs];
    int n;
    int64_t td, tb, ty, tz, txy, tzc;   // totals
};

__device__ __forceinline__ int64_t nsegments(int64_t L, int S) { return L > 0 ? (L + S - 1) / S : 0; }

// Work items of the column passes (segments of Sseg blocks along the pass
// axis; none when Sseg is 0).
struct ColCounts {
    int64_t cy, cz, cxy, czc;
};

// Fills the job info of one submap: from the live block count and block box
// (SNAP = false: the page kernel, which runs in order with the integration),
// or from the snapshot the page kernel stored (SNAP = true: the EDT passes,
// which may run while the next frames are integrated into the same submap).
template <bool SNAP>
__device__ __forceinline__ void job_info(const EsdfJob &job, int C, int Sseg, JobInfo &ji, ColCounts &cc)
{
    const SubmapMeta *m = job.meta;
    const EsdfSnap *sn = job.snap;
    for (int a = 0; a < 3; ++a) { ji.lo[a] = 0; ji.dim[a] = 0; }
    ji.nd = 0;
    ji.nb = 0;
    cc.cy = cc.cz = cc.cxy = cc.czc = 0;
    const int64_t nb = SNAP ? (int64_t)sn->nb : m->n_blocks;
    if (nb <= 0) return;
    ji.nb = nb;
    ji.nd = 1;
    for (int a = 0; a < 3; ++a) {
        ji.lo[a] = SNAP ? sn->lo[a] : m->bmin[a];
        ji.dim[a] = SNAP ? sn->dim[a] : m->bmax[a] - m->bmin[a] + 1;
        ji.nd *= ji.dim[a];
    }
    const int S = kWin - 2 * C;
    cc.cy = (int64_t)ji.dim[0] * ji.dim[2] * nsegments(8 * (int64_t)ji.dim[1], S);
    cc.cz = (int64_t)ji.dim[0] * ji.dim[1] * nsegments(8 * (int64_t)ji.dim[2], S);
    if (Sseg > 0) {
        cc.cxy = (int64_t)ji.dim[0] * ji.dim[2] * nsegments(ji.dim[1], Sseg);
        cc.czc = (int64_t)ji.dim[0] * ji.dim[1] * nsegments(ji.dim[2], Sseg);
    }
}

// The plan of a multi-submap launch: the first wave derives one submap per
// lane with wave prefix sums, then a workgroup barrier publishes it.  A
// single-submap launch keeps its one entry in registers instead (PlanView).
template <bool SNAP, int NJ>
__device__ void make_plan(const JobList<NJ> &jl, int C, int Sseg, Plan &pl)
{
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        JobInfo ji;
        ColCounts cc = {0, 0, 0, 0};
        for (int a = 0; a < 3; ++a) { ji.lo[a] = 0; ji.dim[a] = 0; }
        ji.nd = ji.nb = 0;
        if (lane < jl.n) job_info<SNAP>(jl.j[lane], C, Sseg, ji, cc);
        const int64_t v[6] = {ji.nd, ji.nb, cc.cy, cc.cz, cc.cxy, cc.czc};
        int64_t incl[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            int64_t x = v[k];
            for (int o = 1; o < 64; o <<= 1) {
                const int64_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            incl[k] = x;
        }
        if (lane < jl.n) {
            ji.od = incl[0] - v[0];
            ji.ob = incl[1] - v[1];
            ji.oy = incl[2] - v[2];
            ji.oz = incl[3] - v[3];
            ji.oxy = incl[4] - v[4];
            ji.ozc = incl[5] - v[5];
            pl.info[lane] = ji;
        }
        if (lane == 63) {
            pl.n = jl.n;
            pl.td = incl[0];
            pl.tb = incl[1];
            pl.ty = incl[2];
            pl.tz = incl[3];
            pl.txy = incl[4];
            pl.tzc = incl[5];
        }
    }
    __syncthreads();
}

// Submap owning global work item w of a pass (largest j with offset <= w).
template <int64_t JobInfo::*OFF>
__device__ __forceinline__ int find_job(const Plan &pl, int64_t w)
{
    int lo = 0, hi = pl.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pl.info[mid].*OFF <= w) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Uniform access to the plan: registers for one submap, LDS for several.
template <int NJ, bool SNAP = true>
struct PlanView {
    Plan *pl;
    JobInfo one;
    // totals: dense, allocated, y columns, z columns, y and z column segments
    int64_t t[6];

    __device__ void init(const JobList<NJ> &jl, int C, Plan &lds, int Sseg = 0)
    {
        if constexpr (NJ == 1) {
            ColCounts cc;
            job_info<SNAP>(jl.j[0], C, Sseg, one, cc);
            one.od = one.ob = one.oy = one.oz = one.oxy = one.ozc = 0;
            t[0] = one.nd;
            t[1] = one.nb;
            t[2] = cc.cy;
            t[3] = cc.cz;
            t[4] = cc.cxy;
            t[5] = cc.czc;
            pl = nullptr;
        } else {
            make_plan<SNAP>(jl, C, Sseg, lds);
            pl = &lds;
            t[0] = lds.td;
            t[1] = lds.tb;
            t[2] = lds.ty;
            t[3] = lds.tz;
            t[4] = lds.txy;
            t[5] = lds.tzc;
        }
    }
    template <int64_t JobInfo::*OFF>
    __device__ int job(int64_t w) const
    {
        if constexpr (NJ == 1) return 0;
        else return find_job<OFF>(*pl, w);
    }
    __device__ JobInfo info(int j) const
    {
        if constexpr (NJ == 1) return one;
        else return pl->info[j];
    }
};

__device__ __forceinline__ void dom_coords(const JobInfo &d, int64_t db, int &x, int &y, int &z)
{
    x = (int)(db % d.dim[0]);
    y = (int)((db / d.dim[0]) % d.dim[1]);
    z = (int)(db / ((int64_t)d.dim[0] * d.dim[1]));
}

__device__ __forceinline__ int64_t dom_index(const JobInfo &d, int x, int y, int z)
{
    return ((int64_t)z * d.dim[1] + y) * d.dim[0] + x;
}

// Page (dense block -> buffer index, -1 if unallocated), site masks and the
// snapshot of each submap's domain (block box and block count) that the later
// passes work on.  Two independent loops: one lane per dense block looks its
// key up in the hash table (64 lookups in flight per wave), writes the page
// and, for an unallocated block, empty site masks; one wave per allocated
// block reads its D and W and writes its site masks.  With SEEDS, that wave
// also writes the phi seed of each voxel: NaN when unobserved, D inside the
// band, and otherwise an infinity with the sign of D.  The EDT passes then
// never read the TSDF or the submap's bookkeeping, so that the next frames
// may be integrated while they run.
template <typename S, int NJ, bool SEEDS>
__global__ __launch_bounds__(256) void k_page_sites(const JobList<NJ> jl, int C, float vs, float tau,
                                                    uint64_t *__restrict__ sites, int32_t *__restrict__ blk,
                                                    uint8_t *__restrict__ ddirty)
{
    __shared__ Plan lds;
    PlanView<NJ, false> pv;
    pv.init(jl, C, lds);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (blockIdx.x == 0 && (int)threadIdx.x < jl.n) {
        const JobInfo d = pv.info(threadIdx.x);
        SubmapMeta *m = jl.j[threadIdx.x].meta;
        EsdfSnap *sn = jl.j[threadIdx.x].snap;
        for (int a = 0; a < 3; ++a) {
            m->dom_min[a] = sn->lo[a] = d.lo[a];
            m->dom_dim[a] = sn->dim[a] = d.dim[a];
        }
        m->dom_nblocks = sn->nb = (int32_t)d.nb;
        m->dom_valid = 1;
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pv.t[0];
         g += (int64_t)gridDim.x * blockDim.x) {
        const int j = pv.template job<&JobInfo::od>(g);
        const JobInfo d = pv.info(j);
        const EsdfJob &job = jl.j[j];
        const int64_t db = g - d.od;
        int x, y, z;
        dom_coords(d, db, x, y, z);
        const int64_t idx =
            hash_find(job.tkeys, job.tvals, job.tmask, pack_key(d.lo[0] + x, d.lo[1] + y, d.lo[2] + z));
        job.page[db] = (int32_t)idx;
        if (blk) blk[g] = (int32_t)idx;  // the launch's own copy, read by the column passes
        if (ddirty && idx < 0) ddirty[g] = 0;
        if (idx < 0) {
            uint4 *w = (uint4 *)(sites + g * 8);
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    for (int64_t w = (int64_t)blockIdx.x * 4 + wid; w < pv.t[1]; w += (int64_t)gridDim.x * 4) {
        const int jj = pv.template job<&JobInfo::ob>(w);
        const JobInfo d = pv.info(jj);
        const EsdfJob &job = jl.j[jj];
        const int64_t idx = w - d.ob;
        int bx, by, bz;
        unpack_key(job.keys[idx], bx, by, bz);
        const int64_t g = d.od + dom_index(d, bx - d.lo[0], by - d.lo[1], bz - d.lo[2]);
        if constexpr (SEEDS) {
            // an exact update consumes the block's change flag
            if (lane == 0) {
                if (ddirty) ddirty[g] = job.full ? 1 : job.dirty[idx];
                job.dirty[idx] = 0;
            }
        }
        const S *Db = (const S *)job.D + idx * 512 + lane;
        const S *Wb = (const S *)job.W + idx * 512 + lane;
        // all reads before the first write (the seeds), so that they overlap
        float Dk[8], Wk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            Dk[k] = ldv(Db + 64 * k);
            Wk[k] = ldv(Wb + 64 * k);
        }
        uint64_t wm = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float Dv = Dk[k], Wv = Wk[k];
            const uint64_t m = __ballot(Wv > 0.0f && fabsf(Dv) <= vs);
            if (lane == k) wm = m;
            if constexpr (SEEDS)
                job.seeds[g * 512 + lane + 64 * k] =
                    !(Wv > 0.0f) ? __builtin_nanf("")
                                 : (fabsf(Dv) < tau ? Dv : (Dv > 0.0f ? __builtin_inff() : -__builtin_inff()));
        }
        if (lane < 8) sites[g * 8 + lane] = wm;
    }
}

// The x distances of the 8 voxels of one x-line of a block, as 8 bytes:
// byte x is the distance from bit 8 HB + x of the 128-bit site window
// (lo, hi) to its nearest set bit, or 255 when that exceeds R or the window
// has none.  The window holds the 2 HB + 1 blocks' bytes of the line (the
// own block's byte at bit 8 HB, in lo since HB <= 7; zero above).  The
// nearest sites below and above the own byte are found once per line, and
// each voxel then looks only inside its own byte.
__device__ __forceinline__ uint64_t line_dists(uint64_t lo, uint64_t hi, int HB, int R)
{
    constexpr int kNone = 1000;
    const int p0 = 8 * HB;
    const uint32_t b = (uint32_t)(lo >> p0) & 0xFFu;
    const uint64_t below = lo & ((1ull << p0) - 1ull);  // p0 <= 56
    const int dl0 = below ? p0 - (63 - __clzll((long long)below)) : kNone;  // from bit p0 down
    const uint64_t above = p0 + 8 < 64 ? lo >> (p0 + 8) : 0ull;
    const int dr7 = above ? __ffsll((long long)above)                        // from bit p0 + 7 up
                          : (hi ? 64 - (p0 + 7) + (__ffsll((long long)hi) - 1) : kNone);
    uint64_t out = 0;
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const uint32_t ml = b & ((2u << x) - 1u);  // own sites at or below x
        const uint32_t mr = b >> x;                // own sites at or above x
        const int dl = ml ? x - (31 - __clz((int)ml)) : x + dl0;
        const int dr = mr ? __ffs((int)mr) - 1 : (7 - x) + dr7;
        const int d = min(dl, dr);
        out |= (uint64_t)(d <= R ? d : 255) << (8 * x);
    }
    return out;
}

// ------------------------------------------------------------------------
// Voxel-parallel passes: one 512-lane workgroup per block, one lane per
// voxel (l = x + 8y + 64z), the 2 HB + 1 neighbour blocks along the pass axis
// staged in LDS.  The min-plus search walks outward from the voxel and stops
// once d^2 reaches the best value, so it is exact; its cost follows the
// distance to the nearest site rather than the line length, which suits
// small domains where per-line envelopes leave the GPU idle.

// The y passes' candidates g1^2 + e^2 without the test for 255 (no site
// within R along x): 255 squares to 65025, above every candidate from a real
// distance (at most 2 R^2), so the minimum is the same wherever it is at most
// R^2 (the only values written), and a search still never ends early while
// a voxel has no real candidate (the exit needs e^2 >= its best, e <= R).
static_assert(2 * (8 * kMaxHalo) * (8 * kMaxHalo) < 255 * 255, "255 must square above every real candidate");
__device__ __forceinline__ int cand8(uint32_t byte, int ee) { return (int)(byte * byte) + ee; }

constexpr int kScanStep = 8;  // offsets per exit test of the windowed y and z passes
// 32-bit words a lane stages into LDS per block in the z pass (512 lanes,
// 2 HB + 1 blocks of 256 words)
constexpr int kStageZ = ((2 * kMaxHalo + 1) * 256 + 511) / 512;

// The z passes' candidates g2 + e^2, likewise without the test for 0xFFFF
// (no site within R in the xy plane): 65535 lies above every candidate from
// a real value (g2 <= R^2, so at most 2 R^2), so phi (which takes R^2 as the
// limit) and the exits (e^2 >= best, e <= R) are unchanged.
__device__ __forceinline__ int cand16(uint16_t v, int ee) { return (int)v + ee; }

// x pass: one wave per dense block, lane = (y, z) line of the block.  The
// lane gathers byte y of site word z from the 2 HB + 1 blocks along x into a
// 128-bit mask and stores the 8 distances of its line (x = 0..7, contiguous
// in the block layout) as one 8-byte word; no LDS and no barriers, so
// consecutive blocks of a wave overlap their loads.
template <int NJ>
__global__ __launch_bounds__(256) void k_edt_x(const JobList<NJ> jl, const uint64_t *__restrict__ sites,
                                               uint8_t *__restrict__ g1, int R, int HB)
{
    __shared__ Plan lds;
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int y = lane & 7, z = lane >> 3;
    for (int64_t g = (int64_t)blockIdx.x * 4 + wid; g < pv.t[0]; g += (int64_t)gridDim.x * 4) {
        const JobInfo d = pv.info(pv.template job<&JobInfo::od>(g));
        int bx, by, bz;
        dom_coords(d, g - d.od, bx, by, bz);
        // the site words of the 2 HB + 1 blocks along x, read together
        // (slots past the halo or outside the domain read this block's word
        // and drop it)
        uint64_t wv[2 * kMaxHalo + 1];
#pragma unroll
        for (int i = 0; i < 2 * kMaxHalo + 1; ++i) {
            const int nx = bx + i - HB;
            const bool ok = i < 2 * HB + 1 && nx >= 0 && nx < d.dim[0];
            const uint64_t v = sites[(ok ? g + (i - HB) : g) * 8 + z];
            wv[i] = ok ? v : 0ull;
        }
        uint64_t lo = 0, hi = 0;
#pragma unroll
        for (int i = 0; i < 2 * kMaxHalo + 1; ++i) {
            const uint64_t byte = (wv[i] >> (8 * y)) & 0xFFull;
            const int pos = 8 * i;
            if (pos < 64) lo |= byte << pos;
            else hi |= byte << (pos - 64);
        }
        *(uint64_t *)(g1 + g * 512 + 8 * lane) = line_dists(lo, hi, HB, R);
    }
}

// y pass with a column layout in LDS: the staged g1 values of each (x, z)
// column of the 2 HB + 1 blocks are contiguous (y fastest), so that a lane
// reads four offsets of its column with one 32-bit LDS read per direction
// (two dwords, joined by a byte shift where the four rows straddle them).
// 256 lanes per block, each lane the voxels z and z + 4.  The minimum is the
// same as the windowed pass's: the same offsets, tested for exit every eight.
constexpr int kColBytes = 132;  // per column: 4 bytes of margin, 8 (2 kMaxHalo + 1) rows, margin; 33
                                // dwords, so that the 8 x columns a wave reads fall in different banks

template <int NJ>
__global__ __launch_bounds__(256) void k_edt_y_col(const JobList<NJ> jl, const uint8_t *__restrict__ g1,
                                                   uint16_t *__restrict__ g2, int R, int HB)
{
    constexpr int kStage = ((2 * kMaxHalo + 1) * 128 + 255) / 256;  // staged words per lane
    __shared__ Plan lds;
    __shared__ __align__(16) uint32_t colw[64 * kColBytes / 4 + 4];
    uint8_t *colb = (uint8_t *)colw;
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds);
    const int tid = threadIdx.x;
    const int x = tid & 7, y = (tid >> 3) & 7, z = tid >> 6;  // z in 0..3; the lane also takes z + 4
    const int nb = 2 * HB + 1;
    const int R2 = R * R;
    const int Y = 8 * HB + y;
    const int c0 = x + 8 * z, c1 = x + 8 * (z + 4);
    const uint32_t *cw0 = colw + c0 * (kColBytes / 4), *cw1 = colw + c1 * (kColBytes / 4);
    // row r of a column is byte 4 + r: the rows Y - 4m - 4 .. Y - 4m - 1 start
    // in dword (Y >> 2) - m at byte Y & 3, the rows Y + 4m + 1 .. Y + 4m + 4
    // in dword ((Y + 5) >> 2) + m at byte (Y + 5) & 3
    const int dn = Y >> 2, sdn = Y & 3, up = (Y + 5) >> 2, sup = (Y + 5) & 3;
    for (int64_t g = blockIdx.x; g < pv.t[0]; g += gridDim.x) {
        const JobInfo d = pv.info(pv.template job<&JobInfo::od>(g));
        int bx, by, bz;
        dom_coords(d, g - d.od, bx, by, bz);
        // stage: every read issued before the first LDS write (entries outside
        // the domain read this block's word and drop it)
        uint32_t sv[kStage];
#pragma unroll
        for (int q = 0; q < kStage; ++q) {
            const int e = tid + 256 * q, i = e >> 7, w = e & 127;
            const int ny = by + i - HB;
            const bool ok = e < nb * 128 && ny >= 0 && ny < d.dim[1];
            sv[q] = ((const uint32_t *)(g1 + (g + (ok ? (int64_t)(i - HB) * d.dim[0] : 0)) * 512))[ok ? w : 0];
            sv[q] = ok ? sv[q] : 0xFFFFFFFFu;
        }
        // word w of staged block i holds x = 4 (w & 1) + k, y = (w >> 1) & 7,
        // z = w >> 4 for its bytes k = 0..3: row 8 i + y of column x + 8 z
#pragma unroll
        for (int q = 0; q < kStage; ++q) {
            const int e = tid + 256 * q;
            if (e < nb * 128) {
                const int i = e >> 7, w = e & 127;
                uint8_t *dst = colb + (4 * (w & 1) + 8 * (w >> 4)) * kColBytes + 4 + 8 * i + ((w >> 1) & 7);
#pragma unroll
                for (int k = 0; k < 4; ++k) dst[k * kColBytes] = (uint8_t)(sv[q] >> (8 * k));
            }
        }
        __syncthreads();
        int b0 = cand8(colb[c0 * kColBytes + 4 + Y], 0), b1 = cand8(colb[c1 * kColBytes + 4 + Y], 0);
        // sliding dword windows per direction and voxel
        uint32_t dhi0 = cw0[dn + 1], dhi1 = cw1[dn + 1];  // "-": the dword above the next one
        uint32_t ulo0 = cw0[up], ulo1 = cw1[up];          // "+": the dword below the next one
        for (int dd = 1, m = 0; dd <= R; dd += 8) {
            if (dd * dd >= max(b0, b1)) break;
#pragma unroll
            for (int h = 0; h < 2; ++h, ++m) {
                const uint32_t dlo0 = cw0[dn - m], dlo1 = cw1[dn - m];
                const uint32_t uhi0 = cw0[up + m + 1], uhi1 = cw1[up + m + 1];
                const uint32_t dv0 = __builtin_amdgcn_alignbyte(dhi0, dlo0, sdn);
                const uint32_t dv1 = __builtin_amdgcn_alignbyte(dhi1, dlo1, sdn);
                const uint32_t uv0 = __builtin_amdgcn_alignbyte(uhi0, ulo0, sup);
                const uint32_t uv1 = __builtin_amdgcn_alignbyte(uhi1, ulo1, sup);
                dhi0 = dlo0; dhi1 = dlo1;
                ulo0 = uhi0; ulo1 = uhi1;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int e = 4 * m + 1 + k;  // byte 3 - k going down, byte k going up
                    if (e <= R) {
                        const int ee = e * e;
                        b0 = min(b0, min(cand8((dv0 >> (8 * (3 - k))) & 0xFFu, ee), cand8((uv0 >> (8 * k)) & 0xFFu, ee)));
                        b1 = min(b1, min(cand8((dv1 >> (8 * (3 - k))) & 0xFFu, ee), cand8((uv1 >> (8 * k)) & 0xFFu, ee)));
                    }
                }
            }
        }
        g2[g * 512 + tid] = b0 <= R2 ? (uint16_t)b0 : (uint16_t)0xFFFF;
        g2[g * 512 + tid + 256] = b1 <= R2 ? (uint16_t)b1 : (uint16_t)0xFFFF;
        __syncthreads();
    }
}

// phi of a voxel outside the band from its seed (an infinity with the sign
// of D) and the squared distance search result.
__device__ __forceinline__ float phi_value(float seed, int best, int R2, float vs, float dmax)
{
    const float sg = seed > 0.0f ? 1.0f : -1.0f;
    if (best > R2) return sg * dmax;
    return sg * fminf(dmax, vs * sqrtf((float)best));
}

template <int NJ>
__global__ __launch_bounds__(512) void k_edt_z_vox(const JobList<NJ> jl, const uint16_t *__restrict__ g2, int R,
                                                   int HB, float vs, float dmax)
{
    __shared__ Plan lds;
    __shared__ __align__(16) uint32_t colw[(2 * kMaxHalo + 1) * 256];
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds);
    const uint16_t *col = (const uint16_t *)colw;
    const int tid = threadIdx.x;
    const int z = tid >> 6;
    const int nb = 2 * HB + 1;
    const int R2 = R * R;
    const int Z = 8 * HB + z;
    for (int64_t w = blockIdx.x; w < pv.t[1]; w += gridDim.x) {
        const int jj = pv.template job<&JobInfo::ob>(w);
        const JobInfo d = pv.info(jj);
        const EsdfJob &job = jl.j[jj];
        const int64_t j = w - d.ob;
        int bx, by, bz;
        unpack_key(job.keys[j], bx, by, bz);
        bx -= d.lo[0]; by -= d.lo[1]; bz -= d.lo[2];
        const int64_t g = d.od + dom_index(d, bx, by, bz);
        const int64_t stride_z = (int64_t)d.dim[0] * d.dim[1];
        // stage the column as in the y pass
        uint32_t sv[kStageZ];
#pragma unroll
        for (int r = 0; r < kStageZ; ++r) {
            const int e = tid + 512 * r, i = e >> 8, q = e & 255;
            const int nz = bz + i - HB;
            const bool ok = e < nb * 256 && nz >= 0 && nz < d.dim[2];
            sv[r] = ((const uint32_t *)(g2 + (g + (ok ? (int64_t)(i - HB) * stride_z : 0)) * 512))[ok ? q : 0];
            sv[r] = ok ? sv[r] : 0xFFFFFFFFu;
        }
        const float seed = job.seeds[g * 512 + tid];  // from k_page_sites
#pragma unroll
        for (int r = 0; r < kStageZ; ++r)
            if (tid + 512 * r < nb * 256) colw[tid + 512 * r] = sv[r];
        __syncthreads();
        // an unobserved (NaN) or in-band (D) seed is the result
        float out = seed;
        if (__builtin_isinf(seed)) {
            const int base = tid & 63;
            auto at = [&](int zz) { return col[(zz >> 3) * 512 + base + 64 * (zz & 7)]; };
            int best = cand16(at(Z), 0);
            for (int dd = 1; dd <= R; dd += kScanStep) {  // as in the y pass
                if (dd * dd >= best) break;
#pragma unroll
                for (int q = 0; q < kScanStep; ++q) {
                    const int e = dd + q;
                    if (e <= R) best = min(best, min(cand16(at(Z - e), e * e), cand16(at(Z + e), e * e)));
                }
            }
            out = phi_value(seed, best, R2, vs, dmax);
        }
        job.phi[j * 512 + tid] = out;
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// The region of a partial update (jobs with full = 0): the blocks of the
// launch's page copy (blk) whose phi can change are those within HB blocks,
// along every axis, of a block whose TSDF changed since the last exact
// update -- a site HB + 1 blocks away along some axis is more than 8 HB >= R
// voxels away.  Two dilations of the change flags: k_esdf_dil_x along x into
// dx, then k_esdf_region clears blk for allocated blocks with no flagged dx
// within HB along y and z, which the column passes then neither write nor
// read.  Jobs with full = 1 have every allocated block flagged.
template <int NJ>
__global__ __launch_bounds__(256) void k_esdf_dil_x(const JobList<NJ> jl, int HB, const uint8_t *__restrict__ ddirty,
                                                    uint8_t *__restrict__ dx)
{
    __shared__ Plan lds;
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pv.t[0];
         g += (int64_t)gridDim.x * blockDim.x) {
        const JobInfo d = pv.info(pv.template job<&JobInfo::od>(g));
        int x, y, z;
        dom_coords(d, g - d.od, x, y, z);
        uint8_t any = 0;
        for (int k = max(0, x - HB); k <= min(d.dim[0] - 1, x + HB); ++k) any |= ddirty[g + (k - x)];
        dx[g] = any;
    }
}

template <int NJ>
__global__ __launch_bounds__(256) void k_esdf_region(const JobList<NJ> jl, int HB, const uint8_t *__restrict__ dx,
                                                     int32_t *__restrict__ blk)
{
    __shared__ Plan lds;
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pv.t[0];
         g += (int64_t)gridDim.x * blockDim.x) {
        if (blk[g] < 0) continue;
        const JobInfo d = pv.info(pv.template job<&JobInfo::od>(g));
        int x, y, z;
        dom_coords(d, g - d.od, x, y, z);
        bool any = false;
        for (int zz = max(0, z - HB); zz <= min(d.dim[2] - 1, z + HB) && !any; ++zz)
            for (int yy = max(0, y - HB); yy <= min(d.dim[1] - 1, y + HB) && !any; ++yy)
                any = dx[d.od + dom_index(d, x, yy, zz)] != 0;
        if (!any) blk[g] = -1;
    }
}

// ------------------------------------------------------------------------
// Column passes.  Each workgroup owns a segment of Sseg blocks of one block
// column along the pass axis and stages the segment with HB halo blocks on
// each side once, so that no block is staged more than 1 + 2 HB / Sseg times
// (the per-block passes above stage 2 HB + 1 blocks for every block).
//
// k_edt_xy fuses the x pass into the y pass: the x distances of the staged
// blocks of a y column (bx, *, bz) come from the site masks straight into
// LDS, in the column layout of k_edt_y_col, and g2 is written only for the
// segment's blocks that the z pass reads (those with an allocated block
// within HB blocks along z).  k_edt_z_col stages g2 of a z column (bx, by,
// *) that holds an allocated block and writes phi of its allocated blocks.
// Both passes read the launch's copy of the page (blk: buffer index per
// dense block, -1 when unallocated), never the submap's bookkeeping.
//
// The searches and exit tests are those of k_edt_y_col and k_edt_z_vox, so
// every squared distance, and phi, is the same bit for bit.
constexpr int kColMaxStage = 48;  // staged blocks of a segment: Sseg + 2 HB

template <int NJ>
__global__ __launch_bounds__(256) void k_edt_xy(const JobList<NJ> jl, int Sseg, const uint64_t *__restrict__ sites,
                                                const int32_t *__restrict__ blk, uint16_t *__restrict__ g2, int R,
                                                int HB)
{
    __shared__ Plan lds;
    // 64 columns (x + 8 z) of 4 * (2 nst + 3) bytes: 4 bytes of margin, then
    // the 8 nst staged rows along y; an odd stride in dwords puts the 8 x
    // columns a wave reads in different banks
    __shared__ __align__(16) uint32_t colw[64 * (2 * kColMaxStage + 3)];
    __shared__ uint64_t need_s;
    uint8_t *colb = (uint8_t *)colw;
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds, Sseg);
    const int tid = threadIdx.x;
    const int x = tid & 7, y = (tid >> 3) & 7, z = tid >> 6;  // the lane's voxels: (x, y, z) and (x, y, z + 4)
    const int R2 = R * R;
    for (int64_t c = blockIdx.x; c < pv.t[4]; c += gridDim.x) {
        const JobInfo d = pv.info(pv.template job<&JobInfo::oxy>(c));
        const int nseg = (d.dim[1] + Sseg - 1) / Sseg;
        const int64_t cl = c - d.oxy;
        const int seg = (int)(cl % nseg);
        const int64_t cc = cl / nseg;
        const int bx = (int)(cc % d.dim[0]), bz = (int)(cc / d.dim[0]);
        const int y0 = seg * Sseg, y1 = min(y0 + Sseg, d.dim[1]);
        const int nst = (y1 - y0) + 2 * HB;  // staged blocks y0 - HB .. y1 + HB - 1
        const int colB = 4 * (2 * nst + 3);
        // output blocks that the z pass reads: an allocated block within HB along z
        if (tid < 64) {
            const int j = y0 + tid;
            bool need = false;
            if (j < y1) {
                const int za = max(0, bz - HB), zb = min(d.dim[2] - 1, bz + HB);
                for (int zz = za; zz <= zb; ++zz) need = need || blk[d.od + dom_index(d, bx, j, zz)] >= 0;
            }
            const uint64_t m = __ballot(need);
            if (tid == 0) need_s = m;
        }
        __syncthreads();
        const uint64_t need = need_s;
        if (need != 0) {
            // x distances of the staged blocks, one (y, z) row of 8 voxels per
            // item: byte y of site word z of the 2 HB + 1 blocks along x
            // (outside the domain: no sites; staged blocks outside it: none)
            for (int e = tid; e < nst * 64; e += 256) {
                const int i = e >> 6, yr = e & 7, zr = (e >> 3) & 7;
                const int j = y0 - HB + i;
                uint64_t out = ~0ull;
                if (j >= 0 && j < d.dim[1]) {
                    const int64_t g = d.od + dom_index(d, bx, j, bz);
                    uint64_t wv[2 * kMaxHalo + 1];
#pragma unroll
                    for (int k = 0; k < 2 * kMaxHalo + 1; ++k) {
                        const int nx = bx + k - HB;
                        const bool ok = k < 2 * HB + 1 && nx >= 0 && nx < d.dim[0];
                        const uint64_t v = sites[(ok ? g + (k - HB) : g) * 8 + zr];
                        wv[k] = ok ? v : 0ull;
                    }
                    uint64_t lo = 0, hi = 0;
#pragma unroll
                    for (int k = 0; k < 2 * kMaxHalo + 1; ++k) {
                        const uint64_t byte = (wv[k] >> (8 * yr)) & 0xFFull;
                        const int pos = 8 * k;
                        if (pos < 64) lo |= byte << pos;
                        else hi |= byte << (pos - 64);
                    }
                    out = line_dists(lo, hi, HB, R);
                }
                uint8_t *dst = colb + 8 * zr * colB + 4 + 8 * i + yr;
#pragma unroll
                for (int xx = 0; xx < 8; ++xx) dst[xx * colB] = (uint8_t)(out >> (8 * xx));
            }
            __syncthreads();
            const int c0 = x + 8 * z, c1 = x + 8 * (z + 4);
            const uint32_t *cw0 = colw + c0 * (colB / 4), *cw1 = colw + c1 * (colB / 4);
            for (int io = 0; io < y1 - y0; ++io) {
                if (!((need >> io) & 1ull)) continue;  // uniform
                const int Y = 8 * (HB + io) + y;
                // as in k_edt_y_col: rows Y - 4m - 4 .. Y - 4m - 1 in dword (Y >> 2) - m
                // at byte Y & 3; rows Y + 4m + 1 .. Y + 4m + 4 in dword ((Y + 5) >> 2) + m
                // at byte (Y + 5) & 3
                const int dn = Y >> 2, sdn = Y & 3, up = (Y + 5) >> 2, sup = (Y + 5) & 3;
                int b0 = cand8(colb[c0 * colB + 4 + Y], 0), b1 = cand8(colb[c1 * colB + 4 + Y], 0);
                uint32_t dhi0 = cw0[dn + 1], dhi1 = cw1[dn + 1];
                uint32_t ulo0 = cw0[up], ulo1 = cw1[up];
                for (int dd = 1, m = 0; dd <= R; dd += 8) {
                    if (dd * dd >= max(b0, b1)) break;
#pragma unroll
                    for (int h = 0; h < 2; ++h, ++m) {
                        const uint32_t dlo0 = cw0[dn - m], dlo1 = cw1[dn - m];
                        const uint32_t uhi0 = cw0[up + m + 1], uhi1 = cw1[up + m + 1];
                        const uint32_t dv0 = __builtin_amdgcn_alignbyte(dhi0, dlo0, sdn);
                        const uint32_t dv1 = __builtin_amdgcn_alignbyte(dhi1, dlo1, sdn);
                        const uint32_t uv0 = __builtin_amdgcn_alignbyte(uhi0, ulo0, sup);
                        const uint32_t uv1 = __builtin_amdgcn_alignbyte(uhi1, ulo1, sup);
                        dhi0 = dlo0; dhi1 = dlo1;
                        ulo0 = uhi0; ulo1 = uhi1;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int e = 4 * m + 1 + k;
                            if (e <= R) {
                                const int ee = e * e;
                                b0 = min(b0, min(cand8((dv0 >> (8 * (3 - k))) & 0xFFu, ee), cand8((uv0 >> (8 * k)) & 0xFFu, ee)));
                                b1 = min(b1, min(cand8((dv1 >> (8 * (3 - k))) & 0xFFu, ee), cand8((uv1 >> (8 * k)) & 0xFFu, ee)));
                            }
                        }
                    }
                }
                const int64_t g = d.od + dom_index(d, bx, y0 + io, bz);
                g2[g * 512 + tid] = b0 <= R2 ? (uint16_t)b0 : (uint16_t)0xFFFF;
                g2[g * 512 + tid + 256] = b1 <= R2 ? (uint16_t)b1 : (uint16_t)0xFFFF;
            }
        }
        __syncthreads();
    }
}

template <int NJ>
__global__ __launch_bounds__(512) void k_edt_z_col(const JobList<NJ> jl, int Sseg, const uint16_t *__restrict__ g2,
                                                   const int32_t *__restrict__ blk, int R, int HB, float vs,
                                                   float dmax)
{
    __shared__ Plan lds;
    __shared__ __align__(16) uint32_t colw[kColMaxStage * 256];  // staged g2, block by block
    __shared__ int32_t sblk[kColMaxStage + 2 * kMaxHalo];         // blk of z0 - 2 HB .. z1 + 2 HB - 1
    __shared__ uint8_t sneed[kColMaxStage];                      // staged block read by an allocated block
    PlanView<NJ> pv;
    pv.init(jl, 8 * HB, lds, Sseg);
    const uint16_t *col = (const uint16_t *)colw;
    const int tid = threadIdx.x;
    const int R2 = R * R;
    const int base = tid & 63;
    for (int64_t c = blockIdx.x; c < pv.t[5]; c += gridDim.x) {
        const int jj = pv.template job<&JobInfo::ozc>(c);
        const JobInfo d = pv.info(jj);
        const EsdfJob &job = jl.j[jj];
        const int nseg = (d.dim[2] + Sseg - 1) / Sseg;
        const int64_t cl = c - d.ozc;
        const int seg = (int)(cl % nseg);
        const int64_t cc = cl / nseg;
        const int bx = (int)(cc % d.dim[0]), by = (int)(cc / d.dim[0]);
        const int z0 = seg * Sseg, z1 = min(z0 + Sseg, d.dim[2]);
        const int nst = (z1 - z0) + 2 * HB;  // staged blocks z0 - HB .. z1 + HB - 1
        for (int t = tid; t < nst + 2 * HB; t += 512) {
            const int zz = z0 - 2 * HB + t;
            sblk[t] = zz >= 0 && zz < d.dim[2] ? blk[d.od + dom_index(d, bx, by, zz)] : -1;
        }
        __syncthreads();
        bool any = false;
        for (int i = 0; i < z1 - z0; ++i) any = any || sblk[2 * HB + i] >= 0;
        if (any) {  // uniform
            // staged block i (z = z0 - HB + i) is written by k_edt_xy iff an
            // allocated block lies within HB of it: sblk[i .. i + 2 HB]
            for (int i = tid; i < nst; i += 512) {
                const int zz = z0 - HB + i;
                bool nd = false;
                for (int t = i; t <= i + 2 * HB; ++t) nd = nd || sblk[t] >= 0;
                sneed[i] = nd && zz >= 0 && zz < d.dim[2];
            }
            __syncthreads();
            for (int e = tid; e < nst * 256; e += 512) {
                const int i = e >> 8, q = e & 255;
                uint32_t v = 0xFFFFFFFFu;
                if (sneed[i]) v = ((const uint32_t *)(g2 + (d.od + dom_index(d, bx, by, z0 - HB + i)) * 512))[q];
                colw[e] = v;
            }
            __syncthreads();
            for (int io = 0; io < z1 - z0; ++io) {
                const int32_t idx = sblk[2 * HB + io];
                if (idx < 0) continue;  // uniform
                const int64_t g = d.od + dom_index(d, bx, by, z0 + io);
                const float seed = job.seeds[g * 512 + tid];  // from k_page_sites
                float out = seed;  // unobserved (NaN) or in the band (D)
                if (__builtin_isinf(seed)) {
                    const int Z = 8 * (HB + io) + (tid >> 6);
                    auto at = [&](int zz) { return col[(zz >> 3) * 512 + base + 64 * (zz & 7)]; };
                    int best = cand16(at(Z), 0);
                    for (int dd = 1; dd <= R; dd += kScanStep) {  // as in k_edt_z_vox
                        if (dd * dd >= best) break;
#pragma unroll
                        for (int q = 0; q < kScanStep; ++q) {
                            const int e = dd + q;
                            if (e <= R) best = min(best, min(cand16(at(Z - e), e * e), cand16(at(Z + e), e * e)));
                        }
                    }
                    out = phi_value(seed, best, R2, vs, dmax);
                }
                job.phi[(int64_t)idx * 512 + tid] = out;
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Per-line passes: lower envelope of parabolas (Felzenszwalb and
// Huttenlocher, edt_envelope.h).  One wave per block column; lane = one
// line.  A line longer than kWin voxels is cut into output segments that each
// carry C = 8 HB >= R voxels of context on both sides, which is exact because
// only k <= R^2 is kept.  Work per voxel is a few LDS steps whatever the
// distances, which suits large domains with many lines.

__device__ __forceinline__ void segment(int L, int C, int seg, int S, int &y0, int &y1, int &w0, int &w1)
{
    y0 = seg * S;
    y1 = min(y0 + S, L);
    w0 = max(0, y0 - C);
    w1 = min(L, y1 + C);
}

// Lane = x + 8 z within the block column (bx, *, bz).
template <int NJ>
__global__ __launch_bounds__(64) void k_edt_y_env(const JobList<NJ> jl, const uint8_t *__restrict__ g1,
                                                  uint16_t *__restrict__ g2, int R, int HB)
{
    __shared__ Plan lds;
    __shared__ __align__(16) uint8_t col[kWin * 64];   // [position][lane]
    __shared__ __align__(16) uint8_t stk[kWin * 64];   // [entry][lane]
    __shared__ __align__(16) uint16_t ost[8 * 64];     // one block of outputs [y][lane]
    const int C = 8 * HB;
    PlanView<NJ> pv;
    pv.init(jl, C, lds);
    const int lane = threadIdx.x;
    const int Sg = kWin - 2 * C;
    const int R2 = R * R;
    auto getf = [&](int q) {
        const int a = col[q * 64 + lane];
        return a * a;
    };
    for (int64_t c = blockIdx.x; c < pv.t[2]; c += gridDim.x) {
        const JobInfo d = pv.info(pv.template job<&JobInfo::oy>(c));
        const int L = 8 * d.dim[1];
        const int nseg = (int)nsegments(L, Sg);
        const int64_t cl = c - d.oy;
        const int seg = (int)(cl % nseg);
        const int64_t cc = cl / nseg;
        const int bx = (int)(cc % d.dim[0]), bz = (int)(cc / d.dim[0]);
        int y0, y1, w0, w1;
        segment(L, C, seg, Sg, y0, y1, w0, w1);
        for (int j = w0 / 8; j < w1 / 8; ++j) {
            const int64_t g = d.od + dom_index(d, bx, j, bz);
            const uint64_t v = ((const uint64_t *)(g1 + g * 512))[lane];
            *(uint64_t *)&col[(8 * (j - w0 / 8) + (lane & 7)) * 64 + 8 * (lane >> 3)] = v;
        }
        wave_sync();
        Envelope e;
        env_clear(e);
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
            const int64_t g = d.od + dom_index(d, bx, yb / 8, bz);
            const uint4 o = *(const uint4 *)&ost[(lane & 7) * 64 + 8 * (lane >> 3)];
            *(uint4 *)(g2 + g * 512 + 8 * lane) = o;
            wave_sync();
        }
    }
}

// Lane = x + 8 y, the in-block layout, within the column (bx, by, *).
template <int NJ>
__global__ __launch_bounds__(64) void k_edt_z_env(const JobList<NJ> jl, const uint16_t *__restrict__ g2, int R,
                                                  int HB, float vs, float dmax)
{
    __shared__ Plan lds;
    __shared__ __align__(16) uint16_t col[kWin * 64];  // [position][lane]
    __shared__ __align__(16) uint8_t stk[kWin * 64];
    const int C = 8 * HB;
    PlanView<NJ> pv;
    pv.init(jl, C, lds);
    const int lane = threadIdx.x;
    const int Sg = kWin - 2 * C;
    const int R2 = R * R;
    auto getf = [&](int q) { return (int)col[q * 64 + lane]; };
    for (int64_t c = blockIdx.x; c < pv.t[3]; c += gridDim.x) {
        const int jj = pv.template job<&JobInfo::oz>(c);
        const JobInfo d = pv.info(jj);
        const EsdfJob &job = jl.j[jj];
        const int L = 8 * d.dim[2];
        const int nseg = (int)nsegments(L, Sg);
        const int64_t cl = c - d.oz;
        const int seg = (int)(cl % nseg);
        const int64_t cc = cl / nseg;
        const int bx = (int)(cc % d.dim[0]), by = (int)(cc / d.dim[0]);
        int z0, z1, w0, w1;
        segment(L, C, seg, Sg, z0, z1, w0, w1);
        // nothing to write when no block of the output range is allocated
        bool any = false;
        for (int j0 = z0 / 8; j0 < z1 / 8; j0 += 64) {
            const int j = j0 + lane;
            const bool a = j < z1 / 8 && job.page[dom_index(d, bx, by, j)] >= 0;
            any = any || __ballot(a) != 0;
        }
        if (!any) continue;
        for (int j = w0 / 8; j < w1 / 8; ++j) {
            const uint16_t *src = g2 + (d.od + dom_index(d, bx, by, j)) * 512 + lane;
#pragma unroll
            for (int t = 0; t < 8; ++t) col[(8 * (j - w0 / 8) + t) * 64 + lane] = src[64 * t];
        }
        wave_sync();
        Envelope e;
        env_clear(e);
        const int Wn = w1 - w0;
        for (int q = 0; q < Wn; ++q) {
            const int a = col[q * 64 + lane];
            if (a == 0xFFFF) continue;
            env_push(e, stk, 64, lane, q, a, getf);
        }
        Walker wk;
        if (e.k >= 0) walk_init(wk, e, stk, 64, lane, getf);
        for (int zb = z0; zb < z1; zb += 8) {
            const int64_t idx = job.page[dom_index(d, bx, by, zb / 8)];
            if (idx < 0) continue;
            const float *Sb = job.seeds + (d.od + dom_index(d, bx, by, zb / 8)) * 512 + lane;
            float *Pb = job.phi + idx * 512 + lane;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float seed = Sb[64 * t];  // from k_page_sites
                float out = seed;  // unobserved or in the band
                if (__builtin_isinf(seed)) {
                    const int best = e.k >= 0 ? walk_at(wk, e, stk, 64, lane, zb + t - w0, getf) : kBig;
                    out = phi_value(seed, best, R2, vs, dmax);
                }
                Pb[64 * t] = out;
            }
        }
        wave_sync();
    }
}

// Every ESDF kernel loops over its work items with a grid stride, so the
// grid only needs to fill the chip: the host's bounds on the dense domain
// and the block count are loose, and surplus workgroups would each pay
// their dispatch and set-up for nothing.  2048 workgroups of up to 512
// lanes keep 256 CUs busy.
unsigned clamp_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 2048)); }
// The passes loop over their work with a grid stride, so a smaller grid is
// valid; while they run beside an integration (on their own stream), the
// tuning's cap leaves CUs to it.
unsigned cap_grid(const covox_ctx *ctx, unsigned g)
{
    const int64_t cap = ctx->tune.edt_pipe_max_workgroups;
    return ctx->esdf_edt_stream && cap > 0 ? (unsigned)std::min<int64_t>(g, cap) : g;
}
// Single-wave workgroups (per-line envelopes): up to 64 waves per CU.
unsigned clamp_grid_w(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, 16384)); }

int64_t bound_blocks(const covox_submap *s)
{
    if (!s->bound_valid) return 0;
    int64_t n = 1;
    for (int a = 0; a < 3; ++a) n *= (int64_t)(s->bound_hi[a] - s->bound_lo[a] + 1);
    return n;
}

// Columns (times segments) of a line pass over the host-side bound box:
// axes a and b span the columns, the third axis is the line.
int64_t bound_cols(const covox_submap *s, int a, int b, int HB)
{
    if (!s->bound_valid) return 0;
    const int c = 3 - a - b;
    const int64_t L = 8 * (int64_t)(s->bound_hi[c] - s->bound_lo[c] + 1);
    const int64_t S = kWin - 16 * HB;
    return (int64_t)(s->bound_hi[a] - s->bound_lo[a] + 1) * (s->bound_hi[b] - s->bound_lo[b] + 1) * ((L + S - 1) / S);
}

template <int NJ>
JobList<NJ> make_jobs(covox_submap *const *subs, int n, EsdfSnap *snap, float *seeds, bool partial)
{
    JobList<NJ> jl;
    memset(&jl, 0, sizeof(jl));
    jl.n = n;
    for (int i = 0; i < n; ++i) {
        covox_submap *s = subs[i];
        jl.j[i] = EsdfJob{s->meta, snap + i, s->keys, s->tkeys, s->tvals, (uint64_t)s->tcap - 1, s->D, s->W,
                          s->phi, s->page, seeds, s->dirty, (partial && s->esdf_exact) ? 0 : 1};
    }
    return jl;
}

// Page + site masks (and, with edt, the three EDT passes) for up to NJ
// submaps in one launch per kernel.
// Line segments of the y and z passes over the host bounds of the submaps.
void chunk_cols(covox_submap *const *subs, int n, int HB, int64_t &cy, int64_t &cz)
{
    cy = cz = 0;
    for (int i = 0; i < n; ++i) {
        cy += bound_cols(subs[i], 0, 2, HB);
        cz += bound_cols(subs[i], 0, 1, HB);
    }
}

// Column segments along axis `c` (columns spanned by the other two axes) of
// the column passes over the host-side bound box.
int64_t bound_segs(const covox_submap *s, int c, int S)
{
    if (!s->bound_valid) return 0;
    int64_t cols = 1;
    for (int a = 0; a < 3; ++a)
        if (a != c) cols *= (int64_t)(s->bound_hi[a] - s->bound_lo[a] + 1);
    const int64_t L = s->bound_hi[c] - s->bound_lo[c] + 1;
    return cols * ((L + S - 1) / S);
}

// Segment length of the column passes for halo HB (0: per-block passes).
int col_segment(const covox_ctx *ctx, int HB)
{
    const int64_t S = ctx->tune.edt_col_seg;
    if (S <= 0) return 0;
    return (int)std::max<int64_t>(1, std::min<int64_t>(S, kColMaxStage - 2 * HB));
}

// force < 0: pass layout and shapes by the tuning (or COVOX_EDT_MODE); else
// the per-block passes with bit 0 = y envelopes, bit 1 = z envelopes.
template <int NJ>
int esdf_chunk(covox_ctx *ctx, covox_submap *const *subs, int n, bool edt, int force = -1)
{
    const covox_params &p = ctx->p;
    const int R = (int)std::llround(p.d_max / p.voxel_size);
    const int HB = (R + 7) / 8;
    const int C = 8 * HB;
    int rc;
    // The page kernel runs on the context stream; the passes after it run
    // on ctx->esdf_edt_stream when a pipelined caller sets one (after
    // ev_paged, so that the caller may integrate meanwhile), else on the
    // context stream too.
    hipStream_t edt_stream = ctx->esdf_edt_stream ? ctx->esdf_edt_stream : ctx->stream;
    const int slot = ctx->esdf_slot;
    int64_t nd = 0, nb = 0, cy = 0, cz = 0;
    for (int i = 0; i < n; ++i) {
        covox_submap *s = subs[i];
        nd += std::max<int64_t>(bound_blocks(s), 1);
        nb += std::min(s->nb_upper, s->cap);
    }
    chunk_cols(subs, n, HB, cy, cz);
    const int Sseg = force >= 0 ? 0 : col_segment(ctx, HB);
    const bool cols = edt && Sseg > 0;
    // a partial update (column passes only, never under capture): the
    // submaps whose phi is exact and whose changes since are all flagged
    bool partial = cols && !ctx->capturing && !ctx->tune.esdf_full_recompute;
    if (partial) {
        bool any = false;
        for (int i = 0; i < n; ++i) any = any || subs[i]->esdf_exact;
        partial = any;
    }
    // a buffer that grows is freed: the passes of an earlier update on the
    // other stream may still read it
    bool grows = ctx->sites_cap[slot] < nd ||
                 (edt && (ctx->seeds_cap[slot] < nd || (!cols && ctx->g1_cap < nd) || ctx->g2_cap < nd)) ||
                 (cols && ctx->blk_cap[slot] < nd) || (partial && ctx->ddirty_cap[slot] < 2 * nd);
    for (int i = 0; i < n; ++i) grows = grows || subs[i]->page_cap < std::max<int64_t>(bound_blocks(subs[i]), 1);
    if (grows && edt_stream != ctx->stream && !ctx->capturing &&
        (rc = hip_check(ctx, hipStreamSynchronize(edt_stream), "esdf stream sync")))
        return rc;
    for (int i = 0; i < n; ++i) {
        covox_submap *s = subs[i];
        const int64_t b = std::max<int64_t>(bound_blocks(s), 1);
        if ((rc = ensure_buffer(ctx, (void **)&s->page, &s->page_cap, b, sizeof(int32_t), "page"))) return rc;
    }
    if ((rc = ensure_buffer(ctx, (void **)&ctx->sites[slot], &ctx->sites_cap[slot], nd, 8 * sizeof(uint64_t),
                            "site masks")))
        return rc;
    if (!ctx->snap[slot] && (rc = hip_check(ctx, hipMalloc((void **)&ctx->snap[slot], sizeof(EsdfSnap) * kMaxJobs),
                                            "esdf snapshot")))
        return rc;
    if (edt) {
        if ((rc = ensure_buffer(ctx, (void **)&ctx->seeds[slot], &ctx->seeds_cap[slot], nd, 512 * sizeof(float),
                                "phi seeds")))
            return rc;
        if (!cols && (rc = ensure_buffer(ctx, (void **)&ctx->g1, &ctx->g1_cap, nd, 512, "edt g1"))) return rc;
        if ((rc = ensure_buffer(ctx, (void **)&ctx->g2, &ctx->g2_cap, nd, 1024, "edt g2"))) return rc;
    }
    if (cols && (rc = ensure_buffer(ctx, (void **)&ctx->blk[slot], &ctx->blk_cap[slot], nd, sizeof(int32_t),
                                    "esdf block index")))
        return rc;
    int32_t *const blk = cols ? ctx->blk[slot] : nullptr;
    if (partial && (rc = ensure_buffer(ctx, (void **)&ctx->ddirty[slot], &ctx->ddirty_cap[slot], 2 * nd, 1,
                                       "esdf change flags")))
        return rc;
    uint8_t *const ddirty = partial ? ctx->ddirty[slot] : nullptr;
    uint64_t *const sites = ctx->sites[slot];
    const JobList<NJ> jl = make_jobs<NJ>(subs, n, ctx->snap[slot], ctx->seeds[slot], partial);
    const float vs = (float)p.voxel_size, tau = (float)band_limit(p), dmax = (float)p.d_max;
    const bool h = p.precision == COVOX_FP16;
    {
        TimedLaunch tl(ctx, COVOX_K_ESDF_PAGE);
        const dim3 grid(clamp_grid(std::max((nd + 255) / 256, (nb + 3) / 4)));
        if (h && edt)
            hipLaunchKernelGGL((k_page_sites<__half, NJ, true>), grid, dim3(256), 0, ctx->stream, jl, C, vs, tau,
                               sites, blk, ddirty);
        else if (h)
            hipLaunchKernelGGL((k_page_sites<__half, NJ, false>), grid, dim3(256), 0, ctx->stream, jl, C, vs, tau,
                               sites, blk, ddirty);
        else if (edt)
            hipLaunchKernelGGL((k_page_sites<float, NJ, true>), grid, dim3(256), 0, ctx->stream, jl, C, vs, tau,
                               sites, blk, ddirty);
        else
            hipLaunchKernelGGL((k_page_sites<float, NJ, false>), grid, dim3(256), 0, ctx->stream, jl, C, vs, tau,
                               sites, blk, ddirty);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "page launch"))) return rc;
    for (int i = 0; i < n; ++i) subs[i]->page_version = subs[i]->version;
    if (!edt) return COVOX_OK;
    // Pass shape: per-line envelopes when there are enough lines to fill the
    // GPU, voxel-parallel windowed search otherwise (or as forced by
    // COVOX_EDT_MODE = window | envelope).
    bool env_y = cy >= ctx->tune.edt_y_env_min_cols, env_z = cz >= ctx->tune.edt_z_env_min_cols;
    if (ctx->edt_mode == 1) env_y = env_z = false;
    if (ctx->edt_mode == 2) env_y = env_z = true;
    if (force >= 0) {
        env_y = (force & 1) != 0;
        env_z = (force & 2) != 0;
    }
    ctx->esdf_used_page = !cols && env_z;  // the z envelopes read the page
    // the passes read nothing the next integration writes: on their own
    // stream they wait for the page kernel only
    hipStream_t base = ctx->stream;
    if (edt_stream != base) {
        if ((rc = hip_check(ctx, hipEventRecord(ctx->ev_paged, base), "paged")) ||
            (rc = hip_check(ctx, hipStreamWaitEvent(edt_stream, ctx->ev_paged, 0), "paged wait")))
            return rc;
        ctx->stream = edt_stream;  // for the launches and their timing events below
    }
    if (cols) {
        if (partial) {
            const unsigned gd = cap_grid(ctx, clamp_grid((nd + 255) / 256));
            hipLaunchKernelGGL((k_esdf_dil_x<NJ>), dim3(gd), dim3(256), 0, ctx->stream, jl, HB, ddirty, ddirty + nd);
            hipLaunchKernelGGL((k_esdf_region<NJ>), dim3(gd), dim3(256), 0, ctx->stream, jl, HB, ddirty + nd, blk);
        }
        int64_t sy = 0, sz = 0;
        for (int i = 0; i < n; ++i) {
            sy += std::max<int64_t>(bound_segs(subs[i], 1, Sseg), 1);
            sz += std::max<int64_t>(bound_segs(subs[i], 2, Sseg), 1);
        }
        {
            TimedLaunch tl(ctx, COVOX_K_EDT_Y);
            hipLaunchKernelGGL((k_edt_xy<NJ>), dim3(cap_grid(ctx, clamp_grid(sy))), dim3(256), 0, ctx->stream, jl, Sseg,
                               sites, blk, ctx->g2, R, HB);
        }
        {
            TimedLaunch tl(ctx, COVOX_K_EDT_Z);
            hipLaunchKernelGGL((k_edt_z_col<NJ>), dim3(cap_grid(ctx, clamp_grid(sz))), dim3(512), 0, ctx->stream, jl,
                               Sseg, ctx->g2, blk, R, HB, vs, dmax);
        }
        ctx->stream = base;
        if ((rc = hip_check(ctx, hipGetLastError(), "esdf launch"))) return rc;
        for (int i = 0; i < n; ++i) {
            subs[i]->esdf_version = subs[i]->version;
            if (!ctx->capturing) subs[i]->esdf_exact = true;
        }
        return COVOX_OK;
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_X);
        hipLaunchKernelGGL((k_edt_x<NJ>), dim3(cap_grid(ctx, clamp_grid((nd + 3) / 4))), dim3(256), 0, ctx->stream, jl, sites,
                           ctx->g1, R, HB);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Y);
        if (env_y)
            hipLaunchKernelGGL((k_edt_y_env<NJ>), dim3(clamp_grid_w(cy)), dim3(64), 0, ctx->stream, jl, ctx->g1, ctx->g2,
                               R, HB);
        else
            hipLaunchKernelGGL((k_edt_y_col<NJ>), dim3(cap_grid(ctx, clamp_grid(nd))), dim3(256), 0, ctx->stream, jl, ctx->g1,
                               ctx->g2, R, HB);
    }
    {
        TimedLaunch tl(ctx, COVOX_K_EDT_Z);
        if (env_z)
            hipLaunchKernelGGL((k_edt_z_env<NJ>), dim3(clamp_grid_w(cz)), dim3(64), 0, ctx->stream, jl, ctx->g2, R, HB,
                               vs, dmax);
        else
            hipLaunchKernelGGL((k_edt_z_vox<NJ>), dim3(cap_grid(ctx, clamp_grid(nb))), dim3(512), 0, ctx->stream, jl, ctx->g2, R, HB,
                               vs, dmax);
    }
    ctx->stream = base;
    if ((rc = hip_check(ctx, hipGetLastError(), "esdf launch"))) return rc;
    for (int i = 0; i < n; ++i) {
        subs[i]->esdf_version = subs[i]->version;
        if (!ctx->capturing) subs[i]->esdf_exact = true;
    }
    return COVOX_OK;
}

}  // namespace

int build_page(covox_ctx *ctx, covox_submap *s)
{
    if (s->page_version == s->version) return COVOX_OK;
    return esdf_chunk<1>(ctx, &s, 1, false);
}

int update_esdf_batch(covox_ctx *ctx, covox_submap *const *subs, int n)
{
    std::vector<covox_submap *> todo;
    for (int i = 0; i < n; ++i)
        if (std::find(todo.begin(), todo.end(), subs[i]) == todo.end()) todo.push_back(subs[i]);
    if (todo.empty()) return COVOX_OK;
    if (ctx->p.esdf_mode == COVOX_ESDF_WAVEFRONT) {
        for (covox_submap *s : todo) {
            const int rc = update_esdf_wavefront(ctx, s);
            if (rc) return rc;
        }
        return COVOX_OK;
    }
    if (todo.size() == 1) return esdf_chunk<1>(ctx, todo.data(), 1, true);
    for (size_t i = 0; i < todo.size(); i += kMaxJobs) {
        const int m = (int)std::min<size_t>(kMaxJobs, todo.size() - i);
        const int rc = esdf_chunk<kMaxJobs>(ctx, todo.data() + i, m, true);
        if (rc) return rc;
    }
    return COVOX_OK;
}

int update_esdf(covox_ctx *ctx, covox_submap *s) { return update_esdf_batch(ctx, &s, 1); }

int autotune_esdf(covox_ctx *ctx, covox_submap *const *subs, int n)
{
    std::vector<covox_submap *> todo;
    for (int i = 0; i < n && (int)todo.size() < kMaxJobs; ++i)
        if (std::find(todo.begin(), todo.end(), subs[i]) == todo.end()) todo.push_back(subs[i]);
    if (todo.empty()) return COVOX_OK;
    const int m = (int)todo.size();
    const int R = (int)std::llround(ctx->p.d_max / ctx->p.voxel_size);
    int64_t cy, cz;
    chunk_cols(todo.data(), m, (R + 7) / 8, cy, cz);
    auto run = [&](int force) {
        return m == 1 ? esdf_chunk<1>(ctx, todo.data(), 1, true, force)
                      : esdf_chunk<kMaxJobs>(ctx, todo.data(), m, true, force);
    };
    hipEvent_t e0, e1;
    int rc = hip_check(ctx, hipEventCreate(&e0), "autotune event");
    if (rc) return rc;
    if ((rc = hip_check(ctx, hipEventCreate(&e1), "autotune event"))) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    const int32_t saved_timing = ctx->timing;
    ctx->timing = 0;  // no per-kernel events inside the measured region
    covox_tuning &t = ctx->tune;
    const int64_t saved_seg = t.edt_col_seg, saved_full = t.esdf_full_recompute;
    t.esdf_full_recompute = 1;  // every candidate times a whole update
    // candidates: the four shapes of the per-block passes, then the column
    // passes at five segment lengths
    constexpr int kSegs[5] = {2, 4, 8, 16, 32};
    constexpr int kCand = 4 + 5;
    float best_ms[kCand];
    for (int cand = 0; cand < kCand && !rc; ++cand) {
        best_ms[cand] = 1e30f;
        const int force = cand < 4 ? cand : -1;
        if (cand >= 4) t.edt_col_seg = kSegs[cand - 4];
        rc = run(force);  // warm-up (buffers, caches)
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            rc = hip_check(ctx, hipEventRecord(e0, ctx->stream), "autotune record");
            if (!rc) rc = run(force);
            if (!rc) rc = hip_check(ctx, hipEventRecord(e1, ctx->stream), "autotune record");
            if (!rc) rc = hip_check(ctx, hipEventSynchronize(e1), "autotune sync");
            float ms = 0;
            if (!rc) rc = hip_check(ctx, hipEventElapsedTime(&ms, e0, e1), "autotune elapsed");
            if (!rc) best_ms[cand] = std::min(best_ms[cand], ms);
        }
    }
    t.edt_col_seg = saved_seg;
    t.esdf_full_recompute = saved_full;
    ctx->timing = saved_timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    int best = 0;
    for (int c = 1; c < kCand; ++c)
        if (best_ms[c] < best_ms[best]) best = c;
    if (best >= 4) {
        t.edt_col_seg = kSegs[best - 4];
        return COVOX_OK;
    }
    t.edt_col_seg = 0;
    if (best & 1) t.edt_y_env_min_cols = std::min(t.edt_y_env_min_cols, cy);
    else t.edt_y_env_min_cols = std::max(t.edt_y_env_min_cols, cy + 1);
    if (best & 2) t.edt_z_env_min_cols = std::min(t.edt_z_env_min_cols, cz);
    else t.edt_z_env_min_cols = std::max(t.edt_z_env_min_cols, cz + 1);
    return COVOX_OK;
}

}  // namespace covox
