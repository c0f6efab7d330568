// Internal declarations of the covox HIP library (gfx950).  Not installed;
// the public interface is include/covox.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/covox.h"

namespace covox {

// ------------------------------------------------------------------ keys

constexpr int64_t kKeyOff = 1 << 20;
constexpr uint64_t kEmpty = ~0ull;   // empty hash slot
constexpr int kMaxHalo = 7;          // halo blocks of the EDT passes (R <= 56)

__host__ __device__ inline uint64_t pack_key(int32_t bx, int32_t by, int32_t bz)
{
    return ((uint64_t)(int64_t)(bx + kKeyOff) << 42) | ((uint64_t)(int64_t)(by + kKeyOff) << 21) |
           (uint64_t)(int64_t)(bz + kKeyOff);
}

__host__ __device__ inline void unpack_key(uint64_t k, int32_t &bx, int32_t &by, int32_t &bz)
{
    bx = (int32_t)((k >> 42) & 0x1FFFFF) - (int32_t)kKeyOff;
    by = (int32_t)((k >> 21) & 0x1FFFFF) - (int32_t)kKeyOff;
    bz = (int32_t)(k & 0x1FFFFF) - (int32_t)kKeyOff;
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014): the home bucket
// of a key is mix64(key) & (capacity - 1).
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Lookup in an open-addressing table with linear probing.  The table is
// never more than 85 % full, so the probe ends at the key or an empty slot.
__device__ inline int64_t hash_find(const uint64_t *tkeys, const uint32_t *tvals, uint64_t mask,
                                    uint64_t key)
{
    uint64_t h = mix64(key) & mask;
    for (;;) {
        uint64_t k = tkeys[h];
        if (k == key) return (int64_t)tvals[h];
        if (k == kEmpty) return -1;
        h = (h + 1) & mask;
    }
}

// The same lookup in two steps: hash_first reads the home slot (key and
// value), hash_resolve finishes the lookup, probing on only when the home
// slot holds another key.  Other reads can be in flight in between.
struct HashProbe {
    uint64_t h, k;
    uint32_t v;
};

__device__ inline HashProbe hash_first(const uint64_t *tkeys, const uint32_t *tvals, uint64_t mask, uint64_t key)
{
    HashProbe p;
    p.h = mix64(key) & mask;
    p.k = tkeys[p.h];
    p.v = tvals[p.h];
    return p;
}

__device__ inline int64_t hash_resolve(const HashProbe &p, const uint64_t *tkeys, const uint32_t *tvals,
                                       uint64_t mask, uint64_t key)
{
    if (p.k == key) return (int64_t)p.v;
    if (p.k == kEmpty) return -1;
    for (uint64_t h = (p.h + 1) & mask;; h = (h + 1) & mask) {
        const uint64_t k = tkeys[h];
        if (k == key) return (int64_t)tvals[h];
        if (k == kEmpty) return -1;
    }
}

// Inserts a key known to be absent ("activate": the caller already owns
// its buffer index).
__device__ inline void hash_insert(uint64_t *tkeys, uint32_t *tvals, uint64_t mask, uint64_t key,
                                   uint32_t val)
{
    uint64_t h = mix64(key) & mask;
    for (;;) {
        unsigned long long prev = atomicCAS((unsigned long long *)&tkeys[h], (unsigned long long)kEmpty,
                                            (unsigned long long)key);
        if (prev == kEmpty) {
            tvals[h] = val;
            return;
        }
        h = (h + 1) & mask;
    }
}

// The same insertion (home slot, probe order, compare-and-swap) with the
// probe bounded by `limit` slots, for tables that the caller owns and may
// have filled: returns the number of slots probed past the home slot, or -1
// when `limit` slots were occupied.
__device__ inline int64_t hash_insert_bounded(uint64_t *tkeys, uint32_t *tvals, uint64_t mask, uint64_t key,
                                              uint32_t val, uint64_t limit)
{
    uint64_t h = mix64(key) & mask;
    for (uint64_t step = 0; step < limit; ++step) {
        unsigned long long prev = atomicCAS((unsigned long long *)&tkeys[h], (unsigned long long)kEmpty,
                                            (unsigned long long)key);
        if (prev == kEmpty) {
            tvals[h] = val;
            return (int64_t)step;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

// ----------------------------------------------------------- submap state

// Device-resident bookkeeping of one submap.
struct SubmapMeta {
    int64_t n_blocks;       // allocated blocks
    int32_t bmin[3];        // allocated block box (inclusive); valid when n_blocks > 0
    int32_t bmax[3];
    int32_t status;         // sticky capacity error of an asynchronous integration
    int32_t n_new;          // last frame: new blocks
    int32_t n_touched;      // last frame: touched blocks
    int32_t dom_valid;      // page below describes dom_min / dom_dim
    int32_t dom_min[3];     // ESDF / page domain (block coordinates)
    int32_t dom_dim[3];
    int64_t n_points;       // registration points
    double pbar[3];         // their centroid (binary64)
    unsigned long long n_updates;  // voxel updates since creation / reset
    int64_t batch_n0;       // last frame batch: n_blocks before it
    int32_t batch_frames;   // and its frames committed (a capacity failure stops the batch)
    int32_t dom_nblocks;    // allocated blocks when the page was built
};

// The domain one ESDF update works on (block box and allocated block
// count), stored by the page kernel and read by the passes after it.
struct EsdfSnap {
    int32_t lo[3], dim[3];
    int32_t nb, pad;
};
constexpr int kEsdfMaxJobs = 32;  // submaps per ESDF launch

// Per-frame projection parameters (kernel argument).
struct FrameArgs {
    float R[9];
    float t[3];
    float K[4];
    int32_t H, W;
    int32_t blo[3];    // frustum block box origin
    int32_t bdim[3];   // and extent (z fastest in the linear order)
    const float *depth;
    // Conservative block cull (camera frame): unit normals of the four side
    // planes of the image widened by one pixel, the far limit max_range +
    // tau, and the radius of a block's voxel centres about its centre
    // (inflated against rounding).
    float plane[4][3];
    float zfar;
    float cull_r;
    int32_t weight_mode;  // COVOX_WEIGHT_*
    // Raycasting: submap <- camera rotation and the optical centre in the
    // submap frame (binary64 rounded once), and whether rays start there.
    float Rs[9];
    float o[3];
    int32_t ray_carve;
};

}  // namespace covox

struct covox_submap {
    covox_ctx *ctx = nullptr;
    double T_ws[16];
    int64_t cap = 0;         // block capacity
    int64_t tcap = 0;        // hash slots (power of two)
    uint64_t *keys = nullptr;
    void *D = nullptr;       // float or __half, cap * 512
    void *W = nullptr;
    float *phi = nullptr;
    uint64_t *tkeys = nullptr;
    uint32_t *tvals = nullptr;
    covox::SubmapMeta *meta = nullptr;
    // host-side upper bounds (no device round trip needed)
    int64_t nb_upper = 0;            // >= n_blocks
    // The scan kernels store (sequence << 40) | n_blocks into pinned host
    // memory after each integration call; with the box sizes of the calls
    // enqueued since, it tightens nb_upper without a device round trip.
    volatile uint64_t *pin_nb = nullptr;
    uint64_t *pin_nb_dev = nullptr;  // its device address
    uint64_t seq = 0;                // integration calls enqueued
    static constexpr int kSeqRing = 256;
    int64_t box_ring[kSeqRing] = {};  // box sizes of the last calls, by sequence
    uint32_t *stamp = nullptr;       // per block: id of the last frame batch that listed it
    // per block: 1 once an integration has changed it since the last exact
    // ESDF update (cleared by that update's page kernel); cap bytes, padded
    uint8_t *dirty = nullptr;
    // the submap's phi is the exact ESDF of its TSDF at the last exact update,
    // and the dirty flags cover every change since (else the next exact update
    // recomputes everything)
    bool esdf_exact = false;
    uint32_t batch_id = 0;
    bool bound_valid = false;        // box containing every allocated block
    int32_t bound_lo[3] = {0, 0, 0};
    int32_t bound_hi[3] = {0, 0, 0};
    // dense block page of the bounding box (ESDF, points, alignment field)
    int32_t *page = nullptr;
    int64_t page_cap = 0;
    uint64_t version = 1;            // bumped by every state change
    uint64_t page_version = 0;       // version the page was built from
    uint64_t esdf_version = 0;
    // registration points
    float *pts = nullptr;
    int64_t pts_cap = 0;
    uint64_t pts_version = 0;
    int64_t n_pts = 0;
    double pbar[3] = {0, 0, 0};
    // wavefront ESDF state (esdf_mode COVOX_ESDF_WAVEFRONT): squared distance
    // and packed parent offset per voxel, blocks at the last update (device)
    int32_t *wf_k = nullptr;
    int32_t *wf_p = nullptr;
    int64_t *wf_wn = nullptr;
};

namespace covox {

// Host bookkeeping of a submap (what a graph capture saves and restores).
struct SubmapSnap {
    int64_t nb_upper;
    bool bound_valid;
    int32_t bound_lo[3], bound_hi[3];
    uint64_t version, page_version, esdf_version, pts_version;
    int64_t n_pts;
};

// A submap used by a graph under capture.
struct CaptureEntry {
    covox_submap *s;
    SubmapSnap start, end;
    bool reset_first;  // the first captured operation on it was a reset
    bool integrated;
};

// A submap and its version when an alignment set was prepared.
struct AlignFrozen {
    const covox_submap *s;
    uint64_t version;
};

}  // namespace covox

struct covox_graph {
    covox_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<covox::CaptureEntry> subs;
    std::vector<void *> host_bufs;          // pinned sources of captured copies
    std::vector<covox::AlignFrozen> frozen;  // submaps that captured alignment sets read
};

struct covox_ctx {
    covox_params p;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    std::vector<covox_submap *> subs;  // live submaps of this context
    std::vector<covox_net *> nets;     // live networks of this context (detached by covox_destroy)
    // integration scratch
    uint32_t *cand = nullptr;
    int64_t cand_cap = 0;
    uint64_t *t_key = nullptr;
    int64_t t_key_cap = 0;
    uint32_t *t_idx = nullptr;
    int64_t t_idx_cap = 0;
    double *ray_acc = nullptr;  // raycasting: (sum w, sum t w) per voxel, zero between frames
    int64_t ray_acc_blocks = 0;
    // wavefront ESDF scratch: next-round state, site masks, queue flags and list
    int32_t *wf_nk = nullptr, *wf_np = nullptr;
    int64_t wf_nk_cap = 0, wf_np_cap = 0;
    uint64_t *wf_sites = nullptr;
    int64_t wf_sites_cap = 0;
    uint32_t *wf_flag = nullptr;
    int64_t wf_flag_cap = 0;
    int32_t *wf_list = nullptr;
    int64_t wf_list_cap = 0;
    int64_t *wf_cnt = nullptr;  // [queue size of the last list, block-rounds]
    int64_t wf_cnt_cap = 0;
    int64_t *wf_pin = nullptr;  // pinned copy of wf_cnt
    int64_t wf_last_block_rounds = 0;
    // EDT scratch over a dense block box
    // ESDF scratch written by the page kernel, in two slots: a pipelined
    // map_sequence builds the page of frame k + 1 while the passes of frame
    // k still read slot k mod 2
    uint64_t *sites[2] = {nullptr, nullptr};  // 8 words per dense block
    int64_t sites_cap[2] = {0, 0};            // dense blocks
    float *seeds[2] = {nullptr, nullptr};     // phi seed per voxel of the dense blocks
    int64_t seeds_cap[2] = {0, 0};            // dense blocks
    int32_t *blk[2] = {nullptr, nullptr};     // buffer index per dense block (column passes)
    int64_t blk_cap[2] = {0, 0};              // dense blocks
    uint8_t *ddirty[2] = {nullptr, nullptr};  // dirty flag per dense block, then its dilation along x
    int64_t ddirty_cap[2] = {0, 0};           // dense blocks (two arrays)
    covox::EsdfSnap *snap[2] = {nullptr, nullptr};  // kEsdfMaxJobs per slot
    int esdf_slot = 0;
    uint8_t *g1 = nullptr;      // 512 per dense block
    int64_t g1_cap = 0;
    uint16_t *g2 = nullptr;     // 512 per dense block
    int64_t g2_cap = 0;
    int32_t edt_mode = 0;           // 0 by the tuning below, 1 voxel-parallel window, 2 per-line envelope
    covox_tuning tune;              // per-pass shape thresholds (covox_default_tuning, covox_autotune_esdf)
    // registration-point scratch
    uint32_t *cnt = nullptr;    // per-block counts, then offsets
    int64_t cnt_cap = 0;
    double *psum = nullptr;     // per-block point sums
    int64_t psum_cap = 0;
    // alignment scratch
    void *prob_dev = nullptr;
    int64_t prob_cap = 0;
    void *res_dev = nullptr;
    int64_t res_cap = 0;
    void *sum_dev = nullptr;     // summary requests
    int64_t sum_cap = 0;
    float *net_in = nullptr;     // learned alignment: summaries and network outputs
    int64_t net_in_cap = 0;
    float *net_out = nullptr;
    int64_t net_out_cap = 0;
    covox::FrameArgs *frames_dev = nullptr;  // frame batch parameters
    int64_t frames_cap = 0;
    covox::FrameArgs *frames_pin[2] = {nullptr, nullptr};  // pinned staging, alternating
    hipEvent_t frames_ev[2] = {nullptr, nullptr};          // their uploads
    int frames_slot = 0;
    uint32_t *blist = nullptr;        // frame batch: blocks to update
    int64_t blist_cap = 0;
    uint64_t *fkeys = nullptr;        // frame batch: first frame of each new key (temporary table)
    int64_t fkeys_cap = 0;
    uint32_t *ffirst = nullptr;
    int64_t ffirst_cap = 0;
    int64_t *fcount = nullptr;        // frame batch: new blocks per frame, then frame offsets
    int64_t fcount_cap = 0;
    float *train_y = nullptr;    // proposal training: targets and per-step losses
    int64_t train_y_cap = 0;
    float *loss_hist = nullptr;
    int64_t loss_hist_cap = 0;
    // pinned host staging for small copies
    void *host_pin = nullptr;
    size_t host_pin_cap = 0;
    // map_sequence: the page kernel of each update runs on the context
    // stream right after the integration it reads; the EDT passes run on
    // esdf_stream (set as esdf_edt_stream for the duration), after
    // ev_paged, while the next chunk integrates.  ev_free[slot] follows the
    // passes of the last update that used the slot.
    hipStream_t esdf_stream = nullptr;
    hipStream_t esdf_edt_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_paged = nullptr, ev_join = nullptr;
    hipEvent_t ev_free[2] = {nullptr, nullptr};
    bool esdf_used_page = false;  // the last update's passes read the page (z envelopes)
    // graph capture (on a stream of the library: the legacy default stream
    // cannot be captured)
    hipStream_t cap_stream = nullptr;
    hipStream_t cap_user_stream = nullptr;
    bool capturing = false;
    bool capture_bad = false;
    std::string capture_why;
    std::vector<covox::CaptureEntry> cap_subs;
    std::vector<void *> cap_host;
    std::vector<covox::AlignFrozen> cap_frozen;  // submaps read by alignment sets launched in the capture
    std::vector<covox_align_set *> align_sets;    // live alignment sets (detached by covox_destroy)
    int32_t cap_saved_timing = 0;
    int n_graphs = 0;                 // live graphs: scratch is never freed while > 0
    std::vector<void *> deferred;     // scratch replaced while capturing or while graphs live
    // timing
    int32_t timing = 0;         // bit mask of timed kernel kinds
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
    double ms[COVOX_K_COUNT] = {0};
    int64_t launches[COVOX_K_COUNT] = {0};
};

namespace covox {

// Upper limit (exclusive) of |D| for the TSDF band: the truncation distance
// less tau / 1024, so that voxels clamped in every observation (D = tau up to
// the rounding of the running average or of binary16 storage) stay outside.
inline double band_limit(const covox_params &p) { return p.trunc_vox * p.voxel_size * (1.0 - 1.0 / 1024.0); }

// Status helpers (api.hip).
int fail(covox_ctx *ctx, int code, const std::string &msg);
int hip_check(covox_ctx *ctx, hipError_t e, const char *what);

// Event timing around one kernel launch (api.hip).
struct TimedLaunch {
    covox_ctx *ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(covox_ctx *c, int k);
    ~TimedLaunch();
};

// Graph capture bookkeeping (api.hip): op 0 = reset, 1 = integration,
// 2 = ESDF / page.
void capture_touch(covox_ctx *ctx, covox_submap *s, int op);

// Device allocation helpers (api.hip): grow-only buffers.
int ensure_buffer(covox_ctx *ctx, void **ptr, int64_t *cap, int64_t need, size_t elem, const char *what);

// Orders the LDS accesses of one wave (the per-wave LDS regions need no
// workgroup barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Fill kernels (no hipMemsetAsync, so that callers may capture the work in
// a graph).
void fill_u64(hipStream_t s, uint64_t *p, uint64_t v, int64_t n);
void fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n);

// k_integrate.hip
// F <= kMaxBatch frames in one probe, one scan and one update launch; the
// result equals F integrate_frame calls bit for bit.
constexpr int kMaxBatch = 64;
int integrate_batch(covox_ctx *ctx, covox_submap *s, const float *depths, int32_t F, int32_t H, int32_t W,
                    const float K[4], const double *T_wc, bool *maybe_full);
int integrate_frame(covox_ctx *ctx, covox_submap *s, const float *depth, int32_t H, int32_t W,
                    const float K[4], const double T_wc[16], bool *maybe_full);
// Frame parameters and the frustum's block box (validates the arguments).
int prepare_frame(covox_ctx *ctx, const covox_submap *s, const float *depth, int32_t H, int32_t W, const float K[4],
                  const double T_wc[16], FrameArgs &f, int64_t &n_box);
// Host block-count bound: registers the next call and its box size.
void refresh_block_bound(covox_submap *s, int64_t next_box);
// Host block-box bound after a frame with box f was enqueued.
void grow_bounds(covox_submap *s, const FrameArgs &f);
// Compaction of ctx->cand over the box into ctx->t_key / t_idx, capacity
// check, new-block indices in key order (k_scan).
void launch_block_scan(covox_ctx *ctx, covox_submap *s, const FrameArgs &f, int64_t n_box, int64_t table_limit);

// k_pgo.hip: submap pose-graph optimisation (covox_pgo_solve)
void covox_default_pgo_cfg_impl(covox_pgo_cfg *c);
int pgo_solve(covox_ctx *ctx, covox_submap *const *subs, int32_t n, double *x, const int32_t *reg_pairs,
              int32_t n_reg, const covox_pose_factor *factors, int32_t n_fac, const covox_pgo_cfg *cfg,
              covox_pgo_stats *stats);

// k_hash.hip: stress insertion into a caller-owned table (covox_hash_insert)
int hash_insert_keys(covox_ctx *ctx, uint64_t *tkeys, uint32_t *tvals, int64_t capacity, int64_t n_present,
                     const uint64_t *keys, int64_t n, uint32_t val_base, int64_t *stats);

// k_wavefront.hip: incremental ESDF (esdf_mode COVOX_ESDF_WAVEFRONT)
int update_esdf_wavefront(covox_ctx *ctx, covox_submap *s);
int wavefront_reset(covox_ctx *ctx, covox_submap *s);

// k_raycast.hip
int raycast_frame(covox_ctx *ctx, covox_submap *s, const float *depth, int32_t H, int32_t W, const float K[4],
                  const double T_wc[16], bool *maybe_full);
int ensure_ray_acc(covox_ctx *ctx);  // accumulators for block_capacity blocks (not under capture)

// k_esdf.hip
int build_page(covox_ctx *ctx, covox_submap *s);   // page + site masks of the bounding box
int update_esdf(covox_ctx *ctx, covox_submap *s);
int autotune_esdf(covox_ctx *ctx, covox_submap *const *subs, int n);
int update_esdf_batch(covox_ctx *ctx, covox_submap *const *subs, int n);

// k_align.hip
int extract_points(covox_ctx *ctx, const covox_submap *B);  // synchronous (count read back)

struct AlignProblem {
    const float *phi;            // field of A
    const int32_t *page;         // A's page
    const SubmapMeta *metaA;     // A's domain
    const float *pts;            // points of B
    int64_t n_pts;
    double T[16];                // initial pose (B -> A)
    int32_t max_iter;
    int32_t pad;
};

struct AlignResult {
    double T[16];
    double ne[29];
    double cost;
    int64_t n_used;
    int32_t iters;
    int32_t status;
    int32_t solves;  // binary64 solves made (Gauss-Newton: = iters)
    int32_t pad;
};

int run_alignment(covox_ctx *ctx, const AlignProblem *probs, int n, AlignResult *res);

// Solver settings and launch shape of k_align, taken from a context.
struct AlignLaunch {
    float vs;
    double tol_rho, tol_theta;
    int n_min, dof, lm, threads, pps;
};
AlignLaunch align_launch_of(const covox_ctx *ctx);
// Dispatch order of n problems: longest first (stable).
void align_order(const AlignProblem *probs, int n, int32_t *order);
// k_align over n problems already on the device, results to dres (device);
// enqueues on ctx->stream only, so that it may be captured.
int launch_alignment(covox_ctx *ctx, const AlignProblem *dprob, const int32_t *dorder, int n, AlignResult *dres,
                     const AlignLaunch &L);


// Coarse ESDF summary request (k_align.hip): 32^3 cells of edge `cell`
// centred on the grid origin, grid frame -> submap frame by T.
struct SummaryReq {
    const float *phi;
    const int32_t *page;
    const SubmapMeta *meta;
    float T[12];
    float cell;
    int32_t chan;
    float *out;  // 32^3 x 4 floats (NDHWC)
};
int run_summaries(covox_ctx *ctx, const SummaryReq *reqs, int n);

// k_net.hip
int net_create(covox_ctx *ctx, uint64_t seed, covox_net **out);
covox_ctx *net_ctx(const covox_net *net);  // nullptr once the context is destroyed
void net_destroy(covox_net *net);
// Frees the device memory of a network whose context is being destroyed and
// clears its context; the handle stays valid for net_destroy only.
void net_detach(covox_net *net);
int64_t net_num_params(const covox_net *net);
int net_get_params(covox_net *net, float *host, int64_t n);
int net_set_params(covox_net *net, const float *host, int64_t n);
int net_forward_api(covox_net *net, const float *x_dev, int n, float *out_dev);
// Forward pass with the activations in the library's static device scratch
// (no allocation); n <= COVOX_NET_NOALLOC_MAX_PAIRS.
int net_forward_noalloc(covox_net *net, const float *x_dev, int n, float *out_dev);
// Takes the scratch's device address on ctx->device, once per device.
int noalloc_scratch_init(covox_ctx *ctx);
// One training step enqueued on the context stream (no host synchronisation);
// the step's loss is then at net_loss_dev(net).
int net_train_async(covox_net *net, const float *x_dev, const float *y_dev, int n, float lr, float trans_scale);
const float *net_loss_dev(const covox_net *net);
int net_train_step(covox_net *net, const float *x_dev, const float *y_dev, int n, float lr, float trans_scale,
                   float *loss_host);
int net_grads(covox_net *net, const float *x_dev, const float *y_dev, int n, float trans_scale, float *grad_host,
              float *loss_host);

}  // namespace covox

// Alignment problems prepared once on the device, launched any number of
// times (also under graph capture) and read back on demand.
struct covox_align_set {
    covox_ctx *ctx = nullptr;  // nullptr once the context is destroyed
    int32_t n = 0, n_starts = 1;
    covox::AlignLaunch launch{};
    void *dev = nullptr;                 // n n_starts problems, then their dispatch order
    covox::AlignResult *dres = nullptr;  // n n_starts results
    std::vector<double> T_init;          // n x 16
    std::vector<int64_t> n_points;       // B's registration points per pair
    std::vector<covox::AlignFrozen> frozen;
};
