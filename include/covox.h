/*
 * covox -- projective TSDF integration, exact ESDF and correspondence-free
 * ESDF submap alignment on AMD Instinct MI355X (gfx950).
 *
 * Method: Hoss and De Cristoforis, "coVoxSLAM: GPU accelerated globally
 * consistent dense SLAM" (arXiv 2410.21149).  The map is a collection of
 * submaps; each submap is a sparse set of 8^3-voxel blocks indexed through an
 * open-addressing hash table whose "activate" step hands out buffer indices
 * (Sec. III-B, III-C).  Depth frames are fused by projection mapping
 * (Sec. III-C), the ESDF is derived from the TSDF (Sec. I, III-E), and two
 * submaps are aligned by the correspondence-free ESDF registration term of
 * Eq. (1) (Sec. III-F).
 *
 * Conventions
 *   - Lengths in metres.  Poses are 4x4 row-major binary64 matrices
 *     [R t; 0 0 0 1]; T_a_b maps coordinates in frame b to frame a.
 *   - Cameras: pinhole, x right, y down, z forward; K = {fx, fy, cx, cy};
 *     integer pixel coordinates are pixel centres; a depth image stores the
 *     z coordinate, 0 (or any value outside (0, max_range]) = no measurement.
 *   - Voxel i (int32 x3) of a submap has centre (i + 0.5) * voxel_size in the
 *     submap frame; block b = i >> 3; in-block index l = (x&7) + 8(y&7) +
 *     64(z&7); packed block key ((bx+2^20)<<42) | ((by+2^20)<<21) | (bz+2^20).
 *   - Device pointers are HIP device (or managed) memory on the current
 *     device; host pointers are ordinary host memory.  The library never frees
 *     caller memory.
 *
 * Threading and streams: a context is used by one host thread at a time.  All
 * device work of a context is ordered on the stream given to
 * covox_set_stream (default: the null stream): work that a call runs on a
 * stream of the library's own (covox_map_sequence) starts after an event
 * recorded on that stream and ends before an event the stream waits for.
 * Calls marked "asynchronous" return before the device work finishes;
 * callers keep their device inputs alive until the stream has passed the
 * work.
 *
 * Errors: every call returns a status code (below).  On an error the call
 * leaves the submap unchanged unless stated otherwise; covox_last_error()
 * returns a message for the last failing call of a context.
 */
#ifndef COVOX_H
#define COVOX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define COVOX_OK 0
#define COVOX_EINVAL (-1)        /* bad argument: null pointer, size, non-rigid pose, K */
#define COVOX_EPOOL_FULL (-2)    /* block capacity of the submap would be exceeded */
#define COVOX_ETABLE_FULL (-3)   /* hash-table load would exceed 85 % */
#define COVOX_EHIP (-4)          /* HIP runtime error (message kept) */
#define COVOX_EDEGENERATE (-5)   /* alignment: fewer than n_min residuals or H not PD */
#define COVOX_NOT_CONVERGED 1    /* alignment: iteration cap reached (result valid) */

/* Storage precision of the TSDF distance D and weight W. */
#define COVOX_FP32 0
#define COVOX_FP16 1 /* binary16 storage, binary32 arithmetic */

typedef struct covox_ctx covox_ctx;
typedef struct covox_submap covox_submap;

typedef struct {
    double voxel_size;       /* voxel edge (m), e.g. 0.05 */
    int32_t trunc_vox;       /* truncation distance tau in voxels (tau = trunc_vox * voxel_size) */
    double max_range;        /* depth values above this are ignored (m) */
    double d_max;            /* ESDF range (m); R = round(d_max / voxel_size) <= 56 */
    double w_reg;            /* minimum weight of both endpoints of a registration edge */
    int64_t block_capacity;  /* blocks per submap (pre-allocated, Sec. III-D) */
    int32_t precision;       /* COVOX_FP32 or COVOX_FP16 */
    int32_t max_iter;        /* alignment iteration cap: pose updates (Gauss-Newton) or solves
                                (Levenberg-Marquardt) */
    int32_t n_min;           /* minimum number of residuals for a solve */
    double tol_rho;          /* stop when |delta_rho| < tol_rho (m) ... */
    double tol_theta;        /* ... and |delta_theta| < tol_theta (rad) */
    int32_t align_dof;       /* 6, or 4: translation and yaw only (Sec. III-F: submap poses in
                                R^3 x SO(2) when gravity is known); the 4-DoF step solves rows and
                                columns (rho_x, rho_y, rho_z, theta_z) of the normal equations */
    int32_t weight_mode;     /* observation weight (Sec. III-C, weights after the sensor's noise):
                                COVOX_WEIGHT_CONSTANT (1) or COVOX_WEIGHT_INV_DEPTH2 (1 / d^2, d = the
                                pixel's depth in m) */
    int32_t integrator;      /* COVOX_PROJECTIVE (projection mapping) or COVOX_RAYCAST (Sec. III-C
                                raycasting: see covox_integrate_depth); raycasting needs FP32 storage */
    int32_t ray_carve;       /* raycasting: 1 = rays start at the optical centre (free space is
                                carved, as the paper describes), 0 = at tau before the point */
    int32_t esdf_mode;       /* COVOX_ESDF_EXACT (exact EDT recomputed) or COVOX_ESDF_WAVEFRONT
                                (Sec. III-E incremental propagation: see covox_update_esdf) */
    int32_t align_solver;    /* COVOX_GAUSS_NEWTON or COVOX_LEVENBERG_MARQUARDT (Sec. III-F: LM with a
                                trust region); see covox_align_submaps */
} covox_params;

enum { COVOX_WEIGHT_CONSTANT = 0, COVOX_WEIGHT_INV_DEPTH2 = 1 };
enum { COVOX_PROJECTIVE = 0, COVOX_RAYCAST = 1 };
enum { COVOX_ESDF_EXACT = 0, COVOX_ESDF_WAVEFRONT = 1 };
enum { COVOX_GAUSS_NEWTON = 0, COVOX_LEVENBERG_MARQUARDT = 1 };

/* Fills p with the defaults: 0.05 m voxels, tau = 4 voxels, 5 m range, 2 m
 * ESDF, w_reg = 2, 65536 blocks, FP32, 30 iterations, n_min = 100,
 * tolerances 1e-7 m and 1e-8 rad, 6 DoF, Gauss-Newton, constant weights,
 * projection mapping (rays carved from the optical centre when raycasting). */
void covox_default_params(covox_params *p);

/* Creates a context on the current HIP device.  *out receives the handle.
 * Returns EINVAL for an invalid parameter set, EHIP on a runtime failure. */
int covox_create(covox_ctx **out, const covox_params *p);
void covox_destroy(covox_ctx *ctx);

/* Replaces the parameters that do not shape storage: w_reg, max_iter,
 * n_min, tol_rho, tol_theta, align_dof, weight_mode, integrator, ray_carve,
 * esdf_mode and align_solver (the next calls use them; switching to raycasting
 * allocates its accumulators, 16 bytes per voxel of block_capacity).  COVOX_EINVAL if p is invalid or
 * changes voxel_size, trunc_vox, max_range, d_max, block_capacity or
 * precision.  Registration points are re-extracted after a w_reg change. */
int covox_set_params(covox_ctx *ctx, const covox_params *p);

/* All later device work of ctx goes to `hip_stream` (a hipStream_t). */
int covox_set_stream(covox_ctx *ctx, void *hip_stream);

/* Blocks until all work of ctx has finished.  Returns EHIP on a device
 * error and reports a sticky capacity error of an earlier asynchronous
 * integration as EPOOL_FULL / ETABLE_FULL (once). */
int covox_sync(covox_ctx *ctx);

/* Human-readable status name; never NULL. */
const char *covox_status_string(int status);
/* Message of the last failing call of ctx ("" if none); owned by ctx. */
const char *covox_last_error(const covox_ctx *ctx);

/* ---------------------------------------------------------------- submaps */

/* A submap with pose T_world_submap (16 binary64, host).  Pre-allocates
 * block_capacity blocks and a hash table of the next power of two >= 2 x
 * block_capacity slots (load <= 50 %, Sec. IV hash-table discussion). */
int covox_submap_create(covox_ctx *ctx, const double T_world_submap[16], covox_submap **out);
void covox_submap_destroy(covox_submap *s);
/* Empties a submap (no blocks), asynchronously. */
int covox_submap_reset(covox_ctx *ctx, covox_submap *s);

/*
 * Fuses one depth frame into submap s by projection mapping (Sec. III-C;
 * count / allocate / update of Sec. III-D):
 *   T_cam_submap = T_world_cam^-1 T_world_submap in binary64, rounded once
 *   to binary32; voxel i is valid when its centre projects in front of the
 *   camera onto a pixel (nearest, floor(u + 0.5)) whose depth d lies in
 *   (0, max_range] and sdf = d - z >= -tau; blocks holding a valid voxel
 *   and not yet allocated get buffer indices n_blocks + rank in ascending
 *   packed-key order; every valid voxel takes t = min(sdf, tau),
 *   W' = W + w, D' = (D W + t w) / W' (binary32, no FMA contraction).
 * With integrator = COVOX_RAYCAST (Sec. III-C raycasting, Sec. III-D merge):
 *   T_submap_cam = T_world_submap^-1 T_world_cam (binary64, rounded once);
 *   pixel (c, r) with depth z in (0, max_range] casts the ray q = ((c - cx)
 *   z / fx, (r - cy) z / fy, z), d = R q, length r = |d|, unit u = d / r,
 *   from the optical centre o (ray_carve = 1, else from r - tau) to r + tau;
 *   the voxels it crosses (Amanatides-Woo walk in binary32, each boundary
 *   parameter ((i + [u > 0]) vs - o) * (1 / u) computed from the index,
 *   ties x before y before z) with sdf = r - (centre - o).u >= -tau contribute
 *   t = min(sdf, tau) and w; new blocks are allocated as above; each voxel
 *   sums w and t w over the frame in binary64, then W' = W + sw,
 *   D' = (D W + stw) / W' in binary32.  Every valid pixel contributes.
 * depth_dev: device, H x W binary32, row-major, metres.  K: host, 4 floats.
 * T_world_cam: host, 16 doubles.  Asynchronous.  On EPOOL_FULL / ETABLE_FULL
 * the frame is dropped and the submap is unchanged; the condition is
 * reported by this call when the library cannot rule it out beforehand,
 * otherwise by the next covox_sync.
 */
int covox_integrate_depth(covox_ctx *ctx, covox_submap *s, const float *depth_dev, int32_t H,
                          int32_t W, const float K[4], const double T_world_cam[16]);

/* F frames in order: depths_dev is F x H x W (device), T_world_cam is F x 16
 * doubles (host).  Identical results to F sequential calls. */
int covox_integrate_depth_batch(covox_ctx *ctx, covox_submap *s, const float *depths_dev, int32_t F,
                                int32_t H, int32_t W, const float K[4], const double *T_world_cam);

/* Mapping loop in one call: integrates F frames in order and updates the
 * ESDF after every esdf_every-th frame and after the last frame
 * (esdf_every <= 0: only after the last).  Identical results to the
 * equivalent sequence of covox_integrate_depth / covox_update_esdf calls.
 * With the exact ESDF and more than one update, the EDT passes of each
 * update run on a second stream of the library while the next frames are
 * integrated (each update still computes the ESDF of the TSDF after its
 * own frames); the call joins that stream back into the context stream
 * before it returns.  Arguments as covox_integrate_depth_batch.  Asynchronous. */
int covox_map_sequence(covox_ctx *ctx, covox_submap *s, const float *depths_dev, int32_t F, int32_t H,
                       int32_t W, const float K[4], const double *T_world_cam, int32_t esdf_every);

/*
 * Recomputes the ESDF phi of submap s (Sec. I, III-E): with Obs = {W > 0},
 * Band = Obs and |D| < tau (1 - 2^-10) (voxels clamped to tau in every
 * observation are not in the band, whatever the rounding of their running
 * average), Sites = Obs and |D| <= voxel_size and
 * R = round(d_max / voxel_size):
 *   Band voxels: phi = D;
 *   other observed voxels: k = min over sites of the squared voxel distance
 *   (exact), phi = sign(D) * min(d_max, voxel_size * sqrt(k)) for k <= R^2,
 *   else sign(D) * d_max (sign = +1 for D > 0, else -1);
 *   unobserved voxels: phi = NaN.
 * Asynchronous.
 * Dirty region: with the column passes (tuning edt_col_seg > 0) an update
 * after an exact one writes phi only for the blocks within ceil(R / 8)
 * blocks, along every axis, of a block whose D or W changed since (every
 * integration path flags the blocks it changes); phi elsewhere is kept,
 * being already exact, so the result equals a full recompute bit for bit.
 * The first update, and the first after a reset, a wavefront update or a
 * graph replay, recomputes everything, as does every update under the
 * per-block passes or with tuning esdf_full_recompute = 1.
 * With esdf_mode = COVOX_ESDF_WAVEFRONT, k comes instead from an
 * incremental propagation (Sec. III-E) over the allocated blocks: every
 * voxel keeps a parent site (offset) and its squared distance (<= R^2, else
 * none); sites take themselves, voxels whose parent is no longer a site
 * lose it, and the changed blocks are queued; in synchronous rounds each
 * queued block takes better parents from its neighbours' face voxels (faces
 * -x, +x, -y, +y, -z, +z), sweeps x, y, z forward and backward, and, if it
 * changed, queues itself and its neighbours.  Distances never fall below
 * the exact k; they match it on nearly every voxel.  Synchronous (the round
 * count is read back), not capturable in a graph.
 */
int covox_update_esdf(covox_ctx *ctx, covox_submap *s);

/* ESDF of n submaps (host array of handles), each pass in one launch over
 * all of them (up to 32 submaps per launch).  Identical results to n calls
 * of covox_update_esdf.  Asynchronous. */
int covox_update_esdf_batch(covox_ctx *ctx, covox_submap *const *subs, int32_t n);

/* ---------------------------------------------------------------- align */

typedef struct {
    int64_t n_points;     /* registration points of B */
    int64_t n_used;       /* residuals used at the returned pose */
    int32_t iterations;   /* pose updates applied (Levenberg-Marquardt: steps taken) */
    int32_t status;       /* COVOX_OK, COVOX_NOT_CONVERGED or COVOX_EDEGENERATE */
    int32_t best_start;   /* multi-start: the chosen start, else 0 */
    int32_t solves;       /* binary64 solves made, rejected Levenberg-Marquardt steps included
                             (Gauss-Newton: = iterations) */
} covox_align_stats;

/*
 * Aligns submap B to submap A (Sec. III-F, Eq. 1 registration term):
 * registration points of B are the zero crossings of D_B along voxel edges
 * whose endpoints are both in the band (as for the ESDF) with W >= w_reg; the residual of a
 * point p is the trilinear ESDF of A at T p, its Jacobian [g ; (T p) x g]
 * for T <- Exp(xi) T.  Gauss-Newton with binary64 6x6 Cholesky solves and
 * SE(3) updates on the device; stops when |delta_rho| < tol_rho and
 * |delta_theta| < tol_theta, or after max_iter updates.
 * With align_solver = COVOX_LEVENBERG_MARQUARDT each solve is of
 * (H + mu diag(H)) delta = -b; the trial pose Exp(delta) T is evaluated and
 * taken when the gain ratio (c/n - c'/n') / L is positive, L = -(2 delta.b +
 * delta.H.delta) / n the decrease of the mean cost c/n that the linear model
 * predicts (fewer than n_min residuals at the trial: not taken); then
 * mu *= max(1/3, 1 - (2 rho - 1)^3), nu = 2, else mu *= nu, nu *= 2 (mu starts
 * at 1e-4, nu at 2).  A step below the tolerances, or one whose L is
 * within the binary32 rounding noise of the cost (L n <= 2^-19 Q sqrt(c),
 * c = n times the mean cost, Q the largest norm of a corner of A's ESDF
 * domain in metres), ends the solve as converged without being taken;
 * max_iter caps the solves.
 * T_init_A_B, T_out (host, 16 doubles) map B coordinates into A's frame.
 * cost (host) = mean squared residual at T_out.  stats: nullable.
 * Requires covox_update_esdf(A) after A's last integration.  Synchronous.
 * Returns the alignment status (OK, NOT_CONVERGED, EDEGENERATE) or an error.
 * The map of B is read only; the library keeps B's registration points in
 * a buffer it owns inside B, extracted on the first call after B changes,
 * so calls that take the same B from several host threads must not
 * overlap (as for every call on one context).
 */
int covox_align_submaps(covox_ctx *ctx, const covox_submap *A, const covox_submap *B,
                        const double T_init_A_B[16], double T_out[16], double *cost,
                        covox_align_stats *stats);

/* Multi-start variant: start k of n_starts is T_init Trans(pbar)
 * Rz(2 pi k / n_starts) Trans(-pbar), pbar the centroid of B's points; the
 * result is the least-cost start among those with status != EDEGENERATE and
 * n_used >= max n_used / 2 (ties: smallest k).  Synchronous. */
int covox_align_multistart(covox_ctx *ctx, const covox_submap *A, const covox_submap *B,
                           const double T_init_A_B[16], int32_t n_starts, double T_out[16],
                           double *cost, covox_align_stats *stats);

typedef struct {
    const covox_submap *A;
    const covox_submap *B;
    double T_init_A_B[16];
} covox_pair;

/* n pairs, each with n_starts starts (1 = plain, 8 = multi-start), solved
 * in one persistent launch (one workgroup per pair-start, longest first).
 * Outputs (host): T_out n x 16, cost n, stats n (nullable).  Results equal
 * those of the per-pair calls.  Synchronous. */
int covox_align_batch(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts,
                      double *T_out, double *cost, covox_align_stats *stats);

/*
 * The batch of covox_align_batch in three parts, for callers that capture
 * their work in a HIP graph or repeat one alignment batch many times.
 *
 * covox_align_prepare checks the pairs as covox_align_batch does (A's ESDF
 * current, rigid starts), extracts the registration points, and uploads the
 * n x n_starts problems to device memory that the set owns.  The solver
 * settings, max_iter and the launch shape of the context at this call are
 * the set's.  Synchronous; not during capture.  *out receives the set.
 *
 * covox_align_launch enqueues the one persistent alignment launch of the
 * set on the context stream; results stay in the set's device memory.  It
 * may be called during graph capture: the launch is then recorded, and each
 * replay of the graph recomputes the results.  EINVAL when a submap of the
 * set changed (integration, reset, ESDF update) after covox_align_prepare;
 * covox_graph_launch refuses a graph in that case too, and covox_graph_end
 * refuses a capture that changes a submap that it also aligns.
 *
 * covox_align_collect waits for the stream, copies the results back and
 * selects the start of each pair: T_out (n x 16), cost (n) and stats (n,
 * nullable) as covox_align_batch returns them, bit for bit.  Before any
 * launch has run, every start reads as not converged, unmoved, with an
 * infinite cost.  Synchronous.
 *
 * covox_align_set_destroy frees the set (after the context's pending work;
 * while graphs of the context live, its device memory is kept until the
 * context is destroyed).  Destroy sets and graphs that use a submap before
 * the submap; a set outlives its context as a handle only.
 */
typedef struct covox_align_set covox_align_set;
int covox_align_prepare(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts,
                        covox_align_set **out);
int covox_align_launch(covox_ctx *ctx, covox_align_set *set);
int covox_align_collect(covox_ctx *ctx, covox_align_set *set, double *T_out, double *cost,
                        covox_align_stats *stats);
void covox_align_set_destroy(covox_align_set *set);

/* ------------------------------------------------------------ inspection */

typedef struct {
    int64_t n_blocks;
    int64_t block_capacity;
    int64_t table_capacity;
    int64_t n_updates;    /* voxel updates applied since creation / reset */
    int32_t bbox_min[3];  /* allocated block coordinates, inclusive */
    int32_t bbox_max[3];
    int32_t precision;
    int32_t status;       /* pending sticky capacity error (0 if none) */
} covox_submap_info;

/* Synchronous. */
int covox_submap_info_get(covox_ctx *ctx, const covox_submap *s, covox_submap_info *out);

/* Copies the first min(n_blocks, cap) blocks in buffer order to host arrays
 * (any may be NULL): keys (u64), home bucket mix64(key) & (table_capacity-1)
 * (u32, SplitMix64 finaliser), D, W, phi (binary32, 512 per block; FP16
 * storage is widened).  Returns the number of blocks copied (>= 0) or an
 * error (< 0).  Synchronous. */
int64_t covox_export_blocks(covox_ctx *ctx, const covox_submap *s, uint64_t *keys, uint32_t *home,
                            float *D, float *W, float *phi, int64_t cap);

/* Registration points of B (3 floats each, order: block buffer index,
 * in-block index, axis) copied to host, up to cap points.  Returns the total
 * count or an error.  Synchronous. */
int64_t covox_export_points(covox_ctx *ctx, const covox_submap *B, float *pts, int64_t cap);

/* One evaluation of the normal equations of the pair at T (host, 16
 * doubles): out[0..20] upper triangle of H row by row, out[21..26] b,
 * out[27] sum r^2, out[28] n.  Synchronous. */
int covox_normal_equations(covox_ctx *ctx, const covox_submap *A, const covox_submap *B,
                           const double T_A_B[16], double out[29]);

/* ------------------------------------------------------ learned proposal */
/* Not part of the paper: a small 3-D CNN proposes the relative pose of a
 * pair from coarse ESDF summaries; the ESDF alignment above refines it. */

typedef struct covox_net covox_net;

/* One coarse summary: the 32^3 grid of cells of edge `cell` (m) centred on
 * the grid origin; T_submap_grid maps grid coordinates into the submap
 * frame.  Writes, for every cell c (x fastest), out_dev[4 c + channel] =
 * clamp(phi / d_max, -1, 1) and out_dev[4 c + channel + 1] = 1 where the
 * trilinear ESDF is defined (all 8 corners observed), else 0 and 0.
 * out_dev: device, 32^3 x 4 floats (NDHWC input block of the network);
 * channel is 0 or 2.  Requires a current ESDF. */
typedef struct {
    const covox_submap *s;
    double T_submap_grid[16];
    double cell;
    float *out_dev;
    int32_t channel;
    int32_t reserved;
} covox_summary_req;

int covox_summaries(covox_ctx *ctx, const covox_summary_req *reqs, int32_t n);

/* Network: conv3d 4->16 (stride 1), 16->32, 32->64, 64->64 (stride 2), all
 * 3x3x3 with zero padding and ReLU, global mean, fully connected 64 -> 5
 * (tx, ty, tz, cos yaw, sin yaw).  bf16 weights and activations on the matrix
 * cores with FP32 accumulation; FP32 master weights, FP32 backward, Adam.
 * Weights are initialised from `seed` (He-uniform, SplitMix64). */
int covox_net_create(covox_ctx *ctx, uint64_t seed, covox_net **out);
/* covox_destroy frees the device memory of every net of the context; such
 * a net's handle stays valid for covox_net_destroy (which then frees only
 * the handle) and covox_net_num_params, and every other call on it returns
 * COVOX_EINVAL. */
void covox_net_destroy(covox_net *net);
int64_t covox_net_num_params(const covox_net *net);
int covox_net_get_params(covox_net *net, float *host, int64_t n);
int covox_net_set_params(covox_net *net, const float *host, int64_t n);
/* x_dev: device n x 32^3 x 4 floats; out_dev: device n x 5 floats. */
int covox_net_forward(covox_net *net, const float *x_dev, int32_t n, float *out_dev);

/* Forward pass that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and the same kernels as
 * covox_net_forward, so the outputs are bit-identical to it; asynchronous on
 * the context stream.
 *
 * The activations live in one static device array of the library, about
 * 1.6 MB per pair for COVOX_NET_NOALLOC_MAX_PAIRS pairs (13.2 MB), which each
 * GPU the library runs on holds until the process ends.  Every call on a GPU
 * shares that array: calls that overlap on one GPU (two streams, two
 * contexts or two host threads) race and give undefined outputs.  Each call
 * writes every activation it reads, so nothing carries over between calls.
 *
 *   x_dev    device n x 32^3 x 4 floats (caller-owned, as for covox_net_forward)
 *   out_dev  device n x 5 floats (caller-owned)
 *   n        1 .. COVOX_NET_NOALLOC_MAX_PAIRS; a larger n returns COVOX_EINVAL
 *            with a message and launches nothing.
 * COVOX_EINVAL also for null pointers, n <= 0, or a net whose context is
 * destroyed. */
#define COVOX_NET_NOALLOC_MAX_PAIRS 8
int covox_net_forward_noalloc(covox_net *net, const float *x_dev, int32_t n, float *out_dev);
/* One Adam step (beta 0.9 / 0.999) on the loss mean over the batch of
 * |t - t*|^2 / trans_scale^2 + |(c, s) - (c*, s*)|^2; y_dev: device n x 5.
 * loss_host (nullable) receives the loss (synchronous when given). */
int covox_net_train_step(covox_net *net, const float *x_dev, const float *y_dev, int32_t n, float lr,
                         float trans_scale, float *loss_host);
/* Gradient of that loss with respect to the FP32 parameters (host, n_params
 * floats, same layout as covox_net_get_params) without an update. */
int covox_net_gradients(covox_net *net, const float *x_dev, const float *y_dev, int32_t n, float trans_scale,
                        float *grad_host, float *loss_host);

/* Learned alignment of n pairs: A's grid is centred on the centroid c_A of
 * A's registration points (T_A_grid = Trans(c_A)); B is summarised on the
 * same grid through the prior T_init (T_B_grid = T_init^-1 T_A_grid).  The
 * network's correction C = (t, Rz(yaw)) in grid coordinates gives the
 * proposal T_A_grid C T_A_grid^-1 T_init, refined by single-start alignment.
 * With n_rot > 1 the network also sees the prior turned about the grid
 * centre, T_k = T_A_grid Rz(2 pi k / n_rot) T_A_grid^-1 T_init (k = 0 ..
 * n_rot - 1); each proposal is scored by the mean squared residual at the
 * proposal itself (one evaluation, no update), and among the proposals with
 * at least n_min residuals and at least half the largest count the least
 * cost is refined (ties: smallest k).
 * Pairs whose refined cost exceeds cost_thr (or that are degenerate) fall
 * back to n_starts-start alignment from T_init, and the refined proposal
 * competes with those starts under the multi-start selection rule (it wins
 * ties), so a fallback never returns a higher cost than the refined pose.
 * stats[i].best_start = -1 when the refined proposal was kept, else the
 * chosen start.  A net whose context was destroyed is rejected (EINVAL), as
 * is a net of another context.  Synchronous. */
int covox_align_learned(covox_ctx *ctx, covox_net *net, const covox_pair *pairs, int32_t n, double cell,
                        double cost_thr, int32_t n_rot, int32_t n_starts, double *T_out, double *cost,
                        covox_align_stats *stats);

/* The network's proposals alone for n pairs (the first step of
 * covox_align_learned): for each pair and k = 0 .. n_rot - 1 (1 <= n_rot <=
 * 256), T_A_grid C_k T_A_grid^-1 T_k with T_k the prior turned by
 * 2 pi k / n_rot about the grid centre; host n x n_rot x 16 doubles (pair
 * major).  Synchronous. */
int covox_propose(covox_ctx *ctx, covox_net *net, const covox_pair *pairs, int32_t n, double cell, int32_t n_rot,
                  double *T_prop);

/* Training on re-framings of ground-truth pairs.  Item b of step s draws
 * (SplitMix64 of seed and the counter s * batch + b) a pair j, a correction
 * C = (t, Rz(yaw)) with t uniform in [-trans_xy, trans_xy]^2 x [-trans_z,
 * trans_z] and yaw uniform in [-yaw, yaw], and a tilt E = Rx(roll) Ry(pitch)
 * with roll, pitch uniform in [-tilt, tilt]; the prior is T_init = T_A_grid
 * C^-1 T_A_grid^-1 T_gt E and the network is trained (one Adam step per step)
 * to output C.  The summaries are re-sampled from the existing ESDFs; nothing
 * is re-integrated. */
typedef struct {
    int32_t steps;       /* Adam steps */
    int32_t batch;       /* items per step, 1..256 */
    double lr;           /* Adam learning rate */
    double trans_scale;  /* translation scale of the loss (m) */
    double cell;         /* summary cell edge (m) */
    double trans_xy;     /* correction translation range in x and y (m) */
    double trans_z;      /* correction translation range in z (m) */
    double yaw;          /* correction yaw range (rad) */
    double tilt;         /* roll / pitch range of the prior (rad) */
    uint64_t seed;
} covox_train_cfg;

/* pairs[i].T_init_A_B holds the ground truth T_A_B of the pair; both ESDFs
 * must be current.  loss_host (nullable): the loss of every step (steps
 * floats).  Synchronous. */
int covox_train_proposal(covox_ctx *ctx, covox_net *net, const covox_train_cfg *cfg, const covox_pair *pairs,
                         int32_t n, float *loss_host);

/* --------------------------------------------------- pose graph (Eq. 1) */

/*
 * Submap pose-graph optimisation (Eq. 1, Sec. III-F backend): the poses of
 * n submaps minimise
 *   F = sum_reg c_ij / sigma_reg^2 + sum_factors e^T diag(1 / sigma^2) e
 * where c_ij is the sum of squared alignment residuals phi_i(T_i^-1 T_j p)
 * over the registration points p of submap j (the residual of
 * covox_normal_equations), and e is a 4-DoF relative-pose error.
 *   pose of submap k: x_k = (t_x, t_y, t_z, yaw), T_k = [Rz(yaw) t; 0 1]
 *     (R^3 x SO(2): gravity known); x_0 is held fixed;
 *   factor (i, j) with measured z of T_i^-1 T_j:
 *     e_t = Rz(-z_yaw) (Rz(-yaw_i) (t_j - t_i) - z_t),
 *     e_yaw = wrap(yaw_j - yaw_i - z_yaw);
 *   registration blocks: the 6x6 normal equations of T_ij under the left
 *     perturbation, chained to x_i and x_j through Ad(T_i^-1) and the
 *     first-order twist of (dt, dyaw);
 *   Levenberg-Marquardt: (H + mu diag(H)) delta = -g solved by
 *     block-Jacobi preconditioned CG on the block-sparse system; a step is
 *     taken when the gain ratio is positive; mu follows the update of Madsen,
 *     Nielsen and Tingleff (2004); stops when max |delta| < tol_step.
 * Odometry and loop-closure factors have the same form (their sigmas
 * differ).  Every submap of a registration pair needs a current ESDF (the
 * field side) and registration points (the point side, extracted here).
 */
typedef struct {
    int32_t i, j;         /* submap indices into the pose array */
    int32_t reserved[2];
    double z[4];          /* measured T_i^-1 T_j: (t_x, t_y, t_z) in m, yaw in rad */
    double sigma[4];      /* standard deviations of the four error components (> 0) */
} covox_pose_factor;

typedef struct {
    int32_t max_iter;     /* LM solves (20) */
    int32_t cg_max_iter;  /* PCG iterations per solve; 0 = the system size */
    double sigma_reg;     /* registration residual standard deviation, m (0.05) */
    double lambda0;       /* initial damping, relative to diag(H) (1e-4) */
    double tol_step;      /* stop when max |delta| < tol_step (1e-8) */
    double cg_tol;        /* PCG stop: |r| <= cg_tol |b| (1e-12) */
} covox_pgo_cfg;

typedef struct {
    int32_t iterations;     /* LM solves */
    int32_t accepted;       /* steps taken */
    int32_t converged;      /* 1 when max |delta| fell below tol_step */
    int32_t cg_iterations;  /* PCG iterations over all solves */
    double cost_init;       /* F at the initial poses */
    double cost_final;      /* F at the returned poses */
} covox_pgo_stats;

void covox_default_pgo_cfg(covox_pgo_cfg *cfg);

/* subs: n submaps (n >= 2).  x: host, n x 4 doubles, the initial poses on
 * entry and the optimised ones on return (x_0 unchanged).  reg_pairs: host,
 * n_reg x 2 int32 (i = the submap whose ESDF is sampled, j = the submap whose
 * registration points are moved), i != j.  factors: host, n_fac entries.
 * cfg: nullable (defaults).  stats: nullable.  Synchronous.  EINVAL for bad
 * indices, sigmas or sizes, or when the damped system is not positive
 * definite. */
int covox_pgo_solve(covox_ctx *ctx, covox_submap *const *subs, int32_t n, double *x, const int32_t *reg_pairs,
                    int32_t n_reg, const covox_pose_factor *factors, int32_t n_fac, const covox_pgo_cfg *cfg,
                    covox_pgo_stats *stats);

/* -------------------------------------------------------------- graphs */

/* Capture of the asynchronous calls of a context into a HIP graph, so that a
 * launch-bound sequence (a mapping loop: reset, F frames, ESDF updates) is
 * replayed with one launch.
 *
 * Between covox_graph_begin and covox_graph_end only covox_submap_reset,
 * the integration calls, covox_map_sequence and the ESDF updates may be
 * called on ctx (every other call returns COVOX_EINVAL), and nothing else
 * may use the context stream.  Nothing runs during capture, and the host
 * bookkeeping of every submap is as before covox_graph_begin afterwards.
 * A submap integrated inside the graph must be reset inside it first
 * (covox_graph_end fails otherwise).  Both integrators can be captured
 * (raycasting needs its accumulators, which covox_create / covox_set_params
 * allocate); the wavefront ESDF cannot (it reads its round count back), and
 * its update returns COVOX_EINVAL under capture.
 *
 * covox_graph_launch enqueues the captured kernels on the context stream
 * with their captured arguments: the same submaps, poses, intrinsics and
 * depth pointers (the depth contents may change between launches), and
 * updates the host bookkeeping as the captured calls would.  A submap that
 * the graph updates without resetting must not have grown since the
 * capture (COVOX_EINVAL).  Capacity errors of captured integrations are not
 * reported by the launch: they stay in the submap's sticky status
 * (covox_submap_info, covox_sync).  While any graph of a context exists,
 * the context keeps every scratch buffer it replaces until the last graph
 * is destroyed.  Submaps used by a graph must outlive it, and every graph
 * of a context must be destroyed before the context. */
typedef struct covox_graph covox_graph;
int covox_graph_begin(covox_ctx *ctx);
int covox_graph_end(covox_ctx *ctx, covox_graph **out);
int covox_graph_launch(covox_graph *g);
void covox_graph_destroy(covox_graph *g);

/* ---------------------------------------------------------- hash table */

/* Hash-table stress test (Sec. IV, hash-table stress testing: insertions
 * at a range of load factors).  Inserts n keys into a table that the caller
 * owns, with the routine that maps block coordinates to block indices in
 * every submap (Sec. III-B): open addressing, home slot = SplitMix64
 * finaliser of the key masked to the capacity, linear probing towards
 * higher slots (wrapping), one 64-bit compare-and-swap per probed slot.
 * Concurrent inserts of one call land in slots that depend on scheduling;
 * the set of occupied slots and the probe sum do not (linear probing).
 *
 *   table_keys  device uint64[capacity]; an empty slot holds UINT64_MAX.
 *               The caller fills every slot with UINT64_MAX before the
 *               first insert and keeps the table between calls.
 *   table_vals  device uint32[capacity]; the slot that receives keys[i]
 *               gets val_base + i (modulo 2^32).
 *   capacity    slots: a power of two, 2 .. 2^32.
 *   n_present   keys already in the table.  After the call at most 15/16
 *               of the slots may be occupied (n_present + n), else
 *               COVOX_ETABLE_FULL and nothing runs.
 *   keys        device uint64[n]: distinct, absent from the table, none
 *               equal to UINT64_MAX.  A key already present is inserted
 *               a second time.
 *   stats       device int64[3], raised by the call (the caller clears it):
 *               [0] = max over this call's keys of the probe length (slots
 *               past the home slot), [1] += sum of the probe lengths,
 *               [2] += keys not inserted because capacity slots in a row
 *               were occupied (only when n_present understated the load or
 *               the table was not cleared; such a probe stops there).
 *
 * Asynchronous on the context stream.  COVOX_EINVAL for a null pointer, a
 * capacity that is not a power of two in range, or a negative count. */
int covox_hash_insert(covox_ctx *ctx, uint64_t *table_keys, uint32_t *table_vals, int64_t capacity,
                      int64_t n_present, const uint64_t *keys, int64_t n, uint32_t val_base, int64_t *stats);

/* -------------------------------------------------------------- tuning */

/* Launch shapes chosen per call.  Each line pass of the EDT (y, then z) has
 * two exact implementations: a voxel-parallel windowed search (cost follows
 * the distance to the nearest site) and per-line lower envelopes (cost
 * follows the line length; one lane per line segment).  A pass uses the
 * envelopes when the call has at least *_env_min_cols line segments. */
typedef struct {
    int64_t edt_y_env_min_cols;
    int64_t edt_z_env_min_cols;
    /* Lanes of the workgroup that runs one Gauss-Newton problem (256 or
     * 512).  The FP64 sums are reduced in a fixed order for a given value,
     * so results are reproducible for a given setting and differ between
     * settings only by rounding. */
    int64_t align_threads;
    /* Points a lane handles per step (1 or 2; their loads overlap).  The
     * results do not depend on it. */
    int64_t align_points_per_step;
    /* Most workgroups of each EDT pass launch while the passes run beside
     * an integration (covox_map_sequence): a smaller grid, which the passes
     * cover with a grid stride, leaves CUs to the integration.  0: no
     * limit.  The results do not depend on it. */
    int64_t edt_pipe_max_workgroups;
    /* EDT pass layout.  0: separate x, y and z passes, one work item per
     * block or per line (shapes by the thresholds above).  S > 0: column
     * passes, x fused into y, each workgroup one segment of S blocks of a
     * block column with HB = ceil(R / 8) halo blocks on each side staged
     * once; S is clamped to 48 - 2 HB.  The results do not depend on it. */
    int64_t edt_col_seg;
    /* Exact ESDF updates with the column passes recompute only the blocks
     * within ceil(R / 8) blocks of a block whose TSDF changed since the
     * submap's last exact update (the rest keeps its phi, which is already
     * exact), or everything on the first update, after a reset, a wavefront
     * update or a graph replay.  1: every update recomputes everything (for
     * timing full updates).  The results do not depend on it. */
    int64_t esdf_full_recompute;
    /* Work order of the kernels that gather depth pixels (the probes and the
     * frame-batch integration).  1: workgroup w of a grid of 8 C takes work
     * item (w mod 8) C + floor(w / 8); the dispatcher deals workgroups to
     * the eight XCDs in turn, so each XCD covers one contiguous eighth of
     * the blocks (or of the frame-block pairs of a batch) and the depth rows
     * they read stay in its own L2.  0 (default): items in dispatch order;
     * on MI355X the XCD order gained nothing (outdoor frame batches: probe
     * 12.8 against 11.7 ms per 3000 frames; room probe unchanged).  The
     * results do not depend on it. */
    int64_t mapping_xcd_order;
} covox_tuning;

/* Defaults: y envelopes from 2048 segments up, z always windowed, 256
 * lanes per alignment problem, one point per step, no workgroup cap. */
void covox_default_tuning(covox_tuning *t);
int covox_tuning_get(const covox_ctx *ctx, covox_tuning *out);
int covox_tuning_set(covox_ctx *ctx, const covox_tuning *t);

/* Autotuner: recomputes the ESDF of the (up to 32 distinct) submaps with
 * every combination of pass shapes, times each with HIP events on the
 * context stream (best of 3), and moves the thresholds so that the fastest
 * combination is the one chosen for calls of this size.  The ESDF result
 * is the same for every shape.  out (nullable) receives the new tuning.
 * Synchronous. */
int covox_autotune_esdf(covox_ctx *ctx, covox_submap *const *subs, int32_t n, covox_tuning *out);

/* Autotuner of the alignment launch: runs covox_align_batch on these pairs
 * with 256 and 512 lanes per problem and 1 and 2 points per step (best of 3
 * each) and keeps the fastest.  out (nullable) receives the new tuning.
 * Synchronous. */
int covox_autotune_align(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts, covox_tuning *out);

/* ---------------------------------------------------------------- timing */

enum {
    COVOX_K_PROBE = 0,     /* block candidates: projective any-valid test + hash find */
    COVOX_K_SCAN,          /* compaction, capacity check, index assignment */
    COVOX_K_INTEGRATE,     /* projective TSDF update (+ activate of new blocks) */
    COVOX_K_ESDF_PAGE,     /* dense block page of the submap's box */
    COVOX_K_ESDF_SITES,    /* site bit masks */
    COVOX_K_EDT_X,         /* nearest site along x */
    COVOX_K_EDT_Y,         /* lower envelope along y */
    COVOX_K_EDT_Z,         /* lower envelope along z + phi */
    COVOX_K_ISO,           /* registration points */
    COVOX_K_ALIGN,         /* Gauss-Newton (persistent) */
    COVOX_K_SUMMARY,       /* coarse ESDF summaries */
    COVOX_K_NET,           /* proposal network (forward or backward) */
    COVOX_K_RAY_MARK,      /* raycasting: clear, walk and flag touched blocks, resolve their index */
    COVOX_K_RAY_ACCUM,     /* raycasting: walk again and accumulate (w, t w) per voxel */
    COVOX_K_RAY_APPLY,     /* raycasting: activate new blocks, merge the sums into D and W */
    COVOX_K_PGO,           /* pose graph: term blocks, block-sparse assembly, PCG */
    COVOX_K_WAVEFRONT,     /* incremental ESDF: seeds, rounds (queue, block sweeps, commit), phi */
    COVOX_K_HASH,          /* hash-table stress insertion (covox_hash_insert) */
    COVOX_K_COUNT
};

typedef struct {
    double ms[COVOX_K_COUNT];       /* summed kernel time (HIP events on the ctx stream) */
    int64_t launches[COVOX_K_COUNT];
} covox_timing;

/* Clears the accumulated timing and enables HIP-event timing for the
 * kernel kinds whose bit (1 << COVOX_K_*) is set in `mask` (0 disables,
 * -1 enables all).  Each timed launch is bracketed by two events on the
 * context stream. */
int covox_timing_enable(covox_ctx *ctx, int32_t mask);
/* Synchronizes and returns the accumulated timing. */
int covox_timing_get(covox_ctx *ctx, covox_timing *out);

#ifdef __cplusplus
}
#endif

#endif /* COVOX_H */
