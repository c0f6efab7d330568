// C ABI of the covox library (include/covox.h): contexts, submaps, the
// integrate / ESDF / align entry points, inspection and kernel timing.
#include "covox_impl.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <vector>

namespace covox {

namespace {

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

unsigned fill_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

void fill_u64(hipStream_t s, uint64_t *p, uint64_t v, int64_t n)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

void fill_u32(hipStream_t s, uint32_t *p, uint32_t v, int64_t n)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

int fail(covox_ctx *ctx, int code, const std::string &msg)
{
    if (ctx) ctx->last_error = msg;
    return code;
}

int hip_check(covox_ctx *ctx, hipError_t e, const char *what)
{
    if (e == hipSuccess) return COVOX_OK;
    return fail(ctx, COVOX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

TimedLaunch::TimedLaunch(covox_ctx *c, int k) : ctx(c), kind(k)
{
    if (!(ctx->timing & (1 << kind))) return;
    for (hipEvent_t *e : {&a, &b}) {
        if (!ctx->ev_pool.empty()) {
            *e = ctx->ev_pool.back();
            ctx->ev_pool.pop_back();
        } else if (hipEventCreate(e) != hipSuccess) {
            *e = nullptr;
        }
    }
    if (a) (void)hipEventRecord(a, ctx->stream);
}

TimedLaunch::~TimedLaunch()
{
    if (!(ctx->timing & (1 << kind))) return;
    if (a && b) {
        (void)hipEventRecord(b, ctx->stream);
        ctx->ev_used.push_back({kind, {a, b}});
    } else {
        if (a) ctx->ev_pool.push_back(a);
        if (b) ctx->ev_pool.push_back(b);
    }
}

int ensure_buffer(covox_ctx *ctx, void **ptr, int64_t *cap, int64_t need, size_t elem, const char *what)
{
    if (need <= *cap && *ptr) return COVOX_OK;
    int64_t nc = std::max<int64_t>(need, *cap + *cap / 2);
    if (*ptr) {
        if (ctx->capturing || ctx->n_graphs > 0) {
            // captured kernels may still name the old buffer: keep it
            ctx->deferred.push_back(*ptr);
        } else {
            hipError_t e = hipStreamSynchronize(ctx->stream);
            if (e != hipSuccess) return hip_check(ctx, e, "sync before reallocation");
            (void)hipFree(*ptr);
        }
        *ptr = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc(ptr, (size_t)nc * elem);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(ctx, COVOX_EHIP, std::string("allocating ") + what + ": " + hipGetErrorString(e));
    }
    *cap = nc;
    return COVOX_OK;
}

SubmapSnap snap(const covox_submap *s)
{
    SubmapSnap q;
    q.nb_upper = s->nb_upper;
    q.bound_valid = s->bound_valid;
    for (int a = 0; a < 3; ++a) { q.bound_lo[a] = s->bound_lo[a]; q.bound_hi[a] = s->bound_hi[a]; }
    q.version = s->version;
    q.page_version = s->page_version;
    q.esdf_version = s->esdf_version;
    q.pts_version = s->pts_version;
    q.n_pts = s->n_pts;
    return q;
}

void restore(covox_submap *s, const SubmapSnap &q)
{
    s->nb_upper = q.nb_upper;
    s->bound_valid = q.bound_valid;
    for (int a = 0; a < 3; ++a) { s->bound_lo[a] = q.bound_lo[a]; s->bound_hi[a] = q.bound_hi[a]; }
    s->version = q.version;
    s->page_version = q.page_version;
    s->esdf_version = q.esdf_version;
    s->pts_version = q.pts_version;
    s->n_pts = q.n_pts;
}

void capture_touch(covox_ctx *ctx, covox_submap *s, int op)
{
    if (!ctx->capturing) return;
    CaptureEntry *e = nullptr;
    for (auto &c : ctx->cap_subs)
        if (c.s == s) e = &c;
    if (!e) {
        ctx->cap_subs.push_back(CaptureEntry{s, snap(s), SubmapSnap{}, op == 0, false});
        e = &ctx->cap_subs.back();
    }
    if (op == 1) {
        e->integrated = true;
        if (!e->reset_first) {
            ctx->capture_bad = true;
            ctx->capture_why = "a submap integrated inside a graph must be reset first inside the same graph";
        }
    }
}

}  // namespace covox

using namespace covox;

namespace {

std::vector<covox_submap *> &submaps_of(covox_ctx *ctx) { return ctx->subs; }

// Calls that wait for the device or return device results cannot be
// captured into a graph.
#define COVOX_NOT_DURING_CAPTURE(ctx, what)                                                  \
    do {                                                                                   \
        if ((ctx) && (ctx)->capturing)                                                     \
            return fail((ctx), COVOX_EINVAL, std::string(what) + ": not allowed while capturing a graph"); \
    } while (0)

bool valid_params(const covox_params *p, std::string &why)
{
    if (!(p->voxel_size > 0) || !std::isfinite(p->voxel_size)) { why = "voxel_size must be positive"; return false; }
    if (p->trunc_vox < 1) { why = "trunc_vox must be >= 1"; return false; }
    if (!(p->max_range > 0)) { why = "max_range must be positive"; return false; }
    if (!(p->d_max > 0)) { why = "d_max must be positive"; return false; }
    const long long R = llround(p->d_max / p->voxel_size);
    if (R < 1 || R > 8 * kMaxHalo) { why = "d_max / voxel_size must round to 1..56"; return false; }
    if (p->block_capacity < 1 || p->block_capacity > (1ll << 30)) { why = "block_capacity out of range"; return false; }
    if (p->precision != COVOX_FP32 && p->precision != COVOX_FP16) { why = "precision must be FP32 or FP16"; return false; }
    if (p->max_iter < 0) { why = "max_iter must be >= 0"; return false; }
    if (p->n_min < 1) { why = "n_min must be >= 1"; return false; }
    if (p->align_dof != 6 && p->align_dof != 4) { why = "align_dof must be 6 or 4"; return false; }
    if (p->weight_mode != COVOX_WEIGHT_CONSTANT && p->weight_mode != COVOX_WEIGHT_INV_DEPTH2) {
        why = "weight_mode must be COVOX_WEIGHT_CONSTANT or COVOX_WEIGHT_INV_DEPTH2";
        return false;
    }
    if (p->integrator != COVOX_PROJECTIVE && p->integrator != COVOX_RAYCAST) {
        why = "integrator must be COVOX_PROJECTIVE or COVOX_RAYCAST";
        return false;
    }
    if (p->ray_carve != 0 && p->ray_carve != 1) { why = "ray_carve must be 0 or 1"; return false; }
    if (p->integrator == COVOX_RAYCAST && p->precision != COVOX_FP32) {
        // a voxel near the camera gains one weight per ray and frame
        why = "raycasting needs FP32 storage (weights exceed the binary16 range)";
        return false;
    }
    if (p->esdf_mode != COVOX_ESDF_EXACT && p->esdf_mode != COVOX_ESDF_WAVEFRONT) {
        why = "esdf_mode must be COVOX_ESDF_EXACT or COVOX_ESDF_WAVEFRONT";
        return false;
    }
    if (p->align_solver != COVOX_GAUSS_NEWTON && p->align_solver != COVOX_LEVENBERG_MARQUARDT) {
        why = "align_solver must be COVOX_GAUSS_NEWTON or COVOX_LEVENBERG_MARQUARDT";
        return false;
    }
    return true;
}

int read_meta(covox_ctx *ctx, const covox_submap *s, SubmapMeta *m)
{
    int rc = hip_check(ctx, hipMemcpyAsync(m, s->meta, sizeof(*m), hipMemcpyDeviceToHost, ctx->stream), "meta copy");
    if (rc) return rc;
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "meta sync");
}

__global__ void k_clear_status(SubmapMeta *m) { m->status = 0; }

__global__ void k_reset_meta(SubmapMeta *m)
{
    m->n_blocks = 0;
    for (int a = 0; a < 3; ++a) { m->bmin[a] = 0; m->bmax[a] = -1; m->dom_min[a] = 0; m->dom_dim[a] = 0; }
    m->status = 0;
    m->n_new = 0;
    m->n_touched = 0;
    m->dom_valid = 0;
    m->dom_nblocks = 0;
    m->n_points = 0;
    m->pbar[0] = m->pbar[1] = m->pbar[2] = 0.0;
    m->n_updates = 0;
}

int check_status_after_sync(covox_ctx *ctx, covox_submap *s)
{
    // Under capture nothing runs yet: the device-side capacity check still
    // guards every commit, and its sticky status is read after a launch.
    if (ctx->capturing) return COVOX_OK;
    SubmapMeta m;
    int rc = read_meta(ctx, s, &m);
    if (rc) return rc;
    s->nb_upper = m.n_blocks;
    if (m.status != 0) {
        hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, ctx->stream, s->meta);
        return fail(ctx, m.status, m.status == COVOX_EPOOL_FULL ? "integrate: block capacity exceeded"
                                                                : "integrate: hash table load limit exceeded");
    }
    return COVOX_OK;
}

// F frames in order: one frame per call through the per-frame kernels,
// several through batches of up to kMaxBatch frames.
int integrate_frames(covox_ctx *ctx, covox_submap *s, const float *depths, int32_t F, int32_t H, int32_t W,
                     const float K[4], const double *T_wc)
{
    // raycasting runs frame by frame (a capacity failure stops at its frame)
    const int32_t per_call = ctx->p.integrator == COVOX_RAYCAST ? 1 : kMaxBatch;
    for (int32_t f0 = 0; f0 < F;) {
        const int32_t n = std::min<int32_t>(per_call, F - f0);
        bool maybe_full = false;
        const float *d = depths + (size_t)f0 * H * W;
        int rc = n == 1 ? integrate_frame(ctx, s, d, H, W, K, T_wc + 16 * f0, &maybe_full)
                        : integrate_batch(ctx, s, d, n, H, W, K, T_wc + 16 * f0, &maybe_full);
        if (rc) return rc;
        if (maybe_full && (rc = check_status_after_sync(ctx, s))) return rc;
        f0 += n;
    }
    return COVOX_OK;
}

bool rigid_pose(const double *T)
{
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(T[k])) return false;
    if (T[12] != 0 || T[13] != 0 || T[14] != 0 || T[15] != 1) return false;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + r] * T[4 * k + c];
            if (std::fabs(s - (r == c ? 1.0 : 0.0)) > 1e-6) return false;
        }
    return true;
}

void rigid_inverse_h(const double *T, double *O)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) O[4 * r + c] = T[4 * c + r];
    for (int r = 0; r < 3; ++r) O[4 * r + 3] = -(O[4 * r] * T[3] + O[4 * r + 1] * T[7] + O[4 * r + 2] * T[11]);
    O[12] = 0; O[13] = 0; O[14] = 0; O[15] = 1;
}

void mat_mul4(const double *A, const double *B, double *O)
{
    double t[16];
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) t[4 * r + c] = A[4 * r] * B[c] + A[4 * r + 1] * B[4 + c] + A[4 * r + 2] * B[8 + c] + A[4 * r + 3] * B[12 + c];
    memcpy(O, t, sizeof(t));
}

int prepare_pair(covox_ctx *ctx, const covox_submap *A, const covox_submap *B)
{
    if (!A || !B) return fail(ctx, COVOX_EINVAL, "align: null submap");
    if (A->esdf_version != A->version)
        return fail(ctx, COVOX_EINVAL, "align: the ESDF of A is out of date (call covox_update_esdf)");
    return extract_points(ctx, B);
}

AlignProblem make_problem(covox_ctx *ctx, const covox_submap *A, const covox_submap *B, const double *T, int max_iter)
{
    AlignProblem pr;
    memset(&pr, 0, sizeof(pr));
    pr.phi = A->phi;
    pr.page = A->page;
    pr.metaA = A->meta;
    pr.pts = B->pts;
    pr.n_pts = B->n_pts;
    memcpy(pr.T, T, sizeof(pr.T));
    pr.max_iter = max_iter;
    (void)ctx;
    return pr;
}

void start_pose(const double *T_init, const double pbar[3], int k, int n, double *out)
{
    const double a = 2.0 * M_PI * (double)k / (double)n;
    const double P[16] = {1, 0, 0, pbar[0], 0, 1, 0, pbar[1], 0, 0, 1, pbar[2], 0, 0, 0, 1};
    const double Pm[16] = {1, 0, 0, -pbar[0], 0, 1, 0, -pbar[1], 0, 0, 1, -pbar[2], 0, 0, 0, 1};
    const double Rz[16] = {cos(a), -sin(a), 0, 0, sin(a), cos(a), 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    double S[16];
    mat_mul4(T_init, P, S);
    mat_mul4(S, Rz, S);
    mat_mul4(S, Pm, out);
    out[12] = 0; out[13] = 0; out[14] = 0; out[15] = 1;
}

// Picks the least-cost start among those not degenerate with
// n_used >= max n_used / 2 (ties: smallest k).
int select_start(const AlignResult *r, int n)
{
    int64_t nmax = 0;
    for (int k = 0; k < n; ++k)
        if (r[k].status != COVOX_EDEGENERATE) nmax = std::max(nmax, r[k].n_used);
    int best = -1;
    for (int k = 0; k < n; ++k) {
        if (r[k].status == COVOX_EDEGENERATE) continue;
        if (2 * r[k].n_used < nmax) continue;
        if (best < 0 || r[k].cost < r[best].cost) best = k;
    }
    return best;
}

void fill_stats(covox_align_stats *st, int64_t n_points, const AlignResult &r, int best)
{
    if (!st) return;
    st->n_points = n_points;
    st->n_used = r.n_used;
    st->iterations = r.iters;
    st->status = r.status;
    st->best_start = best;
    st->solves = r.solves;
}

// Per pair: the chosen start (least cost under select_start; one start:
// that start unless degenerate), its pose, cost and statistics.
void finish_pairs(int n, int n_starts, const AlignResult *res, const double *T_init, const int64_t *n_points,
                  double *T_out, double *cost, covox_align_stats *stats)
{
    for (int i = 0; i < n; ++i) {
        const AlignResult *r = &res[(size_t)i * n_starts];
        const int best = n_starts == 1 ? (r[0].status == COVOX_EDEGENERATE ? -1 : 0) : select_start(r, n_starts);
        if (best < 0) {
            memcpy(T_out + 16 * i, T_init + 16 * (size_t)i, sizeof(double) * 16);
            if (n_starts == 1) memcpy(T_out + 16 * i, r[0].T, sizeof(double) * 16);
            cost[i] = n_starts == 1 ? r[0].cost : INFINITY;
            if (stats) {
                if (n_starts == 1) fill_stats(stats + i, n_points[i], r[0], 0);
                else { memset(stats + i, 0, sizeof(*stats)); stats[i].n_points = n_points[i]; }
                stats[i].status = COVOX_EDEGENERATE;
                stats[i].best_start = n_starts == 1 ? 0 : -1;
            }
            continue;
        }
        memcpy(T_out + 16 * i, r[best].T, sizeof(double) * 16);
        cost[i] = r[best].cost;
        fill_stats(stats ? stats + i : nullptr, n_points[i], r[best], best);
    }
}

}  // namespace

extern "C" {

void covox_default_params(covox_params *p)
{
    if (!p) return;
    p->voxel_size = 0.05;
    p->trunc_vox = 4;
    p->max_range = 5.0;
    p->d_max = 2.0;
    p->w_reg = 2.0;
    p->block_capacity = 65536;
    p->precision = COVOX_FP32;
    p->max_iter = 30;
    p->n_min = 100;
    p->tol_rho = 1e-7;
    p->tol_theta = 1e-8;
    p->align_dof = 6;
    p->weight_mode = COVOX_WEIGHT_CONSTANT;
    p->integrator = COVOX_PROJECTIVE;
    p->ray_carve = 1;
    p->esdf_mode = COVOX_ESDF_EXACT;
    p->align_solver = COVOX_GAUSS_NEWTON;
}

const char *covox_status_string(int s)
{
    switch (s) {
    case COVOX_OK: return "COVOX_OK";
    case COVOX_EINVAL: return "COVOX_EINVAL";
    case COVOX_EPOOL_FULL: return "COVOX_EPOOL_FULL";
    case COVOX_ETABLE_FULL: return "COVOX_ETABLE_FULL";
    case COVOX_EHIP: return "COVOX_EHIP";
    case COVOX_EDEGENERATE: return "COVOX_EDEGENERATE";
    case COVOX_NOT_CONVERGED: return "COVOX_NOT_CONVERGED";
    default: return "COVOX_UNKNOWN";
    }
}

const char *covox_last_error(const covox_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int covox_create(covox_ctx **out, const covox_params *p)
{
    if (!out || !p) return COVOX_EINVAL;
    *out = nullptr;
    std::string why;
    if (!valid_params(p, why)) return COVOX_EINVAL;
    covox_ctx *ctx = new covox_ctx();
    ctx->p = *p;
    covox_default_tuning(&ctx->tune);
    if (const char *m = getenv("COVOX_EDT_MODE")) {
        if (!strcmp(m, "window")) ctx->edt_mode = 1;
        else if (!strcmp(m, "envelope")) ctx->edt_mode = 2;
    }
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return COVOX_EHIP;
    }
    if (noalloc_scratch_init(ctx) != COVOX_OK) {
        delete ctx;
        return COVOX_EHIP;
    }
    if (p->integrator == COVOX_RAYCAST && ensure_ray_acc(ctx) != COVOX_OK) {
        delete ctx;
        return COVOX_EHIP;
    }
    *out = ctx;
    return COVOX_OK;
}

void covox_destroy(covox_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    auto &subs = submaps_of(ctx);
    for (covox_submap *s : std::vector<covox_submap *>(subs)) covox_submap_destroy(s);
    // Networks outlive nothing of the context: their device memory goes now,
    // and their handles stay valid for covox_net_destroy alone.
    for (covox_net *net : ctx->nets) net_detach(net);
    ctx->nets.clear();
    // Alignment sets likewise: device memory now, handles for covox_align_set_destroy.
    for (covox_align_set *set : ctx->align_sets) {
        for (void *p : {set->dev, (void *)set->dres})
            if (p) (void)hipFree(p);
        set->dev = nullptr;
        set->dres = nullptr;
        set->ctx = nullptr;
    }
    ctx->align_sets.clear();
    for (void *ptr : {(void *)ctx->cand, (void *)ctx->t_key, (void *)ctx->t_idx, (void *)ctx->sites[0], (void *)ctx->g1,
                      (void *)ctx->g2, (void *)ctx->cnt, (void *)ctx->psum, ctx->prob_dev, ctx->res_dev, ctx->sum_dev,
                      (void *)ctx->net_in, (void *)ctx->net_out, (void *)ctx->train_y, (void *)ctx->loss_hist,
                      (void *)ctx->frames_dev, (void *)ctx->blist, (void *)ctx->fkeys, (void *)ctx->ffirst,
                      (void *)ctx->fcount, (void *)ctx->ray_acc, (void *)ctx->wf_nk, (void *)ctx->wf_np,
                      (void *)ctx->wf_sites, (void *)ctx->wf_flag, (void *)ctx->wf_list, (void *)ctx->wf_cnt,
                      (void *)ctx->sites[1], (void *)ctx->seeds[0], (void *)ctx->seeds[1], (void *)ctx->snap[0],
                      (void *)ctx->snap[1], (void *)ctx->blk[0], (void *)ctx->blk[1], (void *)ctx->ddirty[0],
                      (void *)ctx->ddirty[1]})
        if (ptr) (void)hipFree(ptr);
    for (void *p : ctx->deferred) (void)hipFree(p);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->esdf_stream) {
        (void)hipStreamSynchronize(ctx->esdf_stream);
        (void)hipStreamDestroy(ctx->esdf_stream);
    }
    for (hipEvent_t e : {ctx->ev_fork, ctx->ev_paged, ctx->ev_join, ctx->ev_free[0], ctx->ev_free[1]})
        if (e) (void)hipEventDestroy(e);
    if (ctx->wf_pin) (void)hipHostFree(ctx->wf_pin);
    for (int k = 0; k < 2; ++k) {
        if (ctx->frames_pin[k]) (void)hipHostFree(ctx->frames_pin[k]);
        if (ctx->frames_ev[k]) (void)hipEventDestroy(ctx->frames_ev[k]);
    }
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto &u : ctx->ev_used) {
        (void)hipEventDestroy(u.second.first);
        (void)hipEventDestroy(u.second.second);
    }
    delete ctx;
}

int covox_set_params(covox_ctx *ctx, const covox_params *p)
{
    if (!ctx || !p) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(ctx, "set_params");
    std::string why;
    if (!valid_params(p, why)) return fail(ctx, COVOX_EINVAL, "set_params: " + why);
    const covox_params &o = ctx->p;
    if (p->voxel_size != o.voxel_size || p->trunc_vox != o.trunc_vox || p->max_range != o.max_range ||
        p->d_max != o.d_max || p->block_capacity != o.block_capacity || p->precision != o.precision)
        return fail(ctx, COVOX_EINVAL, "set_params: storage-shaping parameters cannot change");
    if (p->w_reg != o.w_reg)
        for (covox_submap *s : submaps_of(ctx)) s->pts_version = 0;
    ctx->p = *p;
    if (p->integrator == COVOX_RAYCAST) return ensure_ray_acc(ctx);
    return COVOX_OK;
}

int covox_set_stream(covox_ctx *ctx, void *hip_stream)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "set_stream");
    if (!ctx) return COVOX_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return COVOX_OK;
}

int covox_sync(covox_ctx *ctx)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "sync");
    if (!ctx) return COVOX_EINVAL;
    int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync");
    if (rc) return rc;
    for (covox_submap *s : submaps_of(ctx)) {
        rc = check_status_after_sync(ctx, s);
        if (rc) return rc;
    }
    return COVOX_OK;
}

int covox_submap_create(covox_ctx *ctx, const double T_world_submap[16], covox_submap **out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "submap_create");
    if (!ctx || !T_world_submap || !out) return fail(ctx, COVOX_EINVAL, "submap_create: null argument");
    if (!rigid_pose(T_world_submap)) return fail(ctx, COVOX_EINVAL, "submap_create: pose is not rigid");
    *out = nullptr;
    covox_submap *s = new covox_submap();
    s->ctx = ctx;
    memcpy(s->T_ws, T_world_submap, sizeof(s->T_ws));
    s->cap = ctx->p.block_capacity;
    int64_t t = 1;
    while (t < 2 * s->cap) t <<= 1;
    s->tcap = t;
    const size_t es = ctx->p.precision == COVOX_FP16 ? 2 : 4;
    const size_t nvox = (size_t)s->cap * 512;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void **)&s->keys, sizeof(uint64_t) * s->cap);
    if (e == hipSuccess) e = hipMalloc(&s->D, es * nvox);
    if (e == hipSuccess) e = hipMalloc(&s->W, es * nvox);
    if (e == hipSuccess) e = hipMalloc((void **)&s->phi, sizeof(float) * nvox);
    if (e == hipSuccess) e = hipMalloc((void **)&s->tkeys, sizeof(uint64_t) * s->tcap);
    if (e == hipSuccess) e = hipMalloc((void **)&s->tvals, sizeof(uint32_t) * s->tcap);
    if (e == hipSuccess) e = hipMalloc((void **)&s->meta, sizeof(SubmapMeta));
    if (e == hipSuccess) e = hipMalloc((void **)&s->stamp, sizeof(uint32_t) * s->cap);
    if (e == hipSuccess) e = hipMalloc((void **)&s->dirty, (size_t)4 * ((s->cap + 3) / 4));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->pin_nb, sizeof(uint64_t), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
        *s->pin_nb = 0;
        e = hipHostGetDevicePointer((void **)&s->pin_nb_dev, (void *)s->pin_nb, 0);
    }
    if (e != hipSuccess) {
        covox_submap_destroy(s);
        return fail(ctx, COVOX_EHIP, std::string("submap_create: ") + hipGetErrorString(e));
    }
    submaps_of(ctx).push_back(s);
    fill_u32(ctx->stream, s->stamp, 0u, s->cap);  // frame-batch stamps (never reset)
    fill_u32(ctx->stream, (uint32_t *)s->dirty, 0u, (s->cap + 3) / 4);
    int rc = covox_submap_reset(ctx, s);
    if (rc) {
        covox_submap_destroy(s);
        return rc;
    }
    *out = s;
    return COVOX_OK;
}

void covox_submap_destroy(covox_submap *s)
{
    if (!s) return;
    if (s->ctx) {
        (void)hipStreamSynchronize(s->ctx->stream);
        auto &subs = submaps_of(s->ctx);
        subs.erase(std::remove(subs.begin(), subs.end(), s), subs.end());
    }
    for (void *p : {(void *)s->keys, s->D, s->W, (void *)s->phi, (void *)s->tkeys, (void *)s->tvals, (void *)s->meta,
                    (void *)s->page, (void *)s->pts, (void *)s->wf_k, (void *)s->wf_p, (void *)s->wf_wn})
        if (p) (void)hipFree(p);
    if (s->stamp) (void)hipFree(s->stamp);
    if (s->dirty) (void)hipFree(s->dirty);
    if (s->pin_nb) (void)hipHostFree((void *)s->pin_nb);
    delete s;
}

int covox_submap_reset(covox_ctx *ctx, covox_submap *s)
{
    if (!ctx || !s) return fail(ctx, COVOX_EINVAL, "submap_reset: null argument");
    capture_touch(ctx, s, 0);
    fill_u64(ctx->stream, s->tkeys, kEmpty, s->tcap);
    hipLaunchKernelGGL(k_reset_meta, dim3(1), dim3(1), 0, ctx->stream, s->meta);
    int rc = hip_check(ctx, hipGetLastError(), "submap_reset");
    if (rc) return rc;
    s->nb_upper = 0;
    s->bound_valid = false;
    s->version++;
    s->n_pts = 0;
    s->esdf_exact = false;
    return wavefront_reset(ctx, s);
}

int covox_integrate_depth(covox_ctx *ctx, covox_submap *s, const float *depth_dev, int32_t H, int32_t W,
                          const float K[4], const double T_world_cam[16])
{
    if (!ctx || !s) return fail(ctx, COVOX_EINVAL, "integrate: null argument");
    capture_touch(ctx, s, 1);
    bool maybe_full = false;
    int rc = integrate_frame(ctx, s, depth_dev, H, W, K, T_world_cam, &maybe_full);
    if (rc) return rc;
    if (maybe_full) return check_status_after_sync(ctx, s);
    return COVOX_OK;
}

int covox_integrate_depth_batch(covox_ctx *ctx, covox_submap *s, const float *depths_dev, int32_t F, int32_t H,
                                int32_t W, const float K[4], const double *T_world_cam)
{
    if (!ctx || !s || !depths_dev || !T_world_cam || F < 0) return fail(ctx, COVOX_EINVAL, "integrate_batch: bad argument");
    capture_touch(ctx, s, 1);
    return integrate_frames(ctx, s, depths_dev, F, H, W, K, T_world_cam);
}

namespace {

// The second stream and the events of a pipelined map_sequence, created
// once per context (the stream last, so that its presence means all exist).
int ensure_pipeline(covox_ctx *ctx)
{
    if (ctx->esdf_stream) return COVOX_OK;
    int rc;
    for (hipEvent_t *e : {&ctx->ev_fork, &ctx->ev_paged, &ctx->ev_join, &ctx->ev_free[0], &ctx->ev_free[1]})
        if (!*e && (rc = hip_check(ctx, hipEventCreateWithFlags(e, hipEventDisableTiming), "pipeline event")))
            return rc;
    return hip_check(ctx, hipStreamCreateWithFlags(&ctx->esdf_stream, hipStreamNonBlocking), "esdf stream");
}

}  // namespace

int covox_map_sequence(covox_ctx *ctx, covox_submap *s, const float *depths_dev, int32_t F, int32_t H, int32_t W,
                       const float K[4], const double *T_world_cam, int32_t esdf_every)
{
    if (!ctx || !s || !depths_dev || !T_world_cam || F < 0) return fail(ctx, COVOX_EINVAL, "map_sequence: bad argument");
    capture_touch(ctx, s, 1);
    // frames between ESDF updates go through the batched integration
    const int32_t step = esdf_every > 0 ? esdf_every : F;
    // With an exact ESDF update after every chunk, the page kernel of each
    // update (the last ESDF kernel that reads the TSDF) runs right after the
    // chunk's integration on the context stream, and its EDT passes run on a
    // second stream while the next chunk is integrated.  The page kernels
    // alternate between two scratch slots, so that the one of chunk k + 1
    // does not wait for the passes of chunk k.  The results are those of the
    // calls in sequence.
    const bool pipe = esdf_every > 0 && F > step && ctx->p.esdf_mode == COVOX_ESDF_EXACT &&
                      (ctx->esdf_stream || !ctx->capturing);
    if (!pipe) {
        for (int32_t f0 = 0; f0 < F; f0 += step) {
            const int32_t n = std::min(step, F - f0);
            int rc = integrate_frames(ctx, s, depths_dev + (size_t)f0 * H * W, n, H, W, K, T_world_cam + 16 * f0);
            if (rc) return rc;
            rc = update_esdf(ctx, s);
            if (rc) return rc;
        }
        return COVOX_OK;
    }
    int rc = ensure_pipeline(ctx);
    if (rc) return rc;
    hipStream_t base = ctx->stream, aux = ctx->esdf_stream;
    if ((rc = hip_check(ctx, hipEventRecord(ctx->ev_fork, base), "fork")) ||
        (rc = hip_check(ctx, hipStreamWaitEvent(aux, ctx->ev_fork, 0), "fork wait")))
        return rc;
    int rc_loop = COVOX_OK;
    bool in_flight[2] = {false, false};  // an update's passes were enqueued on the slot
    bool prev_read_page = false;         // the last update's passes read the page
    int k = 0;
    for (int32_t f0 = 0; f0 < F && !rc_loop; f0 += step, ++k) {
        const int32_t n = std::min(step, F - f0);
        rc_loop = integrate_frames(ctx, s, depths_dev + (size_t)f0 * H * W, n, H, W, K, T_world_cam + 16 * f0);
        if (rc_loop) break;
        const int slot = k & 1;
        // the slot is free once the passes of the update two chunks back are
        // done; the page, once the last update's passes are, if they read it
        if (in_flight[slot] && (rc_loop = hip_check(ctx, hipStreamWaitEvent(base, ctx->ev_free[slot], 0), "slot wait")))
            break;
        if (prev_read_page && in_flight[1 - slot] &&
            (rc_loop = hip_check(ctx, hipStreamWaitEvent(base, ctx->ev_free[1 - slot], 0), "page wait")))
            break;
        ctx->esdf_slot = slot;
        ctx->esdf_edt_stream = aux;
        ctx->esdf_used_page = false;
        rc_loop = update_esdf(ctx, s);
        ctx->esdf_edt_stream = nullptr;
        ctx->esdf_slot = 0;
        if (rc_loop) break;
        prev_read_page = ctx->esdf_used_page;
        if ((rc_loop = hip_check(ctx, hipEventRecord(ctx->ev_free[slot], aux), "slot free"))) break;
        in_flight[slot] = true;
    }
    // join, after an error too: later work on the context stream follows all of it
    if ((rc = hip_check(ctx, hipEventRecord(ctx->ev_join, aux), "join")) ||
        (rc = hip_check(ctx, hipStreamWaitEvent(base, ctx->ev_join, 0), "join wait"))) {
        if (!rc_loop) rc_loop = rc;
    }
    return rc_loop;
}

int covox_update_esdf_batch(covox_ctx *ctx, covox_submap *const *subs, int32_t n)
{
    if (!ctx || (!subs && n > 0) || n < 0) return fail(ctx, COVOX_EINVAL, "update_esdf_batch: bad argument");
    for (int32_t i = 0; i < n; ++i)
        if (!subs[i]) return fail(ctx, COVOX_EINVAL, "update_esdf_batch: null submap");
    for (int32_t i = 0; i < n; ++i) capture_touch(ctx, subs[i], 2);
    return update_esdf_batch(ctx, subs, n);
}

int covox_update_esdf(covox_ctx *ctx, covox_submap *s)
{
    if (!ctx || !s) return fail(ctx, COVOX_EINVAL, "update_esdf: null argument");
    capture_touch(ctx, s, 2);
    return update_esdf(ctx, s);
}

int covox_align_submaps(covox_ctx *ctx, const covox_submap *A, const covox_submap *B, const double T_init_A_B[16],
                        double T_out[16], double *cost, covox_align_stats *stats)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_submaps");
    if (!ctx || !T_init_A_B || !T_out || !cost) return fail(ctx, COVOX_EINVAL, "align: null argument");
    if (!rigid_pose(T_init_A_B)) return fail(ctx, COVOX_EINVAL, "align: T_init is not rigid");
    int rc = prepare_pair(ctx, A, B);
    if (rc) return rc;
    AlignProblem pr = make_problem(ctx, A, B, T_init_A_B, ctx->p.max_iter);
    AlignResult res;
    if ((rc = run_alignment(ctx, &pr, 1, &res))) return rc;
    memcpy(T_out, res.T, sizeof(res.T));
    *cost = res.cost;
    fill_stats(stats, B->n_pts, res, 0);
    return res.status;
}

int covox_align_multistart(covox_ctx *ctx, const covox_submap *A, const covox_submap *B, const double T_init_A_B[16],
                           int32_t n_starts, double T_out[16], double *cost, covox_align_stats *stats)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_multistart");
    if (!ctx || !T_init_A_B || !T_out || !cost || n_starts < 1) return fail(ctx, COVOX_EINVAL, "align: bad argument");
    if (!rigid_pose(T_init_A_B)) return fail(ctx, COVOX_EINVAL, "align: T_init is not rigid");
    int rc = prepare_pair(ctx, A, B);
    if (rc) return rc;
    std::vector<AlignProblem> prs(n_starts);
    for (int k = 0; k < n_starts; ++k) {
        double S[16];
        start_pose(T_init_A_B, B->pbar, k, n_starts, S);
        prs[k] = make_problem(ctx, A, B, S, ctx->p.max_iter);
    }
    std::vector<AlignResult> res(n_starts);
    if ((rc = run_alignment(ctx, prs.data(), n_starts, res.data()))) return rc;
    const int best = select_start(res.data(), n_starts);
    if (best < 0) {
        memcpy(T_out, T_init_A_B, sizeof(double) * 16);
        *cost = INFINITY;
        if (stats) { memset(stats, 0, sizeof(*stats)); stats->n_points = B->n_pts; stats->status = COVOX_EDEGENERATE; stats->best_start = -1; }
        return COVOX_EDEGENERATE;
    }
    memcpy(T_out, res[best].T, sizeof(double) * 16);
    *cost = res[best].cost;
    fill_stats(stats, B->n_pts, res[best], best);
    return res[best].status;
}

int covox_align_batch(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts, double *T_out,
                      double *cost, covox_align_stats *stats)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_batch");
    if (!ctx || !pairs || n < 0 || n_starts < 1 || !T_out || !cost) return fail(ctx, COVOX_EINVAL, "align_batch: bad argument");
    int rc;
    for (int i = 0; i < n; ++i) {
        if (!rigid_pose(pairs[i].T_init_A_B)) return fail(ctx, COVOX_EINVAL, "align_batch: T_init is not rigid");
        if ((rc = prepare_pair(ctx, pairs[i].A, pairs[i].B))) return rc;
    }
    std::vector<AlignProblem> prs((size_t)n * n_starts);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n_starts; ++k) {
            double S[16];
            if (n_starts == 1) memcpy(S, pairs[i].T_init_A_B, sizeof(S));
            else start_pose(pairs[i].T_init_A_B, pairs[i].B->pbar, k, n_starts, S);
            prs[(size_t)i * n_starts + k] = make_problem(ctx, pairs[i].A, pairs[i].B, S, ctx->p.max_iter);
        }
    std::vector<AlignResult> res(prs.size());
    if ((rc = run_alignment(ctx, prs.data(), (int)prs.size(), res.data()))) return rc;
    std::vector<double> T0((size_t)16 * n);
    std::vector<int64_t> np(n);
    for (int i = 0; i < n; ++i) {
        memcpy(&T0[16 * (size_t)i], pairs[i].T_init_A_B, sizeof(double) * 16);
        np[i] = pairs[i].B->n_pts;
    }
    finish_pairs(n, n_starts, res.data(), T0.data(), np.data(), T_out, cost, stats);
    return COVOX_OK;
}

int covox_align_prepare(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts, covox_align_set **out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_prepare");
    if (!ctx || !pairs || !out || n < 1 || n_starts < 1 || (int64_t)n * n_starts > INT32_MAX / 2)
        return fail(ctx, COVOX_EINVAL, "align_prepare: bad argument");
    *out = nullptr;
    int rc;
    for (int i = 0; i < n; ++i) {
        if (!rigid_pose(pairs[i].T_init_A_B)) return fail(ctx, COVOX_EINVAL, "align_prepare: T_init is not rigid");
        if ((rc = prepare_pair(ctx, pairs[i].A, pairs[i].B))) return rc;
    }
    const int m = n * n_starts;
    const size_t pbytes = sizeof(AlignProblem) * m + sizeof(int32_t) * m;
    std::vector<char> stage(pbytes);
    AlignProblem *prs = (AlignProblem *)stage.data();
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n_starts; ++k) {
            double S[16];
            if (n_starts == 1) memcpy(S, pairs[i].T_init_A_B, sizeof(S));
            else start_pose(pairs[i].T_init_A_B, pairs[i].B->pbar, k, n_starts, S);
            prs[(size_t)i * n_starts + k] = make_problem(ctx, pairs[i].A, pairs[i].B, S, ctx->p.max_iter);
        }
    align_order(prs, m, (int32_t *)(stage.data() + sizeof(AlignProblem) * m));
    covox_align_set *set = new covox_align_set();
    set->ctx = ctx;
    set->n = n;
    set->n_starts = n_starts;
    set->launch = align_launch_of(ctx);
    set->T_init.resize((size_t)16 * n);
    set->n_points.resize(n);
    for (int i = 0; i < n; ++i) {
        memcpy(&set->T_init[16 * (size_t)i], pairs[i].T_init_A_B, sizeof(double) * 16);
        set->n_points[i] = pairs[i].B->n_pts;
        for (const covox_submap *q : {pairs[i].A, pairs[i].B}) {
            bool seen = false;
            for (const auto &f : set->frozen) seen = seen || f.s == q;
            if (!seen) set->frozen.push_back(AlignFrozen{q, q->version});
        }
    }
    // results before the first launch (or replay): each start as given, no
    // update made, NOT_CONVERGED
    std::vector<AlignResult> init(m);
    for (int q = 0; q < m; ++q) {
        memset(&init[q], 0, sizeof(AlignResult));
        memcpy(init[q].T, prs[q].T, sizeof(init[q].T));
        init[q].cost = INFINITY;
        init[q].status = COVOX_NOT_CONVERGED;
    }
    hipError_t e = hipMalloc(&set->dev, pbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&set->dres, sizeof(AlignResult) * m);
    if (e == hipSuccess) e = hipMemcpyAsync(set->dev, stage.data(), pbytes, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(set->dres, init.data(), sizeof(AlignResult) * m, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        if (set->dev) (void)hipFree(set->dev);
        if (set->dres) (void)hipFree(set->dres);
        delete set;
        return hip_check(ctx, e, "align_prepare");
    }
    ctx->align_sets.push_back(set);
    *out = set;
    return COVOX_OK;
}

int covox_align_launch(covox_ctx *ctx, covox_align_set *set)
{
    if (!ctx || !set || set->ctx != ctx) return fail(ctx, COVOX_EINVAL, "align_launch: bad argument");
    for (const auto &f : set->frozen)
        if (f.s->version != f.version)
            return fail(ctx, COVOX_EINVAL, "align_launch: a submap of the set changed since covox_align_prepare");
    if (ctx->capturing)
        for (const auto &f : set->frozen) ctx->cap_frozen.push_back(f);
    const int m = set->n * set->n_starts;
    return launch_alignment(ctx, (const AlignProblem *)set->dev,
                            (const int32_t *)((const char *)set->dev + sizeof(AlignProblem) * m), m, set->dres,
                            set->launch);
}

int covox_align_collect(covox_ctx *ctx, covox_align_set *set, double *T_out, double *cost, covox_align_stats *stats)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_collect");
    if (!ctx || !set || set->ctx != ctx || !T_out || !cost) return fail(ctx, COVOX_EINVAL, "align_collect: bad argument");
    const int m = set->n * set->n_starts;
    std::vector<AlignResult> res(m);
    int rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(res.data(), set->dres, sizeof(AlignResult) * m, hipMemcpyDeviceToHost,
                                            ctx->stream),
                        "align_collect copy")))
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "align_collect sync"))) return rc;
    finish_pairs(set->n, set->n_starts, res.data(), set->T_init.data(), set->n_points.data(), T_out, cost, stats);
    return COVOX_OK;
}

void covox_align_set_destroy(covox_align_set *set)
{
    if (!set) return;
    covox_ctx *ctx = set->ctx;
    if (ctx) {
        (void)hipStreamSynchronize(ctx->stream);
        auto &v = ctx->align_sets;
        v.erase(std::remove(v.begin(), v.end(), set), v.end());
        for (void *p : {set->dev, (void *)set->dres}) {
            if (!p) continue;
            if (ctx->capturing || ctx->n_graphs > 0) ctx->deferred.push_back(p);  // a graph may still name it
            else (void)hipFree(p);
        }
    }
    delete set;
}

int covox_normal_equations(covox_ctx *ctx, const covox_submap *A, const covox_submap *B, const double T_A_B[16],
                           double out[29])
{
    COVOX_NOT_DURING_CAPTURE(ctx, "normal_equations");
    if (!ctx || !T_A_B || !out) return fail(ctx, COVOX_EINVAL, "normal_equations: null argument");
    int rc = prepare_pair(ctx, A, B);
    if (rc) return rc;
    AlignProblem pr = make_problem(ctx, A, B, T_A_B, 0);
    AlignResult res;
    if ((rc = run_alignment(ctx, &pr, 1, &res))) return rc;
    memcpy(out, res.ne, sizeof(res.ne));
    return COVOX_OK;
}

void covox_default_pgo_cfg(covox_pgo_cfg *cfg)
{
    if (cfg) covox_default_pgo_cfg_impl(cfg);
}

int covox_pgo_solve(covox_ctx *ctx, covox_submap *const *subs, int32_t n, double *x, const int32_t *reg_pairs,
                    int32_t n_reg, const covox_pose_factor *factors, int32_t n_fac, const covox_pgo_cfg *cfg,
                    covox_pgo_stats *stats)
{
    if (!ctx) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(ctx, "pgo_solve");
    return pgo_solve(ctx, subs, n, x, reg_pairs, n_reg, factors, n_fac, cfg, stats);
}

int covox_hash_insert(covox_ctx *ctx, uint64_t *table_keys, uint32_t *table_vals, int64_t capacity,
                      int64_t n_present, const uint64_t *keys, int64_t n, uint32_t val_base, int64_t *stats)
{
    if (!ctx) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(ctx, "hash_insert");
    return hash_insert_keys(ctx, table_keys, table_vals, capacity, n_present, keys, n, val_base, stats);
}

int covox_submap_info_get(covox_ctx *ctx, const covox_submap *s, covox_submap_info *out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "submap_info_get");
    if (!ctx || !s || !out) return fail(ctx, COVOX_EINVAL, "submap_info: null argument");
    SubmapMeta m;
    int rc = read_meta(ctx, s, &m);
    if (rc) return rc;
    out->n_blocks = m.n_blocks;
    out->block_capacity = s->cap;
    out->table_capacity = s->tcap;
    out->n_updates = (int64_t)m.n_updates;
    for (int a = 0; a < 3; ++a) { out->bbox_min[a] = m.bmin[a]; out->bbox_max[a] = m.bmax[a]; }
    out->precision = ctx->p.precision;
    out->status = m.status;
    return COVOX_OK;
}

int64_t covox_export_blocks(covox_ctx *ctx, const covox_submap *s, uint64_t *keys, uint32_t *home, float *D, float *W,
                            float *phi, int64_t cap)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "export_blocks");
    if (!ctx || !s || cap < 0) return fail(ctx, COVOX_EINVAL, "export_blocks: bad argument");
    SubmapMeta m;
    int rc = read_meta(ctx, s, &m);
    if (rc) return rc;
    const int64_t n = std::min<int64_t>(m.n_blocks, cap);
    if (n <= 0) return 0;
    std::vector<uint64_t> k(n);
    if ((rc = hip_check(ctx, hipMemcpy(k.data(), s->keys, sizeof(uint64_t) * n, hipMemcpyDeviceToHost), "keys copy")))
        return rc;
    if (keys) memcpy(keys, k.data(), sizeof(uint64_t) * n);
    if (home)
        for (int64_t j = 0; j < n; ++j) home[j] = (uint32_t)(mix64(k[j]) & (uint64_t)(s->tcap - 1));
    const size_t nv = (size_t)n * 512;
    auto copy_field = [&](const void *src, float *dst) -> int {
        if (!dst) return COVOX_OK;
        if (ctx->p.precision == COVOX_FP16) {
            std::vector<__half> h(nv);
            int r = hip_check(ctx, hipMemcpy(h.data(), src, sizeof(__half) * nv, hipMemcpyDeviceToHost), "field copy");
            if (r) return r;
            for (size_t i = 0; i < nv; ++i) dst[i] = __half2float(h[i]);
            return COVOX_OK;
        }
        return hip_check(ctx, hipMemcpy(dst, src, sizeof(float) * nv, hipMemcpyDeviceToHost), "field copy");
    };
    if ((rc = copy_field(s->D, D))) return rc;
    if ((rc = copy_field(s->W, W))) return rc;
    if (phi && (rc = hip_check(ctx, hipMemcpy(phi, s->phi, sizeof(float) * nv, hipMemcpyDeviceToHost), "phi copy")))
        return rc;
    return n;
}

int64_t covox_export_points(covox_ctx *ctx, const covox_submap *B, float *pts, int64_t cap)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "export_points");
    if (!ctx || !B || cap < 0) return fail(ctx, COVOX_EINVAL, "export_points: bad argument");
    int rc = extract_points(ctx, B);
    if (rc) return rc;
    const int64_t n = std::min(cap, B->n_pts);
    if (pts && n > 0 &&
        (rc = hip_check(ctx, hipMemcpy(pts, B->pts, sizeof(float) * 3 * n, hipMemcpyDeviceToHost), "points copy")))
        return rc;
    return B->n_pts;
}

int covox_summaries(covox_ctx *ctx, const covox_summary_req *reqs, int32_t n)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "summaries");
    if (!ctx || (!reqs && n > 0) || n < 0) return fail(ctx, COVOX_EINVAL, "summaries: bad argument");
    std::vector<SummaryReq> rq(n);
    for (int32_t i = 0; i < n; ++i) {
        const covox_summary_req &r = reqs[i];
        if (!r.s || !r.out_dev || (r.channel != 0 && r.channel != 2) || !(r.cell > 0) || !rigid_pose(r.T_submap_grid))
            return fail(ctx, COVOX_EINVAL, "summaries: bad request");
        if (r.s->esdf_version != r.s->version)
            return fail(ctx, COVOX_EINVAL, "summaries: the ESDF of a submap is out of date");
        rq[i].phi = r.s->phi;
        rq[i].page = r.s->page;
        rq[i].meta = r.s->meta;
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 4; ++c) rq[i].T[4 * a + c] = (float)r.T_submap_grid[4 * a + c];
        rq[i].cell = (float)r.cell;
        rq[i].chan = r.channel;
        rq[i].out = r.out_dev;
    }
    int rc = run_summaries(ctx, rq.data(), n);
    if (rc) return rc;
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "summaries sync");
}

int covox_net_create(covox_ctx *ctx, uint64_t seed, covox_net **out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "net_create");
    if (!ctx || !out) return fail(ctx, COVOX_EINVAL, "net_create: null argument");
    return net_create(ctx, seed, out);
}

void covox_net_destroy(covox_net *net) { net_destroy(net); }

int64_t covox_net_num_params(const covox_net *net) { return net ? net_num_params(net) : COVOX_EINVAL; }

int covox_net_get_params(covox_net *net, float *host, int64_t n)
{
    if (!net || !net_ctx(net) || !host) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(net_ctx(net), "net_get_params");
    return net_get_params(net, host, n);
}

int covox_net_set_params(covox_net *net, const float *host, int64_t n)
{
    if (!net || !net_ctx(net) || !host) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(net_ctx(net), "net_set_params");
    return net_set_params(net, host, n);
}

int covox_net_forward(covox_net *net, const float *x_dev, int32_t n, float *out_dev)
{
    if (!net || !net_ctx(net) || !x_dev || !out_dev || n <= 0) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(net_ctx(net), "net_forward");
    return net_forward_api(net, x_dev, n, out_dev);
}

int covox_net_forward_noalloc(covox_net *net, const float *x_dev, int32_t n, float *out_dev)
{
    if (!net || !net_ctx(net) || !x_dev || !out_dev || n <= 0) return COVOX_EINVAL;
    return net_forward_noalloc(net, x_dev, n, out_dev);
}

int covox_net_train_step(covox_net *net, const float *x_dev, const float *y_dev, int32_t n, float lr, float trans_scale,
                         float *loss_host)
{
    if (!net || !net_ctx(net) || !x_dev || !y_dev || n <= 0 || !(trans_scale > 0)) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(net_ctx(net), "net_train_step");
    return net_train_step(net, x_dev, y_dev, n, lr, trans_scale, loss_host);
}

int covox_net_gradients(covox_net *net, const float *x_dev, const float *y_dev, int32_t n, float trans_scale,
                        float *grad_host, float *loss_host)
{
    if (!net || !net_ctx(net) || !x_dev || !y_dev || !grad_host || n <= 0 || !(trans_scale > 0)) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(net_ctx(net), "net_gradients");
    return net_grads(net, x_dev, y_dev, n, trans_scale, grad_host, loss_host);
}

namespace {

// T_A_grid = Trans(c_A): the summary grid of a pair is centred on the
// centroid of A's registration points.
void grid_of(const covox_submap *A, double *G)
{
    const double Gv[16] = {1, 0, 0, A->pbar[0], 0, 1, 0, A->pbar[1], 0, 0, 1, A->pbar[2], 0, 0, 0, 1};
    ::memcpy(G, Gv, sizeof(Gv));
}

// Correction C = (Rz(yaw), t) in grid coordinates.
void correction(double tx, double ty, double tz, double yaw, double *C)
{
    const double c = cos(yaw), s = sin(yaw);
    const double Cv[16] = {c, -s, 0, tx, s, c, 0, ty, 0, 0, 1, tz, 0, 0, 0, 1};
    ::memcpy(C, Cv, sizeof(Cv));
}

// out = G X G^-1 Y for rigid 4x4 matrices (last row exact).
void conj_mul(const double *G, const double *X, const double *Y, double *out)
{
    double Gi[16], A1[16], A2[16];
    rigid_inverse_h(G, Gi);
    mat_mul4(G, X, A1);
    mat_mul4(A1, Gi, A2);
    mat_mul4(A2, Y, out);
    out[12] = 0; out[13] = 0; out[14] = 0; out[15] = 1;
}

// Both ESDFs current, A's registration points (and centroid) extracted.
int prepare_learned(covox_ctx *ctx, const covox_pair *pairs, int n, const char *what)
{
    int rc;
    for (int i = 0; i < n; ++i) {
        const covox_pair &pr = pairs[i];
        if (!pr.A || !pr.B) return fail(ctx, COVOX_EINVAL, std::string(what) + ": null submap");
        if (!rigid_pose(pr.T_init_A_B)) return fail(ctx, COVOX_EINVAL, std::string(what) + ": pose is not rigid");
        if ((rc = prepare_pair(ctx, pr.A, pr.B))) return rc;
        if (pr.B->esdf_version != pr.B->version)
            return fail(ctx, COVOX_EINVAL, std::string(what) + ": the ESDF of B is out of date");
        if ((rc = extract_points(ctx, pr.A))) return rc;
    }
    return COVOX_OK;
}

// Summaries of m pairs through their priors into the network input block
// (A on channels 0-1, B on 2-3); G receives the m grid poses T_A_grid.
int pair_summaries(covox_ctx *ctx, const covox_pair *pairs, int m, double cell, double *G)
{
    int rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->net_in, &ctx->net_in_cap, (int64_t)m * 32768 * 4, sizeof(float),
                            "net input")))
        return rc;
    std::vector<SummaryReq> rq(2 * m);
    for (int k = 0; k < m; ++k) {
        const covox_pair &pr = pairs[k];
        double *Gk = G + 16 * k, inv[16], TB[16];
        grid_of(pr.A, Gk);
        rigid_inverse_h(pr.T_init_A_B, inv);
        mat_mul4(inv, Gk, TB);  // T_B_grid = T_init^-1 T_A_grid
        const double *Ts[2] = {Gk, TB};
        const covox_submap *ss[2] = {pr.A, pr.B};
        for (int side = 0; side < 2; ++side) {
            SummaryReq &r = rq[2 * k + side];
            r.phi = ss[side]->phi;
            r.page = ss[side]->page;
            r.meta = ss[side]->meta;
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 4; ++c) r.T[4 * a + c] = (float)Ts[side][4 * a + c];
            r.cell = (float)cell;
            r.chan = 2 * side;
            r.out = ctx->net_in + (int64_t)k * 32768 * 4;
        }
    }
    return run_summaries(ctx, rq.data(), 2 * m);
}

// Network proposals T_A_grid C T_A_grid^-1 T_init of m <= 256 pairs
// (host, m x 16).  Synchronous.
int propose_chunk(covox_ctx *ctx, covox_net *net, const covox_pair *pairs, int m, double cell, double *Tp)
{
    int rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->net_out, &ctx->net_out_cap, (int64_t)m * 5, sizeof(float),
                            "net output")))
        return rc;
    std::vector<double> G((size_t)16 * m);
    if ((rc = pair_summaries(ctx, pairs, m, cell, G.data()))) return rc;
    if ((rc = net_forward_api(net, ctx->net_in, m, ctx->net_out))) return rc;
    std::vector<float> outs((size_t)5 * m);
    if ((rc = hip_check(ctx, hipMemcpyAsync(outs.data(), ctx->net_out, sizeof(float) * 5 * m, hipMemcpyDeviceToHost,
                                            ctx->stream), "net output copy")))
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "net sync"))) return rc;
    for (int k = 0; k < m; ++k) {
        const float *o = &outs[5 * k];
        double C[16];
        correction(o[0], o[1], o[2], atan2((double)o[4], (double)o[3]), C);
        conj_mul(&G[16 * k], C, pairs[k].T_init_A_B, Tp + 16 * k);
    }
    return COVOX_OK;
}

constexpr int kLearnChunk = 256;

// The proposal of a pair to refine, from the sums at each proposal: among
// those with at least n_min residuals and at least half the largest count,
// the least cost (ties: smallest k); 0 when none qualifies.
int pick_proposal(const AlignResult *r, int n, int n_min)
{
    int64_t nmax = 0;
    for (int k = 0; k < n; ++k)
        if (r[k].n_used >= n_min) nmax = std::max(nmax, r[k].n_used);
    int best = -1;
    for (int k = 0; k < n; ++k) {
        if (r[k].n_used < n_min || 2 * r[k].n_used < nmax) continue;
        if (best < 0 || r[k].cost < r[best].cost) best = k;
    }
    return best < 0 ? 0 : best;
}

// The pairs with their priors turned about the summary grid centre: item
// j n_rot + k carries T_A_grid Rz(2 pi k / n_rot) T_A_grid^-1 T_init of pair
// j (k = 0: the prior itself).
std::vector<covox_pair> turned_pairs(const covox_pair *pairs, int m, int n_rot)
{
    std::vector<covox_pair> out((size_t)m * n_rot);
    for (int j = 0; j < m; ++j)
        for (int k = 0; k < n_rot; ++k) {
            covox_pair &q = out[(size_t)j * n_rot + k];
            q = pairs[j];
            if (k == 0) continue;
            const double a = 2.0 * M_PI * (double)k / (double)n_rot;
            double G[16], Gi[16], R[16] = {cos(a), -sin(a), 0, 0, sin(a), cos(a), 0, 0, 0, 0, 1, 0, 0, 0, 0, 1}, M[16];
            grid_of(pairs[j].A, G);
            rigid_inverse_h(G, Gi);
            mat_mul4(G, R, M);
            mat_mul4(M, Gi, M);
            mat_mul4(M, pairs[j].T_init_A_B, q.T_init_A_B);
            q.T_init_A_B[12] = 0; q.T_init_A_B[13] = 0; q.T_init_A_B[14] = 0; q.T_init_A_B[15] = 1;
        }
    return out;
}

// Uniform draw in [0, 1) number k of item `item` (SplitMix64 of the seed
// and a counter).
double draw(uint64_t seed, uint64_t item, int k)
{
    const uint64_t z = mix64(seed ^ mix64(item * 16u + (uint64_t)k + 1u));
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

int covox_propose(covox_ctx *ctx, covox_net *net, const covox_pair *pairs, int32_t n, double cell, int32_t n_rot,
                  double *T_prop)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "propose");
    if (!ctx || !net || net_ctx(net) != ctx || (!pairs && n > 0) || n < 0 || !(cell > 0) || (!T_prop && n > 0) ||
        n_rot < 1 || n_rot > kLearnChunk)
        return fail(ctx, COVOX_EINVAL, "propose: bad argument");
    int rc = prepare_learned(ctx, pairs, n, "propose");
    if (rc) return rc;
    const int per = kLearnChunk / n_rot;
    for (int i0 = 0; i0 < n; i0 += per) {
        const int m = std::min(per, n - i0);
        const std::vector<covox_pair> tp = turned_pairs(pairs + i0, m, n_rot);
        if ((rc = propose_chunk(ctx, net, tp.data(), m * n_rot, cell, T_prop + (size_t)16 * n_rot * i0))) return rc;
    }
    return COVOX_OK;
}

int covox_train_proposal(covox_ctx *ctx, covox_net *net, const covox_train_cfg *cfg, const covox_pair *pairs,
                         int32_t n, float *loss_host)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "train_proposal");
    if (!ctx || !net || net_ctx(net) != ctx || !cfg || !pairs || n <= 0 || cfg->steps < 0 || cfg->batch < 1 ||
        cfg->batch > kLearnChunk || !(cfg->cell > 0) || !(cfg->trans_scale > 0) || !(cfg->lr >= 0) || !(cfg->trans_xy >= 0) ||
        !(cfg->trans_z >= 0) || !(cfg->yaw >= 0) || !(cfg->tilt >= 0))
        return fail(ctx, COVOX_EINVAL, "train_proposal: bad argument");
    int rc = prepare_learned(ctx, pairs, n, "train_proposal");
    if (rc) return rc;
    const int B = cfg->batch;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->train_y, &ctx->train_y_cap, (int64_t)B * 5, sizeof(float),
                            "training targets")))
        return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->loss_hist, &ctx->loss_hist_cap, std::max(1, cfg->steps),
                            sizeof(float), "training losses")))
        return rc;
    std::vector<covox_pair> items(B);
    std::vector<float> y((size_t)5 * B);
    std::vector<double> G((size_t)16 * B);
    for (int32_t st = 0; st < cfg->steps; ++st) {
        for (int b = 0; b < B; ++b) {
            const uint64_t item = (uint64_t)st * (uint64_t)B + (uint64_t)b;
            const int j = std::min(n - 1, (int)(draw(cfg->seed, item, 0) * n));
            const double tx = (2 * draw(cfg->seed, item, 1) - 1) * cfg->trans_xy;
            const double ty = (2 * draw(cfg->seed, item, 2) - 1) * cfg->trans_xy;
            const double tz = (2 * draw(cfg->seed, item, 3) - 1) * cfg->trans_z;
            const double yaw = (2 * draw(cfg->seed, item, 4) - 1) * cfg->yaw;
            const double roll = (2 * draw(cfg->seed, item, 5) - 1) * cfg->tilt;
            const double pitch = (2 * draw(cfg->seed, item, 6) - 1) * cfg->tilt;
            // prior T_init = G C^-1 G^-1 T_gt E, E = Rx(roll) Ry(pitch) (not predicted)
            double Gj[16], C[16], Ci[16], E[16], TE[16];
            grid_of(pairs[j].A, Gj);
            correction(tx, ty, tz, yaw, C);
            rigid_inverse_h(C, Ci);
            const double cr = cos(roll), sr = sin(roll), cp = cos(pitch), sp = sin(pitch);
            const double Ev[16] = {cp, 0, sp, 0, sr * sp, cr, -sr * cp, 0, -cr * sp, sr, cr * cp, 0, 0, 0, 0, 1};
            ::memcpy(E, Ev, sizeof(Ev));
            mat_mul4(pairs[j].T_init_A_B, E, TE);
            items[b] = pairs[j];
            conj_mul(Gj, Ci, TE, items[b].T_init_A_B);
            y[5 * b + 0] = (float)tx;
            y[5 * b + 1] = (float)ty;
            y[5 * b + 2] = (float)tz;
            y[5 * b + 3] = (float)cos(yaw);
            y[5 * b + 4] = (float)sin(yaw);
        }
        if ((rc = pair_summaries(ctx, items.data(), B, cfg->cell, G.data()))) return rc;
        if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->train_y, y.data(), sizeof(float) * 5 * B, hipMemcpyHostToDevice,
                                                ctx->stream), "target upload")))
            return rc;
        if ((rc = net_train_async(net, ctx->net_in, ctx->train_y, B, (float)cfg->lr, (float)cfg->trans_scale)))
            return rc;
        if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->loss_hist + st, net_loss_dev(net), sizeof(float),
                                                hipMemcpyDeviceToDevice, ctx->stream), "loss copy")))
            return rc;
        // the host vectors are refilled next step
        if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "train sync"))) return rc;
    }
    if (loss_host && cfg->steps > 0 &&
        (rc = hip_check(ctx, hipMemcpy(loss_host, ctx->loss_hist, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost),
                        "loss history copy")))
        return rc;
    return COVOX_OK;
}

int covox_align_learned(covox_ctx *ctx, covox_net *net, const covox_pair *pairs, int32_t n, double cell,
                        double cost_thr, int32_t n_rot, int32_t n_starts, double *T_out, double *cost,
                        covox_align_stats *stats)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "align_learned");
    if (!ctx || !net || net_ctx(net) != ctx || (!pairs && n > 0) || n < 0 || !(cell > 0) || n_starts < 1 || !T_out ||
        !cost || n_rot < 1 || n_rot > kLearnChunk || (int64_t)n * n_rot > INT32_MAX / 2)
        return fail(ctx, COVOX_EINVAL, "align_learned: bad argument");
    int rc = prepare_learned(ctx, pairs, n, "align_learned");
    if (rc) return rc;
    // proposals in chunks of at most kLearnChunk network items, then one
    // alignment launch for all of them (the launch lasts as long as its
    // slowest problem, so fewer, larger launches finish sooner)
    const int per = kLearnChunk / n_rot;
    const int nq = n * n_rot;
    std::vector<double> Tp((size_t)16 * nq);
    std::vector<covox_pair> tp((size_t)nq);
    for (int i0 = 0; i0 < n; i0 += per) {
        const int m = std::min(per, n - i0);
        const std::vector<covox_pair> t = turned_pairs(pairs + i0, m, n_rot);
        std::copy(t.begin(), t.end(), tp.begin() + (size_t)i0 * n_rot);
        if ((rc = propose_chunk(ctx, net, t.data(), m * n_rot, cell, &Tp[(size_t)16 * n_rot * i0]))) return rc;
    }
    // with turned priors, each proposal is scored by the cost at the
    // proposal itself (sums at the start pose, no update) and only the best
    // one is refined
    std::vector<int> pick(n, 0);
    if (n_rot > 1) {
        std::vector<AlignProblem> ev(nq);
        for (int q = 0; q < nq; ++q) ev[q] = make_problem(ctx, tp[q].A, tp[q].B, &Tp[16 * (size_t)q], 0);
        std::vector<AlignResult> r0(nq);
        if ((rc = run_alignment(ctx, ev.data(), nq, r0.data()))) return rc;
        for (int j = 0; j < n; ++j) pick[j] = pick_proposal(&r0[(size_t)j * n_rot], n_rot, ctx->p.n_min);
    }
    std::vector<AlignProblem> rp(n);
    for (int j = 0; j < n; ++j) {
        const size_t q = (size_t)j * n_rot + pick[j];
        rp[j] = make_problem(ctx, tp[q].A, tp[q].B, &Tp[16 * q], ctx->p.max_iter);
    }
    std::vector<AlignResult> res(n);
    if ((rc = run_alignment(ctx, rp.data(), n, res.data()))) return rc;
    // fallback to multi-start from the prior
    std::vector<int> fb;
    for (int i = 0; i < n; ++i)
        if (res[i].status == COVOX_EDEGENERATE || !(res[i].cost <= cost_thr)) fb.push_back(i);
    std::vector<int> best(n, -1);
    if (!fb.empty()) {
        std::vector<AlignProblem> prs((size_t)fb.size() * n_starts);
        for (size_t j = 0; j < fb.size(); ++j) {
            const covox_pair &pr = pairs[fb[j]];
            for (int k = 0; k < n_starts; ++k) {
                double S[16];
                if (n_starts == 1) ::memcpy(S, pr.T_init_A_B, sizeof(S));
                else start_pose(pr.T_init_A_B, pr.B->pbar, k, n_starts, S);
                prs[j * n_starts + k] = make_problem(ctx, pr.A, pr.B, S, ctx->p.max_iter);
            }
        }
        std::vector<AlignResult> r2(prs.size());
        if ((rc = run_alignment(ctx, prs.data(), (int)prs.size(), r2.data()))) return rc;
        // The refined proposal competes with the starts under the start
        // selection rule (candidate 0; ties keep it), so a fallback never
        // returns a pose of higher cost than the one it already had.
        std::vector<AlignResult> cand((size_t)n_starts + 1);
        for (size_t j = 0; j < fb.size(); ++j) {
            cand[0] = res[fb[j]];
            for (int k = 0; k < n_starts; ++k) cand[1 + k] = r2[j * n_starts + k];
            const int b = select_start(cand.data(), n_starts + 1);
            if (b >= 1) {
                res[fb[j]] = cand[b];
                best[fb[j]] = b - 1;
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        ::memcpy(T_out + 16 * i, res[i].T, sizeof(double) * 16);
        cost[i] = res[i].cost;
        fill_stats(stats ? stats + i : nullptr, pairs[i].B->n_pts, res[i], best[i]);
    }
    return COVOX_OK;
}

int covox_graph_begin(covox_ctx *ctx)
{
    if (!ctx) return COVOX_EINVAL;
    COVOX_NOT_DURING_CAPTURE(ctx, "graph_begin");
    int rc;
    if (!ctx->cap_stream &&
        (rc = hip_check(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "capture stream")))
        return rc;
    if ((rc = hip_check(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed), "begin capture")))
        return rc;
    ctx->cap_user_stream = ctx->stream;
    ctx->stream = ctx->cap_stream;
    ctx->capturing = true;
    ctx->capture_bad = false;
    ctx->capture_why.clear();
    ctx->cap_subs.clear();
    ctx->cap_host.clear();
    ctx->cap_frozen.clear();
    ctx->cap_saved_timing = ctx->timing;
    ctx->timing = 0;  // no timing events inside a graph
    return COVOX_OK;
}

int covox_graph_end(covox_ctx *ctx, covox_graph **out)
{
    if (!ctx || !out) return COVOX_EINVAL;
    if (!ctx->capturing) return fail(ctx, COVOX_EINVAL, "graph_end: no capture in progress");
    *out = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    ctx->stream = ctx->cap_user_stream;
    ctx->capturing = false;
    ctx->timing = ctx->cap_saved_timing;
    // The captured calls ran their host bookkeeping without running any
    // work: put every submap back as it was, keep the end state for launches.
    for (auto &c : ctx->cap_subs) {
        c.end = snap(c.s);
        restore(c.s, c.start);
    }
    auto drop = [&](const std::string &why, int code) {
        if (graph) (void)hipGraphDestroy(graph);
        for (void *h : ctx->cap_host) (void)hipHostFree(h);
        ctx->cap_host.clear();
        ctx->cap_subs.clear();
        ctx->cap_frozen.clear();
        return fail(ctx, code, why);
    };
    if (e != hipSuccess) return drop(std::string("graph_end: ") + hipGetErrorString(e), COVOX_EHIP);
    if (ctx->capture_bad) return drop("graph_end: " + ctx->capture_why, COVOX_EINVAL);
    for (const auto &f : ctx->cap_frozen)
        for (const auto &c : ctx->cap_subs)
            if (c.s == f.s) return drop("graph_end: a submap that the graph aligns is also changed in it", COVOX_EINVAL);
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return drop(std::string("graph_end: instantiate: ") + hipGetErrorString(e), COVOX_EHIP);
    covox_graph *g = new covox_graph();
    g->ctx = ctx;
    g->graph = graph;
    g->exec = exec;
    g->subs = ctx->cap_subs;
    g->host_bufs = ctx->cap_host;
    g->frozen = ctx->cap_frozen;
    ctx->cap_subs.clear();
    ctx->cap_host.clear();
    ctx->cap_frozen.clear();
    ctx->n_graphs++;
    *out = g;
    return COVOX_OK;
}

int covox_graph_launch(covox_graph *g)
{
    if (!g || !g->ctx) return COVOX_EINVAL;
    covox_ctx *ctx = g->ctx;
    COVOX_NOT_DURING_CAPTURE(ctx, "graph_launch");
    // Scratch and pages were sized for the bounds at capture: a submap used
    // without a reset in the graph must not have grown since.
    for (const auto &c : g->subs) {
        if (c.reset_first) continue;
        const covox_submap *s = c.s;
        bool ok = !s->bound_valid || c.start.bound_valid;
        for (int a = 0; a < 3 && ok && s->bound_valid; ++a)
            ok = s->bound_lo[a] >= c.start.bound_lo[a] && s->bound_hi[a] <= c.start.bound_hi[a];
        if (!ok) return fail(ctx, COVOX_EINVAL, "graph_launch: a submap grew beyond its bounds at capture");
    }
    for (const auto &f : g->frozen)
        if (f.s->version != f.version)
            return fail(ctx, COVOX_EINVAL, "graph_launch: a submap that the graph aligns changed since its set was prepared");
    int rc = hip_check(ctx, hipGraphLaunch(g->exec, ctx->stream), "graph launch");
    if (rc) return rc;
    for (const auto &c : g->subs) {
        covox_submap *s = c.s;
        const bool esdf_current = c.end.esdf_version == c.end.version;
        const bool page_current = c.end.page_version == c.end.version;
        const uint64_t v = std::max(s->version, c.end.version) + 1;
        if (c.reset_first) {
            restore(s, c.end);
            s->pts_version = 0;
        }
        s->version = v;
        if (esdf_current) s->esdf_version = v;
        if (page_current) s->page_version = v;
        s->esdf_exact = false;  // the next eager exact update recomputes everything
    }
    return COVOX_OK;
}

void covox_graph_destroy(covox_graph *g)
{
    if (!g) return;
    covox_ctx *ctx = g->ctx;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (void *h : g->host_bufs) (void)hipHostFree(h);
    if (ctx && --ctx->n_graphs == 0 && !ctx->capturing) {
        for (void *p : ctx->deferred) (void)hipFree(p);
        ctx->deferred.clear();
    }
    delete g;
}

void covox_default_tuning(covox_tuning *t)
{
    if (!t) return;
    memset(t, 0, sizeof(*t));
    // measured on MI355X: per-line envelopes win the y pass once there are a
    // few thousand segments; the windowed z pass, which only visits
    // allocated blocks, won at every size tried
    t->edt_y_env_min_cols = 2048;
    t->edt_z_env_min_cols = INT64_MAX;
    t->align_threads = 256;
    t->align_points_per_step = 1;
    // no cap: on the room step (MI355X) a cap of 512 gave a graph replay about
    // 5 % faster but eager calls no faster, and made each pass slower
    t->edt_pipe_max_workgroups = 0;
}

int covox_tuning_get(const covox_ctx *ctx, covox_tuning *out)
{
    if (!ctx || !out) return COVOX_EINVAL;
    *out = ctx->tune;
    return COVOX_OK;
}

int covox_tuning_set(covox_ctx *ctx, const covox_tuning *t)
{
    if (!ctx || !t) return COVOX_EINVAL;
    if (t->edt_y_env_min_cols < 0 || t->edt_z_env_min_cols < 0)
        return fail(ctx, COVOX_EINVAL, "tuning_set: negative threshold");
    if (t->align_threads != 256 && t->align_threads != 512)
        return fail(ctx, COVOX_EINVAL, "tuning_set: align_threads must be 256 or 512");
    if (t->align_points_per_step != 1 && t->align_points_per_step != 2)
        return fail(ctx, COVOX_EINVAL, "tuning_set: align_points_per_step must be 1 or 2");
    if (t->edt_pipe_max_workgroups < 0)
        return fail(ctx, COVOX_EINVAL, "tuning_set: edt_pipe_max_workgroups must be >= 0");
    if (t->edt_col_seg < 0) return fail(ctx, COVOX_EINVAL, "tuning_set: edt_col_seg must be >= 0");
    if (t->esdf_full_recompute != 0 && t->esdf_full_recompute != 1)
        return fail(ctx, COVOX_EINVAL, "tuning_set: esdf_full_recompute must be 0 or 1");
    if (t->mapping_xcd_order != 0 && t->mapping_xcd_order != 1)
        return fail(ctx, COVOX_EINVAL, "tuning_set: mapping_xcd_order must be 0 or 1");
    ctx->tune = *t;
    return COVOX_OK;
}

int covox_autotune_esdf(covox_ctx *ctx, covox_submap *const *subs, int32_t n, covox_tuning *out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "autotune_esdf");
    if (!ctx || (!subs && n > 0) || n < 0) return fail(ctx, COVOX_EINVAL, "autotune_esdf: bad argument");
    for (int32_t i = 0; i < n; ++i)
        if (!subs[i]) return fail(ctx, COVOX_EINVAL, "autotune_esdf: null submap");
    int rc = autotune_esdf(ctx, subs, n);
    if (rc) return rc;
    if (out) *out = ctx->tune;
    return COVOX_OK;
}

int covox_autotune_align(covox_ctx *ctx, const covox_pair *pairs, int32_t n, int32_t n_starts, covox_tuning *out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "autotune_align");
    if (!ctx || !pairs || n <= 0 || n_starts < 1) return fail(ctx, COVOX_EINVAL, "autotune_align: bad argument");
    std::vector<double> T((size_t)16 * n), cost(n);
    const covox_tuning saved = ctx->tune;
    double best_ms = 1e300;
    covox_tuning best = saved;
    for (int cfg = 0; cfg < 4; ++cfg) {
        ctx->tune.align_threads = cfg & 1 ? 512 : 256;
        ctx->tune.align_points_per_step = cfg & 2 ? 2 : 1;
        int rc = covox_align_batch(ctx, pairs, n, n_starts, T.data(), cost.data(), nullptr);  // warm
        for (int rep = 0; rep < 3 && !rc; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            rc = covox_align_batch(ctx, pairs, n, n_starts, T.data(), cost.data(), nullptr);
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (!rc && ms < best_ms) {
                best_ms = ms;
                best = ctx->tune;
            }
        }
        if (rc) {
            ctx->tune = saved;
            return rc;
        }
    }
    ctx->tune = best;
    if (out) *out = ctx->tune;
    return COVOX_OK;
}

int covox_timing_enable(covox_ctx *ctx, int32_t mask)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "timing_enable");
    if (!ctx) return COVOX_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &u : ctx->ev_used) {
        ctx->ev_pool.push_back(u.second.first);
        ctx->ev_pool.push_back(u.second.second);
    }
    ctx->ev_used.clear();
    for (int k = 0; k < COVOX_K_COUNT; ++k) { ctx->ms[k] = 0; ctx->launches[k] = 0; }
    ctx->timing = mask;
    return COVOX_OK;
}

int covox_timing_get(covox_ctx *ctx, covox_timing *out)
{
    COVOX_NOT_DURING_CAPTURE(ctx, "timing_get");
    if (!ctx || !out) return COVOX_EINVAL;
    int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "timing sync");
    if (rc) return rc;
    for (auto &u : ctx->ev_used) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, u.second.first, u.second.second) == hipSuccess) ctx->ms[u.first] += ms;
        ctx->launches[u.first] += 1;
        ctx->ev_pool.push_back(u.second.first);
        ctx->ev_pool.push_back(u.second.second);
    }
    ctx->ev_used.clear();
    for (int k = 0; k < COVOX_K_COUNT; ++k) { out->ms[k] = ctx->ms[k]; out->launches[k] = ctx->launches[k]; }
    return COVOX_OK;
}

}  // extern "C"
