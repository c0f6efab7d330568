// Submap pose-graph optimisation (paper Eq. 1, Sec. III-F backend):
// registration, odometry and loop-closure terms over submap poses in
// R^3 x SO(2), solved by Levenberg-Marquardt with conjugate gradients on the
// reduced (block-sparse) system, all linear algebra on the GPU.
//
// One linearisation is three device steps:
//   registration normal equations of every pair at T_i^-1 T_j: one batched
//     alignment launch with no pose update (k_align, k_align.hip);
//   k_pgo_terms   one lane per term: its four 4x4 blocks (ii, ij, ji, jj),
//                 two gradient pieces and its cost, in binary64;
//   k_pgo_reduce  one lane per output value (block entry, gradient entry,
//                 cost): sums its contributions in a fixed order, so the
//                 assembled system does not depend on scheduling.
// One step is one launch:
//   k_pgo_cg      one workgroup: (H + mu diag(H)) delta = -g by conjugate
//                 gradients with the inverses of the damped 4x4 diagonal
//                 blocks as preconditioner (vectors in LDS when they fit),
//                 then the model's predicted reduction
//                 -(2 delta.g + delta.H.delta).
// The host runs the Levenberg-Marquardt loop: gain ratio, damping update
// (Madsen, Nielsen and Tingleff 2004), stopping on the step size.
#include "covox_impl.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

namespace covox {

namespace {

struct PgoTerm {
    int32_t i, j;
    int32_t kind;  // 0 registration (normal equations `reg`), 1 relative-pose factor
    int32_t reg;
    double z[4];   // factor: measured (t, yaw) of T_i^-1 T_j
    double w[4];   // factor: 1 / sigma^2
};

constexpr int kTermOut = 4 * 16 + 2 * 4 + 1;  // blocks ii, ij, ji, jj; gradients i, j; cost

__device__ void rz3(double a, double R[9])
{
    double s, c;
    sincos(a, &s, &c);
    R[0] = c; R[1] = -s; R[2] = 0.0;
    R[3] = s; R[4] = c;  R[5] = 0.0;
    R[6] = 0.0; R[7] = 0.0; R[8] = 1.0;
}

__device__ double wrap_angle(double a)
{
    a = fmod(a + M_PI, 2.0 * M_PI);
    if (a <= 0.0) a += 2.0 * M_PI;
    return a - M_PI;
}

// out = A^T B C for A (r x 4), B (r x r), C (r x 4), row-major, r = 6 or 4.
template <int R>
__device__ void atbc(const double *A, const double *B, const double *C, double *out, double scale)
{
    double BC[R * 4];
    for (int p = 0; p < R; ++p)
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += B[p * R + k] * C[k * 4 + q];
            BC[p * 4 + q] = s;
        }
    for (int p = 0; p < 4; ++p)
        for (int q = 0; q < 4; ++q) {
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += A[k * 4 + p] * BC[k * 4 + q];
            out[p * 4 + q] = scale * s;
        }
}

template <int R>
__device__ void atv(const double *A, const double *v, double *out, double scale)
{
    for (int p = 0; p < 4; ++p) {
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += A[k * 4 + p] * v[k];
        out[p] = scale * s;
    }
}

__global__ __launch_bounds__(64) void k_pgo_terms(const PgoTerm *__restrict__ terms, int n_terms,
                                                  const double *__restrict__ x, const double *__restrict__ ne,
                                                  double w_reg, double *__restrict__ out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_terms) return;
    const PgoTerm T = terms[t];
    const double *xi = x + 4 * T.i, *xj = x + 4 * T.j;
    double *o = out + (int64_t)t * kTermOut;
    if (T.kind == 0) {
        // xi of T_ij = T_i^-1 T_j under T_k <- T(x_k + dx_k): Ad(T_i^-1) M(t_j) dx_j
        // - Ad(T_i^-1) M(t_i) dx_i, with M(t) dx = (dt - dyaw z x t, dyaw z)
        double Ri[9];
        rz3(xi[3], Ri);
        double Rt[9], ut[3];  // T_i^-1 = (Ri^T, -Ri^T t_i)
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Rt[3 * r + c] = Ri[3 * c + r];
        for (int r = 0; r < 3; ++r) ut[r] = -(Rt[3 * r] * xi[0] + Rt[3 * r + 1] * xi[1] + Rt[3 * r + 2] * xi[2]);
        double Ad[36] = {0};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                Ad[6 * r + c] = Rt[3 * r + c];
                Ad[6 * (r + 3) + c + 3] = Rt[3 * r + c];
                // [ut]x Rt
                const double hx[3] = {r == 0 ? 0.0 : (r == 1 ? ut[2] : -ut[1]),
                                      r == 0 ? -ut[2] : (r == 1 ? 0.0 : ut[0]),
                                      r == 0 ? ut[1] : (r == 1 ? -ut[0] : 0.0)};
                Ad[6 * r + c + 3] = hx[0] * Rt[c] + hx[1] * Rt[3 + c] + hx[2] * Rt[6 + c];
            }
        double A[2][24];
        for (int s = 0; s < 2; ++s) {
            const double *tp = s == 0 ? xi : xj;
            const double sign = s == 0 ? -1.0 : 1.0;
            double M[24] = {0};
            M[0 * 4 + 0] = 1.0; M[1 * 4 + 1] = 1.0; M[2 * 4 + 2] = 1.0;
            M[0 * 4 + 3] = tp[1];
            M[1 * 4 + 3] = -tp[0];
            M[5 * 4 + 3] = 1.0;
            for (int r = 0; r < 6; ++r)
                for (int c = 0; c < 4; ++c) {
                    double v = 0.0;
                    for (int k = 0; k < 6; ++k) v += Ad[6 * r + k] * M[4 * k + c];
                    A[s][4 * r + c] = sign * v;
                }
        }
        const double *q = ne + (int64_t)T.reg * 29;
        double H6[36], b6[6];
        int k = 0;
        for (int r = 0; r < 6; ++r)
            for (int c = r; c < 6; ++c) {
                H6[6 * r + c] = H6[6 * c + r] = q[k];
                ++k;
            }
        for (int r = 0; r < 6; ++r) b6[r] = q[21 + r];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) atbc<6>(A[a], H6, A[b], o + 16 * (2 * a + b), w_reg);
        for (int a = 0; a < 2; ++a) atv<6>(A[a], b6, o + 64 + 4 * a, w_reg);
        o[72] = w_reg * q[27];
    } else {
        // e_t = Rz(-z_yaw) (Rz(-yaw_i) (t_j - t_i) - z_t), e_yaw = wrap(yaw_j - yaw_i - z_yaw)
        double Rzm[9], Rim[9], Q[9];
        rz3(-T.z[3], Rzm);
        rz3(-xi[3], Rim);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Q[3 * r + c] = Rzm[3 * r] * Rim[c] + Rzm[3 * r + 1] * Rim[3 + c] + Rzm[3 * r + 2] * Rim[6 + c];
        const double d[3] = {xj[0] - xi[0], xj[1] - xi[1], xj[2] - xi[2]};
        double e[4];
        for (int r = 0; r < 3; ++r)
            e[r] = (Q[3 * r] * d[0] + Q[3 * r + 1] * d[1] + Q[3 * r + 2] * d[2]) -
                   (Rzm[3 * r] * T.z[0] + Rzm[3 * r + 1] * T.z[1] + Rzm[3 * r + 2] * T.z[2]);
        e[3] = wrap_angle(xj[3] - xi[3] - T.z[3]);
        const double zd[3] = {-d[1], d[0], 0.0};  // z x d
        double J[2][16] = {{0}, {0}};
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) {
                J[0][4 * r + c] = -Q[3 * r + c];
                J[1][4 * r + c] = Q[3 * r + c];
            }
            J[0][4 * r + 3] = -(Q[3 * r] * zd[0] + Q[3 * r + 1] * zd[1] + Q[3 * r + 2] * zd[2]);
        }
        J[0][15] = -1.0;
        J[1][15] = 1.0;
        const double Om[16] = {T.w[0], 0, 0, 0, 0, T.w[1], 0, 0, 0, 0, T.w[2], 0, 0, 0, 0, T.w[3]};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) atbc<4>(J[a], Om, J[b], o + 16 * (2 * a + b), 1.0);
        const double we[4] = {T.w[0] * e[0], T.w[1] * e[1], T.w[2] * e[2], T.w[3] * e[3]};
        for (int a = 0; a < 2; ++a) atv<4>(J[a], we, o + 64 + 4 * a, 1.0);
        o[72] = e[0] * we[0] + e[1] * we[1] + e[2] * we[2] + e[3] * we[3];
    }
}

// out[dst[k]] = sum of src[off[p]] for p in [ptr[k], ptr[k + 1]), in order.
__global__ __launch_bounds__(256) void k_pgo_reduce(int n_items, const int32_t *__restrict__ dst,
                                                    const int32_t *__restrict__ ptr, const int32_t *__restrict__ off,
                                                    const double *__restrict__ src, double *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_items) return;
    double s = 0.0;
    for (int p = ptr[k]; p < ptr[k + 1]; ++p) s += src[off[p]];
    out[dst[k]] = s;
}

constexpr int kCgThreads = 256;
constexpr int kCgWaves = kCgThreads / 64;

// Sums of (a, b) over the workgroup: butterfly within each wave, then the
// four wave totals in order (deterministic).  Two barriers.
__device__ void block_sum2(double &a, double &b, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * wid] = a;
        red[2 * wid + 1] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int w = 0; w < kCgWaves; ++w) {
        a += red[2 * w];
        b += red[2 * w + 1];
    }
    __syncthreads();
}

// Rows 4 r .. 4 r + 3 of (H + mu diag(H)) p.
__device__ __forceinline__ void bsr_row(int r, const int32_t *rp, const int32_t *ci, const double *vals,
                                        const int32_t *dslot, double mu, const double *p, double y[4])
{
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = rp[r]; s < rp[r + 1]; ++s) {
        const double *B = vals + 16 * (int64_t)s;
        const double *pc = p + 4 * ci[s];
        for (int a = 0; a < 4; ++a) acc[a] += B[4 * a] * pc[0] + B[4 * a + 1] * pc[1] + B[4 * a + 2] * pc[2] + B[4 * a + 3] * pc[3];
    }
    const double *Dg = vals + 16 * (int64_t)dslot[r];
    for (int a = 0; a < 4; ++a) y[a] = acc[a] + mu * Dg[5 * a] * p[4 * r + a];
}

// info[0] = iterations, info[1] = 1 on success (0: not positive definite),
// info[2] = predicted reduction, info[3] = final relative residual.
// Each lane owns whole block rows (b = lane, lane + 256, ...), so that the
// preconditioner and the vector updates need no barrier; the five vectors
// (solution, r, z, p, Ap) live in LDS when they fit (dynamic shared memory
// of 40 n bytes), else in `work`.
__global__ __launch_bounds__(kCgThreads) void k_pgo_cg(int nb, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci, const double *__restrict__ vals,
                                                       const int32_t *__restrict__ dslot, const double *__restrict__ g,
                                                       double mu, double tol, int max_it, double *__restrict__ work,
                                                       double *__restrict__ delta_out, double *__restrict__ info,
                                                       int vec_in_lds)
{
    __shared__ double red[2 * kCgWaves];
    __shared__ int s_bad;
    extern __shared__ double dyn[];
    const int n = 4 * nb, tid = threadIdx.x;
    double *Pinv = work;
    double *vec = vec_in_lds ? dyn : work + 16 * (int64_t)nb;
    double *r = vec, *z = r + n, *p = z + n, *Ap = p + n, *x = Ap + n;
    if (tid == 0) s_bad = 0;
    __syncthreads();
    // inverses of the damped diagonal blocks (Cholesky)
    for (int b = tid; b < nb; b += kCgThreads) {
        const double *B = vals + 16 * (int64_t)dslot[b];
        double A[16], L[16] = {0}, Li[16] = {0};
        for (int k = 0; k < 16; ++k) A[k] = B[k];
        for (int a = 0; a < 4; ++a) A[5 * a] += mu * B[5 * a];
        bool ok = true;
        for (int j = 0; j < 4 && ok; ++j) {
            double sj = A[5 * j];
            for (int k = 0; k < j; ++k) sj -= L[4 * j + k] * L[4 * j + k];
            if (!(sj > 0.0)) { ok = false; break; }
            L[5 * j] = sqrt(sj);
            for (int i = j + 1; i < 4; ++i) {
                double t = A[4 * i + j];
                for (int k = 0; k < j; ++k) t -= L[4 * i + k] * L[4 * j + k];
                L[4 * i + j] = t / L[5 * j];
            }
        }
        if (!ok) {
            s_bad = 1;
            continue;
        }
        for (int c = 0; c < 4; ++c)  // L^-1 by forward substitution
            for (int i = 0; i < 4; ++i) {
                double t = i == c ? 1.0 : 0.0;
                for (int k = 0; k < i; ++k) t -= L[4 * i + k] * Li[4 * k + c];
                Li[4 * i + c] = t / L[5 * i];
            }
        double *P = Pinv + 16 * (int64_t)b;  // (L L^T)^-1 = L^-T L^-1
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                double t = 0.0;
                for (int k = 0; k < 4; ++k) t += Li[4 * k + i] * Li[4 * k + j];
                P[4 * i + j] = t;
            }
    }
    __syncthreads();
    if (s_bad) {
        if (tid == 0) { info[0] = 0; info[1] = 0; info[2] = 0; info[3] = 0; }
        return;
    }
    // z = P r for owned block row b (r already set)
    auto precond_row = [&](int b, double &rr, double &rzp) {
        const double *P = Pinv + 16 * (int64_t)b;
        const double *rb = r + 4 * b;
        for (int a = 0; a < 4; ++a) {
            const double za = P[4 * a] * rb[0] + P[4 * a + 1] * rb[1] + P[4 * a + 2] * rb[2] + P[4 * a + 3] * rb[3];
            z[4 * b + a] = za;
            rr += rb[a] * rb[a];
            rzp += rb[a] * za;
        }
    };
    double bb = 0.0, rz = 0.0;
    for (int b = tid; b < nb; b += kCgThreads) {
        for (int a = 0; a < 4; ++a) {
            x[4 * b + a] = 0.0;
            r[4 * b + a] = -g[4 * b + a];
        }
        precond_row(b, bb, rz);  // bb accumulates |r|^2 = |g|^2
        for (int a = 0; a < 4; ++a) p[4 * b + a] = z[4 * b + a];
    }
    block_sum2(bb, rz, red);  // also orders the p writes before the first product
    const double bnorm = sqrt(bb);
    int it = 0;
    int ok = 1;
    double rel = bnorm > 0.0 ? 1.0 : 0.0;
    while (bnorm > 0.0 && it < max_it) {
        double pap = 0.0, unused = 0.0;
        for (int b = tid; b < nb; b += kCgThreads) {
            double y[4];
            bsr_row(b, rp, ci, vals, dslot, mu, p, y);
            for (int a = 0; a < 4; ++a) {
                Ap[4 * b + a] = y[a];
                pap += p[4 * b + a] * y[a];
            }
        }
        block_sum2(pap, unused, red);
        if (!(pap > 0.0)) { ok = 0; break; }
        const double alpha = rz / pap;
        double rr = 0.0, rz2 = 0.0;
        for (int b = tid; b < nb; b += kCgThreads) {
            for (int a = 0; a < 4; ++a) {
                x[4 * b + a] += alpha * p[4 * b + a];
                r[4 * b + a] -= alpha * Ap[4 * b + a];
            }
            precond_row(b, rr, rz2);
        }
        block_sum2(rr, rz2, red);
        ++it;
        rel = sqrt(rr) / bnorm;
        if (rel <= tol) break;
        const double beta = rz2 / rz;
        rz = rz2;
        for (int b = tid; b < nb; b += kCgThreads)
            for (int a = 0; a < 4; ++a) p[4 * b + a] = z[4 * b + a] + beta * p[4 * b + a];
        __syncthreads();
    }
    // predicted reduction of the undamped model: -(2 x.g + x.H.x)
    __syncthreads();
    double pr = 0.0, unused = 0.0;
    for (int b = tid; b < nb; b += kCgThreads) {
        double y[4];
        bsr_row(b, rp, ci, vals, dslot, 0.0, x, y);
        for (int a = 0; a < 4; ++a) {
            pr += 2.0 * x[4 * b + a] * g[4 * b + a] + x[4 * b + a] * y[a];
            delta_out[4 * b + a] = x[4 * b + a];
        }
    }
    block_sum2(pr, unused, red);
    if (tid == 0) {
        info[0] = it;
        info[1] = ok;
        info[2] = -pr;
        info[3] = rel;
    }
}

// T = [Rz(yaw) t; 0 1] of x = (t, yaw), row-major 4x4.
void pose_of(const double *x, double *T)
{
    const double c = cos(x[3]), s = sin(x[3]);
    const double M[16] = {c, -s, 0, x[0], s, c, 0, x[1], 0, 0, 1, x[2], 0, 0, 0, 1};
    memcpy(T, M, sizeof(M));
}

// T_i^-1 T_j of two poses (binary64).
void relative_pose(const double *xi, const double *xj, double *T)
{
    double Ti[16], Tj[16];
    pose_of(xi, Ti);
    pose_of(xj, Tj);
    double Inv[16] = {0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Inv[4 * r + c] = Ti[4 * c + r];
    for (int r = 0; r < 3; ++r) Inv[4 * r + 3] = -(Inv[4 * r] * Ti[3] + Inv[4 * r + 1] * Ti[7] + Inv[4 * r + 2] * Ti[11]);
    Inv[15] = 1.0;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            T[4 * r + c] = Inv[4 * r] * Tj[c] + Inv[4 * r + 1] * Tj[4 + c] + Inv[4 * r + 2] * Tj[8 + c] + Inv[4 * r + 3] * Tj[12 + c];
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

}  // namespace

void covox_default_pgo_cfg_impl(covox_pgo_cfg *c)
{
    c->max_iter = 20;
    c->cg_max_iter = 0;
    c->sigma_reg = 0.05;
    c->lambda0 = 1e-4;
    c->tol_step = 1e-8;
    c->cg_tol = 1e-12;
}

int pgo_solve(covox_ctx *ctx, covox_submap *const *subs, int32_t N, double *x, const int32_t *reg_pairs,
              int32_t n_reg, const covox_pose_factor *factors, int32_t n_fac, const covox_pgo_cfg *cfg_in,
              covox_pgo_stats *stats)
{
    covox_pgo_cfg cfg;
    if (cfg_in) cfg = *cfg_in;
    else covox_default_pgo_cfg_impl(&cfg);
    if (!subs || !x || N < 2 || n_reg < 0 || n_fac < 0 || (n_reg > 0 && !reg_pairs) || (n_fac > 0 && !factors))
        return fail(ctx, COVOX_EINVAL, "pgo: bad argument");
    if (cfg.max_iter < 0 || cfg.cg_max_iter < 0 || !(cfg.sigma_reg > 0) || !(cfg.lambda0 >= 0) ||
        !(cfg.tol_step >= 0) || !(cfg.cg_tol >= 0))
        return fail(ctx, COVOX_EINVAL, "pgo: bad configuration");
    for (int32_t k = 0; k < 4 * N; ++k)
        if (!std::isfinite(x[k])) return fail(ctx, COVOX_EINVAL, "pgo: poses must be finite");
    std::vector<PgoTerm> terms;
    for (int32_t k = 0; k < n_reg; ++k) {
        const int32_t i = reg_pairs[2 * k], j = reg_pairs[2 * k + 1];
        if (i < 0 || j < 0 || i >= N || j >= N || i == j || !subs[i] || !subs[j])
            return fail(ctx, COVOX_EINVAL, "pgo: bad registration pair");
        PgoTerm t{};
        t.i = i; t.j = j; t.kind = 0; t.reg = k;
        terms.push_back(t);
    }
    for (int32_t k = 0; k < n_fac; ++k) {
        const covox_pose_factor &f = factors[k];
        if (f.i < 0 || f.j < 0 || f.i >= N || f.j >= N || f.i == f.j)
            return fail(ctx, COVOX_EINVAL, "pgo: bad factor indices");
        PgoTerm t{};
        t.i = f.i; t.j = f.j; t.kind = 1; t.reg = -1;
        for (int a = 0; a < 4; ++a) {
            if (!(f.sigma[a] > 0) || !std::isfinite(f.z[a])) return fail(ctx, COVOX_EINVAL, "pgo: bad factor");
            t.z[a] = f.z[a];
            t.w[a] = 1.0 / (f.sigma[a] * f.sigma[a]);
        }
        terms.push_back(t);
    }
    const int n_terms = (int)terms.size();
    if (n_terms == 0) return fail(ctx, COVOX_EINVAL, "pgo: no terms");
    int rc;
    for (int32_t k = 0; k < n_reg; ++k) {
        covox_submap *A = subs[reg_pairs[2 * k]], *B = subs[reg_pairs[2 * k + 1]];
        if (A->esdf_version != A->version)
            return fail(ctx, COVOX_EINVAL, "pgo: an ESDF of a registration pair is out of date");
        if ((rc = extract_points(ctx, B))) return rc;
    }

    // block-sparse pattern over the free poses 1..N-1 (block row r = pose r + 1)
    const int nb = N - 1, n = 4 * nb;
    std::vector<std::vector<int>> cols(nb);
    for (int r = 0; r < nb; ++r) cols[r].push_back(r);
    for (const PgoTerm &t : terms)
        if (t.i > 0 && t.j > 0) {
            cols[t.i - 1].push_back(t.j - 1);
            cols[t.j - 1].push_back(t.i - 1);
        }
    std::vector<int32_t> rp(nb + 1, 0), ci, dslot(nb);
    std::map<std::pair<int, int>, int> slot;
    for (int r = 0; r < nb; ++r) {
        std::sort(cols[r].begin(), cols[r].end());
        cols[r].erase(std::unique(cols[r].begin(), cols[r].end()), cols[r].end());
        for (int c : cols[r]) {
            if (c == r) dslot[r] = (int32_t)ci.size();
            slot[{r, c}] = (int32_t)ci.size();
            ci.push_back(c);
        }
        rp[r + 1] = (int32_t)ci.size();
    }
    const int nnzb = (int)ci.size();
    // reduction plan: output = [blocks (16 nnzb) | gradient (n) | cost]
    std::vector<std::vector<int32_t>> src(16 * nnzb + n + 1);
    for (int t = 0; t < n_terms; ++t) {
        const int ends[2] = {terms[t].i, terms[t].j};
        for (int a = 0; a < 2; ++a) {
            if (ends[a] == 0) continue;
            for (int b = 0; b < 2; ++b) {
                if (ends[b] == 0) continue;
                const int s = slot[{ends[a] - 1, ends[b] - 1}];
                for (int e = 0; e < 16; ++e) src[16 * s + e].push_back(t * kTermOut + 16 * (2 * a + b) + e);
            }
            for (int e = 0; e < 4; ++e) src[16 * nnzb + 4 * (ends[a] - 1) + e].push_back(t * kTermOut + 64 + 4 * a + e);
        }
        src[16 * nnzb + n].push_back(t * kTermOut + 72);
    }
    const int n_out = 16 * nnzb + n + 1;
    std::vector<int32_t> pdst, pptr(1, 0), poff;
    for (int k = 0; k < n_out; ++k) {
        pdst.push_back(k);
        for (int32_t o : src[k]) poff.push_back(o);
        pptr.push_back((int32_t)poff.size());
    }

    // device buffers
    DevBuf b_terms, b_x, b_ne, b_tout, b_out[2], b_rp, b_ci, b_dslot, b_pdst, b_pptr, b_poff, b_work, b_delta, b_info;
    auto alloc = [&](DevBuf &b, size_t bytes) {
        return hip_check(ctx, hipMalloc(&b.p, std::max<size_t>(bytes, 8)), "pgo buffers");
    };
    if ((rc = alloc(b_terms, sizeof(PgoTerm) * n_terms)) || (rc = alloc(b_x, sizeof(double) * 4 * N)) ||
        (rc = alloc(b_ne, sizeof(double) * 29 * std::max(n_reg, 1))) ||
        (rc = alloc(b_tout, sizeof(double) * kTermOut * n_terms)) || (rc = alloc(b_out[0], sizeof(double) * n_out)) ||
        (rc = alloc(b_out[1], sizeof(double) * n_out)) || (rc = alloc(b_rp, sizeof(int32_t) * (nb + 1))) ||
        (rc = alloc(b_ci, sizeof(int32_t) * nnzb)) || (rc = alloc(b_dslot, sizeof(int32_t) * nb)) ||
        (rc = alloc(b_pdst, sizeof(int32_t) * pdst.size())) || (rc = alloc(b_pptr, sizeof(int32_t) * pptr.size())) ||
        (rc = alloc(b_poff, sizeof(int32_t) * std::max<size_t>(poff.size(), 1))) ||
        (rc = alloc(b_work, sizeof(double) * (16 * (size_t)nb + 5 * (size_t)n))) ||
        (rc = alloc(b_delta, sizeof(double) * n)) || (rc = alloc(b_info, sizeof(double) * 4)))
        return rc;
    hipStream_t st = ctx->stream;
    auto up = [&](DevBuf &b, const void *h, size_t bytes) {
        return hip_check(ctx, hipMemcpyAsync(b.p, h, bytes, hipMemcpyHostToDevice, st), "pgo upload");
    };
    if ((rc = up(b_terms, terms.data(), sizeof(PgoTerm) * n_terms)) ||
        (rc = up(b_rp, rp.data(), sizeof(int32_t) * rp.size())) || (rc = up(b_ci, ci.data(), sizeof(int32_t) * nnzb)) ||
        (rc = up(b_dslot, dslot.data(), sizeof(int32_t) * nb)) ||
        (rc = up(b_pdst, pdst.data(), sizeof(int32_t) * pdst.size())) ||
        (rc = up(b_pptr, pptr.data(), sizeof(int32_t) * pptr.size())) ||
        (poff.size() && (rc = up(b_poff, poff.data(), sizeof(int32_t) * poff.size()))))
        return rc;

    std::vector<AlignProblem> probs(n_reg);
    std::vector<AlignResult> res(n_reg);
    std::vector<double> ne(29 * (size_t)std::max(n_reg, 1));
    const double w_reg = 1.0 / (cfg.sigma_reg * cfg.sigma_reg);
    // F, g and H at poses xs into output buffer `which`; F returned on the host
    auto linearize = [&](const double *xs, int which, double *F) -> int {
        int rc2;
        for (int32_t k = 0; k < n_reg; ++k) {
            const covox_submap *A = subs[reg_pairs[2 * k]], *B = subs[reg_pairs[2 * k + 1]];
            AlignProblem &pr = probs[k];
            memset(&pr, 0, sizeof(pr));
            pr.phi = A->phi;
            pr.page = A->page;
            pr.metaA = A->meta;
            pr.pts = B->pts;
            pr.n_pts = B->n_pts;
            relative_pose(xs + 4 * reg_pairs[2 * k], xs + 4 * reg_pairs[2 * k + 1], pr.T);
            pr.max_iter = 0;
        }
        if (n_reg > 0) {
            if ((rc2 = run_alignment(ctx, probs.data(), n_reg, res.data()))) return rc2;
            for (int32_t k = 0; k < n_reg; ++k) memcpy(&ne[29 * (size_t)k], res[k].ne, sizeof(double) * 29);
            if ((rc2 = up(b_ne, ne.data(), sizeof(double) * 29 * n_reg))) return rc2;
        }
        if ((rc2 = up(b_x, xs, sizeof(double) * 4 * N))) return rc2;
        {
            TimedLaunch tl(ctx, COVOX_K_PGO);
            hipLaunchKernelGGL(k_pgo_terms, dim3((n_terms + 63) / 64), dim3(64), 0, st, (const PgoTerm *)b_terms.p,
                               n_terms, (const double *)b_x.p, (const double *)b_ne.p, w_reg, (double *)b_tout.p);
            hipLaunchKernelGGL(k_pgo_reduce, dim3((n_out + 255) / 256), dim3(256), 0, st, n_out,
                               (const int32_t *)b_pdst.p, (const int32_t *)b_pptr.p, (const int32_t *)b_poff.p,
                               (const double *)b_tout.p, (double *)b_out[which].p);
        }
        if ((rc2 = hip_check(ctx, hipGetLastError(), "pgo launch"))) return rc2;
        if ((rc2 = hip_check(ctx, hipMemcpyAsync(F, (double *)b_out[which].p + 16 * nnzb + n, sizeof(double),
                                                 hipMemcpyDeviceToHost, st), "pgo cost")))
            return rc2;
        return hip_check(ctx, hipStreamSynchronize(st), "pgo sync");
    };
    const int cg_max = cfg.cg_max_iter > 0 ? cfg.cg_max_iter : 4 * n;
    // vectors in LDS up to 48 KB (n <= 1228), beside the 2 KB reduction buffer
    const size_t lds_bytes = 5 * sizeof(double) * (size_t)n <= 48 * 1024 ? 5 * sizeof(double) * (size_t)n : 0;
    std::vector<double> delta(n);
    double info[4];
    auto step = [&](int which, double mu) -> int {
        {
            TimedLaunch tl(ctx, COVOX_K_PGO);
            const double *out = (const double *)b_out[which].p;
            hipLaunchKernelGGL(k_pgo_cg, dim3(1), dim3(kCgThreads), lds_bytes, st, nb, (const int32_t *)b_rp.p,
                               (const int32_t *)b_ci.p, out, (const int32_t *)b_dslot.p, out + 16 * nnzb, mu,
                               cfg.cg_tol, cg_max, (double *)b_work.p, (double *)b_delta.p, (double *)b_info.p,
                               lds_bytes > 0 ? 1 : 0);
        }
        int rc2;
        if ((rc2 = hip_check(ctx, hipGetLastError(), "pgo cg launch"))) return rc2;
        if ((rc2 = hip_check(ctx, hipMemcpyAsync(delta.data(), b_delta.p, sizeof(double) * n, hipMemcpyDeviceToHost, st),
                             "pgo step copy")) ||
            (rc2 = hip_check(ctx, hipMemcpyAsync(info, b_info.p, sizeof(info), hipMemcpyDeviceToHost, st), "pgo info")))
            return rc2;
        return hip_check(ctx, hipStreamSynchronize(st), "pgo sync");
    };

    std::vector<double> xc(x, x + 4 * N), xn(4 * N);
    double F = 0.0, Fn = 0.0;
    int cur = 0;
    if ((rc = linearize(xc.data(), cur, &F))) return rc;
    const double F0 = F;
    double mu = cfg.lambda0, nu = 2.0;
    int it = 0, acc = 0, conv = 0, cg_total = 0;
    while (it < cfg.max_iter) {
        ++it;
        if ((rc = step(cur, mu))) return rc;
        if (info[1] == 0.0) return fail(ctx, COVOX_EINVAL, "pgo: the damped system is not positive definite");
        cg_total += (int)info[0];
        double dmax = 0.0;
        for (double d : delta) dmax = std::max(dmax, std::fabs(d));
        if (dmax < cfg.tol_step) {
            conv = 1;
            break;
        }
        xn = xc;
        for (int k = 0; k < n; ++k) xn[4 + k] += delta[k];
        if ((rc = linearize(xn.data(), cur ^ 1, &Fn))) return rc;
        const double pred = info[2];
        const double rho = pred > 0.0 ? (F - Fn) / pred : -1.0;
        if (rho > 0.0) {
            xc.swap(xn);
            F = Fn;
            cur ^= 1;
            ++acc;
            mu *= std::max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) * (2.0 * rho - 1.0) * (2.0 * rho - 1.0));
            nu = 2.0;
        } else {
            mu *= nu;
            nu *= 2.0;
        }
    }
    memcpy(x, xc.data(), sizeof(double) * 4 * N);
    if (stats) {
        stats->iterations = it;
        stats->accepted = acc;
        stats->converged = conv;
        stats->cg_iterations = cg_total;
        stats->cost_init = F0;
        stats->cost_final = F;
    }
    return COVOX_OK;
}

}  // namespace covox
