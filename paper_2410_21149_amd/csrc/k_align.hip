// Correspondence-free ESDF alignment of two submaps (paper Sec. I and
// Sec. III-F: the registration term of Eq. (1); registration points chosen
// by weight; residuals, Jacobians and the least-squares solve on the GPU).
//
// Registration points of B: zero crossings of D_B along voxel edges whose
// endpoints are both in the band with W >= w_reg (k_iso_count, k_iso_scan,
// k_iso_write; order = block buffer index, in-block index, axis).
//
// k_align: one workgroup per (pair, start), persistent over the
// Gauss-Newton iterations.  Per point (binary32): q = T p, trilinear ESDF of
// A and its gradient g, J = [g ; q x g]; exact binary64 products summed per
// lane in binary64, then a fixed-order wave / workgroup reduction into the
// 21 + 6 + 1 + 1 sums of the normal equations.  Lane 0 solves the 6x6 system
// by binary64 Cholesky and applies T <- Exp(delta) T.
#include "covox_impl.h"

#include <string.h>

#include <algorithm>
#include <vector>

namespace covox {

namespace {

template <typename S> __device__ __forceinline__ float ldw(const S *p);
template <> __device__ __forceinline__ float ldw<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float ldw<__half>(const __half *p) { return __half2float(*p); }

struct DomArgs {
    int32_t lo[3], dim[3];
};

__device__ __forceinline__ DomArgs dom_of(const SubmapMeta *m)
{
    DomArgs d;
    for (int a = 0; a < 3; ++a) { d.lo[a] = m->dom_min[a]; d.dim[a] = m->dom_dim[a]; }
    return d;
}

// Buffer index of block (bx, by, bz) through a dense page, -1 when absent.
__device__ __forceinline__ int64_t page_lookup(const int32_t *page, const DomArgs &d, int bx, int by, int bz)
{
    const int x = bx - d.lo[0], y = by - d.lo[1], z = bz - d.lo[2];
    if (x < 0 || y < 0 || z < 0 || x >= d.dim[0] || y >= d.dim[1] || z >= d.dim[2]) return -1;
    return page[((int64_t)z * d.dim[1] + y) * d.dim[0] + x];
}

// The three +x, +y, +z edges of voxel lane + 64 z of block `idx`.
template <typename S>
__device__ __forceinline__ void edge_tests(const S *D, const S *W, int64_t idx, const int64_t nb[3], int lane, int z,
                                           float tau, float wreg, bool ok[3], float Di_out[1], float Dn_out[3])
{
    const int x = lane & 7, y = lane >> 3;
    const int64_t o = idx * 512 + lane + 64 * z;
    const float Di = ldw(D + o), Wi = ldw(W + o);
    Di_out[0] = Di;
    const bool base = Wi >= wreg && fabsf(Di) < tau;
    const int c[3] = {x, y, z};
    const int step[3] = {1, 8, 64};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int64_t on;
        if (c[a] < 7) on = o + step[a];
        else on = nb[a] >= 0 ? nb[a] * 512 + (lane + 64 * z) - 7 * step[a] : -1;
        ok[a] = false;
        Dn_out[a] = 0.0f;
        if (!base || on < 0) continue;
        const float Dn = ldw(D + on), Wn = ldw(W + on);
        Dn_out[a] = Dn;
        ok[a] = Wn >= wreg && fabsf(Dn) < tau && ((Di < 0.0f) != (Dn < 0.0f));
    }
}

template <typename S>
__global__ __launch_bounds__(256) void k_iso(const SubmapMeta *__restrict__ meta, const uint64_t *__restrict__ keys,
                                             const int32_t *__restrict__ page, const S *__restrict__ D,
                                             const S *__restrict__ W, float vs, float tau, float wreg, int write,
                                             uint32_t *__restrict__ cnt, float *__restrict__ pts,
                                             double *__restrict__ psum)
{
    const int64_t nbk = meta->n_blocks;
    const DomArgs dm = dom_of(meta);
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < nbk; j += nwaves) {
        int bx, by, bz;
        unpack_key(keys[j], bx, by, bz);
        int64_t nb[3];
        nb[0] = page_lookup(page, dm, bx + 1, by, bz);
        nb[1] = page_lookup(page, dm, bx, by + 1, bz);
        nb[2] = page_lookup(page, dm, bx, by, bz + 1);
        int64_t base = write ? (int64_t)cnt[j] : 0;
        uint32_t total = 0;
        double s0 = 0, s1 = 0, s2 = 0;
        for (int z = 0; z < 8; ++z) {
            bool ok[3];
            float Di, Dn[3];
            edge_tests(D, W, j, nb, lane, z, tau, wreg, ok, &Di, Dn);
            const int c = (int)ok[0] + (int)ok[1] + (int)ok[2];
            // wave exclusive prefix of c (ascending lane = ascending l)
            int incl = c;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y2 = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y2;
            }
            const int wtot = __shfl(incl, 63, 64);
            if (write && c) {
                int64_t at = base + (incl - c);
                const int ix = 8 * bx + (lane & 7), iy = 8 * by + (lane >> 3), iz = 8 * bz + z;
                const float cx = ((float)ix + 0.5f) * vs, cy = ((float)iy + 0.5f) * vs, cz = ((float)iz + 0.5f) * vs;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (!ok[a]) continue;
                    const float sfr = Di / (Di - Dn[a]);
                    float p[3] = {cx, cy, cz};
                    p[a] = p[a] + sfr * vs;
                    pts[3 * at + 0] = p[0];
                    pts[3 * at + 1] = p[1];
                    pts[3 * at + 2] = p[2];
                    s0 += (double)p[0];
                    s1 += (double)p[1];
                    s2 += (double)p[2];
                    ++at;
                }
            }
            base += wtot;
            total += (uint32_t)wtot;
        }
        if (!write) {
            if (lane == 0) cnt[j] = total;
        } else {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                s0 += __shfl_xor(s0, o, 64);
                s1 += __shfl_xor(s1, o, 64);
                s2 += __shfl_xor(s2, o, 64);
            }
            if (lane == 0) {
                psum[3 * j + 0] = s0;
                psum[3 * j + 1] = s1;
                psum[3 * j + 2] = s2;
            }
        }
    }
}

// Exclusive scan of cnt[0, n) in place (one 1024-lane workgroup, each lane a
// contiguous chunk), total into meta->n_points.
__global__ __launch_bounds__(1024) void k_iso_scan(SubmapMeta *meta, uint32_t *cnt)
{
    __shared__ int64_t lds[16];
    const int64_t n = meta->n_blocks;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    const int64_t C = (n + blockDim.x - 1) / blockDim.x;
    const int64_t beg = std::min<int64_t>((int64_t)tid * C, n), end = std::min<int64_t>(beg + C, n);
    int64_t s = 0;
    for (int64_t j = beg; j < end; ++j) s += cnt[j];
    int64_t x = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int64_t w = lane < nw ? lds[lane] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < nw) lds[lane] = w;
    }
    __syncthreads();
    int64_t run = (wid > 0 ? lds[wid - 1] : 0) + x - s;
    for (int64_t j = beg; j < end; ++j) {
        const uint32_t c = cnt[j];
        cnt[j] = (uint32_t)run;
        run += c;
    }
    if (tid == 0) meta->n_points = lds[nw - 1];
}

// Centroid of the points from per-block sums, summed in block order.
__global__ void k_pbar(SubmapMeta *meta, const double *psum)
{
    if (threadIdx.x != 0) return;
    const int64_t n = meta->n_blocks;
    double s[3] = {0, 0, 0};
    for (int64_t j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) s[a] += psum[3 * j + a];
    const double np = (double)(meta->n_points > 0 ? meta->n_points : 1);
    for (int a = 0; a < 3; ++a) meta->pbar[a] = s[a] / np;
}

// ------------------------------------------------------------ alignment

__device__ __forceinline__ float phi_at(const float *phi, const int32_t *page, const DomArgs &d, int jx, int jy,
                                        int jz)
{
    const int64_t idx = page_lookup(page, d, jx >> 3, jy >> 3, jz >> 3);
    if (idx < 0) return __builtin_nanf("");
    return phi[idx * 512 + (jx & 7) + 8 * (jy & 7) + 64 * (jz & 7)];
}

// phi at voxel j without branches (NaN when the voxel's block is outside the
// page or unallocated): the loads go to clamped addresses and the result is
// selected, so the corner loads of several points can be in flight at once.
__device__ __forceinline__ float phi_at_nb(const float *phi, const int32_t *page, const DomArgs &d, int jx, int jy,
                                           int jz)
{
    const int x = (jx >> 3) - d.lo[0], y = (jy >> 3) - d.lo[1], z = (jz >> 3) - d.lo[2];
    const bool in = x >= 0 && y >= 0 && z >= 0 && x < d.dim[0] && y < d.dim[1] && z < d.dim[2];
    const int64_t pi = in ? ((int64_t)z * d.dim[1] + y) * d.dim[0] + x : 0;
    const int32_t b = page[pi];
    const bool ok = in && b >= 0;
    const float v = phi[(int64_t)(ok ? b : 0) * 512 + (jx & 7) + 8 * (jy & 7) + 64 * (jz & 7)];
    return ok ? v : __builtin_nanf("");
}

// Residual and Jacobian of U points (indices i0 + u stride, those beyond n
// are invalid) with all their loads issued before any is used; ok[u] false
// when a cell corner is unobserved or the point is far outside A.  Per
// point: q = T p; g = q / vs - 1/2, j0 = floor(g), f = g - j0; r is the
// trilinear value of the 8 corners and J = [grad; q x grad] with the
// gradient of the trilinear patch divided by vs.
template <int U>
__device__ __forceinline__ void residual_u(const float *Tf, const float *pts, int64_t i0, int64_t stride, int64_t n,
                                          float vs, const float *phi, const int32_t *page, const DomArgs &d,
                                          float J[U][6], float r[U], bool ok[U])
{
    float c[U][8], f[U][3], q[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = i0 + u * stride;
        const bool in = i < n;
        const int64_t ii = in ? i : 0;
        const float p[3] = {pts[3 * ii], pts[3 * ii + 1], pts[3 * ii + 2]};
        int j0[3];
        bool fin = in;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            q[u][a] = ((Tf[4 * a + 0] * p[0] + Tf[4 * a + 1] * p[1]) + Tf[4 * a + 2] * p[2]) + Tf[4 * a + 3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float g = (q[u][a] / vs) - 0.5f;
            fin = fin && fabsf(g) < 1.0e8f;
            g = fabsf(g) < 1.0e8f ? g : 0.0f;  // keeps the clamped addresses sane
            const float fl = floorf(g);
            j0[a] = (int)fl;
            f[u][a] = g - fl;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c[u][k] = phi_at_nb(phi, page, d, j0[0] + (k & 1), j0[1] + ((k >> 1) & 1), j0[2] + ((k >> 2) & 1));
        ok[u] = fin;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        bool good = ok[u];
#pragma unroll
        for (int k = 0; k < 8; ++k) good = good && !isnan(c[u][k]);
        ok[u] = good;
        const float *cc = c[u];
        const float wx0 = 1.0f - f[u][0], wx1 = f[u][0], wy0 = 1.0f - f[u][1], wy1 = f[u][1], wz0 = 1.0f - f[u][2],
                    wz1 = f[u][2];
        const float c00 = cc[0] * wx0 + cc[1] * wx1, c10 = cc[2] * wx0 + cc[3] * wx1;
        const float c01 = cc[4] * wx0 + cc[5] * wx1, c11 = cc[6] * wx0 + cc[7] * wx1;
        const float c0 = c00 * wy0 + c10 * wy1, c1 = c01 * wy0 + c11 * wy1;
        r[u] = c0 * wz0 + c1 * wz1;
        const float dx = ((cc[1] - cc[0]) * wy0 + (cc[3] - cc[2]) * wy1) * wz0 +
                         ((cc[5] - cc[4]) * wy0 + (cc[7] - cc[6]) * wy1) * wz1;
        const float dy = (c10 - c00) * wz0 + (c11 - c01) * wz1;
        const float dz = c1 - c0;
        const float g0 = dx / vs, g1 = dy / vs, g2 = dz / vs;
        J[u][0] = g0;
        J[u][1] = g1;
        J[u][2] = g2;
        J[u][3] = q[u][1] * g2 - q[u][2] * g1;
        J[u][4] = q[u][2] * g0 - q[u][0] * g2;
        J[u][5] = q[u][0] * g1 - q[u][1] * g0;
    }
}

// 4-DoF step (translation and yaw): rows and columns 0, 1, 2, 5 of the
// normal equations, diagonal damped by mu (0: Gauss-Newton), by Cholesky;
// x = (rho, 0, 0, theta_z).
__device__ bool solve_xyz_yaw(const double *ne, double mu, double x[6])
{
    const int sel[4] = {0, 1, 2, 5};
    double H[4][4], b[4], L[4][4];
    for (int a = 0; a < 4; ++a) {
        for (int c = 0; c < 4; ++c) {
            int r = sel[a], q = sel[c];
            if (r > q) { const int t = r; r = q; q = t; }
            H[a][c] = ne[r * 6 - r * (r - 1) / 2 + (q - r)];
            L[a][c] = 0.0;
        }
        b[a] = ne[21 + sel[a]];
    }
    if (mu != 0.0)
        for (int a = 0; a < 4; ++a) H[a][a] = H[a][a] + mu * H[a][a];
    for (int j = 0; j < 4; ++j) {
        double sj = H[j][j];
        for (int k = 0; k < j; ++k) sj -= L[j][k] * L[j][k];
        if (!(sj > 0.0)) return false;
        L[j][j] = sqrt(sj);
        for (int i = j + 1; i < 4; ++i) {
            double t = H[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    double y[4], z[4];
    for (int i = 0; i < 4; ++i) {
        double t = -b[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 4; ++k) t -= L[k][i] * z[k];
        z[i] = t / L[i][i];
    }
    x[0] = z[0]; x[1] = z[1]; x[2] = z[2];
    x[3] = 0.0; x[4] = 0.0; x[5] = z[3];
    return true;
}

// 6x6 Cholesky solve of (H + mu diag(H)) x = -b (H from the packed upper
// triangle; mu = 0 is the Gauss-Newton step).
__device__ bool solve6(const double *ne, double mu, double x[6])
{
    double L[6][6];
    for (int j = 0; j < 6; ++j) {
        for (int i = 0; i < 6; ++i) L[j][i] = 0.0;
    }
    auto Hat = [&](int a, int b) {
        if (a > b) { const int t = a; a = b; b = t; }
        return ne[a * 6 - a * (a - 1) / 2 + (b - a)];
    };
    for (int j = 0; j < 6; ++j) {
        double s = Hat(j, j);
        if (mu != 0.0) s = s + mu * s;
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) return false;
        L[j][j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = Hat(i, j);
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double t = -ne[21 + i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (int i = 5; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 6; ++k) t -= L[k][i] * x[k];
        x[i] = t / L[i][i];
    }
    return true;
}

// Decrease of the sum of squares that the linear model predicts for the step
// d: -(2 d.b + d.H.d), from the packed normal equations.
__device__ double lm_predicted(const double *ne, const double d[6])
{
    double g = 0.0, q = 0.0;
    for (int a = 0; a < 6; ++a) {
        double s = 0.0;
        for (int b = 0; b < 6; ++b) {
            const int r = a < b ? a : b, c = a < b ? b : a;
            s += ne[r * 6 - r * (r - 1) / 2 + (c - r)] * d[b];
        }
        q += d[a] * s;
        g += d[a] * ne[21 + a];
    }
    return -(2.0 * g + q);
}

// T <- Exp(xi) T for xi = (rho, theta); T is the top 3x4 of a rigid
// transform, row-major.
__device__ void se3_left_update(const double xi[6], double T[12])
{
    const double *w = xi + 3;
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        const double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
    double K2[3][3], Rm[3][3], V[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) K2[r][c] = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            const double I = r == c ? 1.0 : 0.0;
            Rm[r][c] = I + A * K[r][c] + B * K2[r][c];
            V[r][c] = I + B * K[r][c] + C * K2[r][c];
        }
    double tE[3];
    for (int r = 0; r < 3; ++r) tE[r] = V[r][0] * xi[0] + V[r][1] * xi[1] + V[r][2] * xi[2];
    double O[12];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) O[4 * r + c] = (Rm[r][0] * T[c] + Rm[r][1] * T[4 + c]) + Rm[r][2] * T[8 + c];
        O[4 * r + 3] = ((Rm[r][0] * T[3] + Rm[r][1] * T[7]) + Rm[r][2] * T[11]) + tE[r];
    }
    for (int k = 0; k < 12; ++k) T[k] = O[k];
}

// One workgroup of kAlignThreads lanes per problem (pair and start); each
// lane takes U points per step (same points, same order, for every U).
// LM = false: Gauss-Newton, every solve taken.  LM = true: Levenberg-
// Marquardt (the trust-region least squares Sec. III-F names): the solve is
// damped by mu diag(H), its trial pose is evaluated, and the step is taken
// when the mean cost falls (gain ratio > 0); max_iter then caps the solves.
// LM also ends as converged when the decrease L that the model predicts is
// within the cost's binary32 rounding noise, L <= 2^-19 Q sqrt(c): each
// residual carries an error of up to 16 u Q (u = 2^-24, Q the largest norm
// of a corner of A's ESDF domain, in metres), and over the residuals these
// errors add in root-sum-square to at most 2 * 16 u Q sqrt(c) in c = sum r^2;
// below that the gain ratio is rounding noise.
constexpr double kCostNoise32 = 1.0 / 524288.0;  // 2 * 16 * 2^-24
template <int kAlignThreads, int U, bool LM>
__global__ __launch_bounds__(kAlignThreads) void k_align(const AlignProblem *__restrict__ probs,
                                                         const int32_t *__restrict__ order, AlignResult *res,
                                                         float vs, double tol_rho, double tol_theta, int n_min,
                                                         int dof)
{
    __shared__ double sT[12];
    __shared__ float sTf[12];
    __shared__ double red[kAlignThreads / 64][29];
    __shared__ double tot[29];
    __shared__ int s_state[3];  // final flag, iterations (LM: solves), status
    __shared__ double sPrev[29], sTt[12], sD[6], sMu[2];  // LM: accepted sums, trial pose, step, mu and nu
    __shared__ int s_lm[2];                               // LM: accepted sums present, steps taken
    const int pid = order[blockIdx.x];
    const AlignProblem &P = probs[pid];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const DomArgs d = dom_of(P.metaA);
    double noise = 0.0;  // LM: the floor of the predicted decrease is noise sqrt(c)
    if (LM) {
        double q2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double lo = (8.0 * (double)vs) * (double)d.lo[a], hi = (8.0 * (double)vs) * (double)(d.lo[a] + d.dim[a]);
            const double m = fmax(fabs(lo), fabs(hi));
            q2 += m * m;
        }
        noise = kCostNoise32 * sqrt(q2);
    }
    if (tid < 12) {
        sT[tid] = P.T[tid];
        sTf[tid] = (float)P.T[tid];
    }
    if (tid == 0) {
        s_state[0] = 0;
        s_state[1] = 0;
        s_state[2] = COVOX_NOT_CONVERGED;
        if (LM) {
            s_lm[0] = 0;
            s_lm[1] = 0;
            sMu[0] = 1e-4;
            sMu[1] = 2.0;
        }
    }
    __syncthreads();
    for (;;) {
        double acc[29];
#pragma unroll
        for (int k = 0; k < 29; ++k) acc[k] = 0.0;
        float Tf[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) Tf[k] = sTf[k];
        // each lane takes its points tid, tid + T, tid + 2T, ... in order, U
        // per step with their loads overlapped
        for (int64_t i0 = tid; i0 < P.n_pts; i0 += U * kAlignThreads) {
            float J[U][6], r[U];
            bool ok[U];
            residual_u<U>(Tf, P.pts, i0, kAlignThreads, P.n_pts, vs, P.phi, P.page, d, J, r, ok);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!ok[u]) continue;
                double Jd[6];
#pragma unroll
                for (int a = 0; a < 6; ++a) Jd[a] = (double)J[u][a];
                const double rd = (double)r[u];
                int m = 0;
#pragma unroll
                for (int a = 0; a < 6; ++a)
#pragma unroll
                    for (int b = a; b < 6; ++b) acc[m++] += Jd[a] * Jd[b];
#pragma unroll
                for (int a = 0; a < 6; ++a) acc[21 + a] += Jd[a] * rd;
                acc[27] += rd * rd;
                acc[28] += 1.0;
            }
        }
#pragma unroll
        for (int k = 0; k < 29; ++k) {
            double v = acc[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
            if (lane == 0) red[wid][k] = v;
        }
        __syncthreads();
        if (tid < 29) {
            double v = 0.0;
            for (int w = 0; w < kAlignThreads / 64; ++w) v += red[w][tid];
            tot[tid] = v;
        }
        __syncthreads();
        bool stop = false;
        if (LM && tid == 0) {
            bool solve = true;
            if (!s_lm[0]) {  // sums at the start pose
                if (P.max_iter <= 0) {
                    stop = true;
                    solve = false;
                } else if (tot[28] < (double)n_min) {
                    s_state[2] = COVOX_EDEGENERATE;
                    stop = true;
                    solve = false;
                } else {
                    for (int k = 0; k < 29; ++k) sPrev[k] = tot[k];
                    s_lm[0] = 1;
                }
            } else {  // sums at the trial pose: take the step or raise the damping
                const double pred = lm_predicted(sPrev, sD);
                double rho = -1.0;
                if (tot[28] >= (double)n_min && pred > 0.0)
                    rho = (sPrev[27] / sPrev[28] - tot[27] / tot[28]) / (pred / sPrev[28]);
                if (rho > 0.0) {
                    for (int k = 0; k < 12; ++k) sT[k] = sTt[k];
                    for (int k = 0; k < 29; ++k) sPrev[k] = tot[k];
                    s_lm[1] += 1;
                    const double s = 2.0 * rho - 1.0, f = 1.0 - s * s * s;
                    sMu[0] *= f > 1.0 / 3.0 ? f : 1.0 / 3.0;
                    sMu[1] = 2.0;
                } else {
                    sMu[0] *= sMu[1];
                    sMu[1] *= 2.0;
                }
            }
            if (solve) {
                double dl[6];
                if (s_state[1] >= P.max_iter) {
                    stop = true;
                } else if (!(dof == 4 ? solve_xyz_yaw(sPrev, sMu[0], dl) : solve6(sPrev, sMu[0], dl))) {
                    s_state[2] = COVOX_EDEGENERATE;
                    stop = true;
                } else {
                    s_state[1] += 1;
                    const double nr = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
                    const double nt = sqrt(dl[3] * dl[3] + dl[4] * dl[4] + dl[5] * dl[5]);
                    if ((nr < tol_rho && nt < tol_theta) || lm_predicted(sPrev, dl) <= noise * sqrt(sPrev[27])) {
                        s_state[2] = COVOX_OK;  // converged; the step is not taken
                        stop = true;
                    } else {
                        double T[12];
                        for (int k = 0; k < 12; ++k) T[k] = sT[k];
                        se3_left_update(dl, T);
                        for (int k = 0; k < 6; ++k) sD[k] = dl[k];
                        for (int k = 0; k < 12; ++k) {
                            sTt[k] = T[k];
                            sTf[k] = (float)T[k];
                        }
                    }
                }
            }
            red[0][0] = stop ? 1.0 : 0.0;
        } else if (tid == 0) {
            if (s_state[0] || s_state[1] >= P.max_iter) {
                stop = true;
            } else if (tot[28] < (double)n_min) {
                s_state[2] = COVOX_EDEGENERATE;
                stop = true;
            } else {
                double dl[6];
                if (!(dof == 4 ? solve_xyz_yaw(tot, 0.0, dl) : solve6(tot, 0.0, dl))) {
                    s_state[2] = COVOX_EDEGENERATE;
                    stop = true;
                } else {
                    double T[12];
                    for (int k = 0; k < 12; ++k) T[k] = sT[k];
                    se3_left_update(dl, T);
                    for (int k = 0; k < 12; ++k) {
                        sT[k] = T[k];
                        sTf[k] = (float)T[k];
                    }
                    s_state[1] += 1;
                    const double nr = sqrt(dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2]);
                    const double nt = sqrt(dl[3] * dl[3] + dl[4] * dl[4] + dl[5] * dl[5]);
                    if (nr < tol_rho && nt < tol_theta) {
                        s_state[2] = COVOX_OK;
                        s_state[0] = 1;  // one more evaluation at the final pose
                    }
                }
            }
            red[0][0] = stop ? 1.0 : 0.0;
        }
        __syncthreads();
        stop = red[0][0] != 0.0;
        __syncthreads();
        if (stop) break;
    }
    if (tid == 0) {
        AlignResult &R = res[pid];
        const bool acc = LM && s_lm[0];  // LM: the sums of the accepted pose
        const double *ne = acc ? sPrev : tot;
        for (int k = 0; k < 12; ++k) R.T[k] = sT[k];
        R.T[12] = 0; R.T[13] = 0; R.T[14] = 0; R.T[15] = 1;
        for (int k = 0; k < 29; ++k) R.ne[k] = ne[k];
        R.n_used = (int64_t)ne[28];
        R.cost = ne[28] > 0 ? ne[27] / ne[28] : __builtin_inf();
        R.iters = acc ? s_lm[1] : s_state[1];
        R.solves = s_state[1];
        R.status = s_state[2];
    }
}

// ---------------------------------------------------------------- summaries

// ESDF value at q by trilinear interpolation of the 8 cell corners (the
// residual's operation order); false when a corner is unobserved.
__device__ __forceinline__ bool phi_trilinear(const float q[3], float vs, const float *phi, const int32_t *page,
                                              const DomArgs &d, float &r)
{
    float f[3];
    int j0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float g = (q[a] / vs) - 0.5f;
        if (!(fabsf(g) < 1.0e8f)) return false;
        const float fl = floorf(g);
        j0[a] = (int)fl;
        f[a] = g - fl;
    }
    float c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        c[k] = phi_at(phi, page, d, j0[0] + (k & 1), j0[1] + ((k >> 1) & 1), j0[2] + ((k >> 2) & 1));
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (isnan(c[k])) return false;
    const float wx0 = 1.0f - f[0], wx1 = f[0], wy0 = 1.0f - f[1], wy1 = f[1], wz0 = 1.0f - f[2], wz1 = f[2];
    const float c00 = c[0] * wx0 + c[1] * wx1, c10 = c[2] * wx0 + c[3] * wx1;
    const float c01 = c[4] * wx0 + c[5] * wx1, c11 = c[6] * wx0 + c[7] * wx1;
    const float c0 = c00 * wy0 + c10 * wy1, c1 = c01 * wy0 + c11 * wy1;
    r = c0 * wz0 + c1 * wz1;
    return true;
}

// One lane per cell of a 32^3 grid: cell centre ((i + 0.5) - 16) * cell in the
// grid frame, mapped to the submap by T (binary32, row-major 3x4); writes
// (clamp(phi / d_max, -1, 1), 1) or (0, 0) to channels chan, chan + 1 of a
// 4-channel NDHWC block.
__global__ __launch_bounds__(256) void k_summary(const SummaryReq *__restrict__ reqs, int n, float vs, float dmax)
{
    const int64_t total = (int64_t)n * 32768;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const SummaryReq &R = reqs[i >> 15];
        const int c = (int)(i & 32767);
        const int cx = c & 31, cy = (c >> 5) & 31, cz = c >> 10;
        const float g[3] = {(((float)cx + 0.5f) - 16.0f) * R.cell, (((float)cy + 0.5f) - 16.0f) * R.cell,
                            (((float)cz + 0.5f) - 16.0f) * R.cell};
        float q[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) q[a] = ((R.T[4 * a] * g[0] + R.T[4 * a + 1] * g[1]) + R.T[4 * a + 2] * g[2]) + R.T[4 * a + 3];
        const DomArgs d = dom_of(R.meta);
        float r, val = 0.0f, msk = 0.0f;
        if (phi_trilinear(q, vs, R.phi, R.page, d, r)) {
            val = fminf(1.0f, fmaxf(-1.0f, r / dmax));
            msk = 1.0f;
        }
        R.out[4 * c + R.chan] = val;
        R.out[4 * c + R.chan + 1] = msk;
    }
}

unsigned grid_waves(int64_t waves)
{
    const int64_t g = (waves + 3) / 4;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

int extract_points(covox_ctx *ctx, const covox_submap *Bc)
{
    // The registration points, the page and their versions are a cache the
    // library keeps inside the submap; the map itself (keys, D, W) is only
    // read here.
    covox_submap *B = const_cast<covox_submap *>(Bc);
    if (B->pts_version == B->version) return COVOX_OK;
    int rc;
    if ((rc = build_page(ctx, B))) return rc;
    const int64_t nbk = std::max<int64_t>(1, std::min(B->nb_upper, B->cap));
    if ((rc = ensure_buffer(ctx, (void **)&ctx->cnt, &ctx->cnt_cap, nbk, sizeof(uint32_t), "point counts"))) return rc;
    if ((rc = ensure_buffer(ctx, (void **)&ctx->psum, &ctx->psum_cap, nbk, 3 * sizeof(double), "point sums")))
        return rc;
    const covox_params &p = ctx->p;
    const float vs = (float)p.voxel_size, tau = (float)band_limit(p), wreg = (float)p.w_reg;
    const bool h = p.precision == COVOX_FP16;
    {
        TimedLaunch tl(ctx, COVOX_K_ISO);
        if (h)
            hipLaunchKernelGGL(k_iso<__half>, dim3(grid_waves(nbk)), dim3(256), 0, ctx->stream, B->meta, B->keys,
                               B->page, (const __half *)B->D, (const __half *)B->W, vs, tau, wreg, 0, ctx->cnt,
                               (float *)nullptr, (double *)nullptr);
        else
            hipLaunchKernelGGL(k_iso<float>, dim3(grid_waves(nbk)), dim3(256), 0, ctx->stream, B->meta, B->keys,
                               B->page, (const float *)B->D, (const float *)B->W, vs, tau, wreg, 0, ctx->cnt,
                               (float *)nullptr, (double *)nullptr);
        hipLaunchKernelGGL(k_iso_scan, dim3(1), dim3(1024), 0, ctx->stream, B->meta, ctx->cnt);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "point count launch"))) return rc;
    SubmapMeta m;
    if ((rc = hip_check(ctx, hipMemcpyAsync(&m, B->meta, sizeof(m), hipMemcpyDeviceToHost, ctx->stream), "meta copy")))
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "point count sync"))) return rc;
    const int64_t n = m.n_points;
    if ((rc = ensure_buffer(ctx, (void **)&B->pts, &B->pts_cap, std::max<int64_t>(n, 1), 3 * sizeof(float), "points")))
        return rc;
    {
        TimedLaunch tl(ctx, COVOX_K_ISO);
        if (h)
            hipLaunchKernelGGL(k_iso<__half>, dim3(grid_waves(nbk)), dim3(256), 0, ctx->stream, B->meta, B->keys,
                               B->page, (const __half *)B->D, (const __half *)B->W, vs, tau, wreg, 1, ctx->cnt, B->pts,
                               ctx->psum);
        else
            hipLaunchKernelGGL(k_iso<float>, dim3(grid_waves(nbk)), dim3(256), 0, ctx->stream, B->meta, B->keys,
                               B->page, (const float *)B->D, (const float *)B->W, vs, tau, wreg, 1, ctx->cnt, B->pts,
                               ctx->psum);
        hipLaunchKernelGGL(k_pbar, dim3(1), dim3(64), 0, ctx->stream, B->meta, ctx->psum);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "point write launch"))) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(&m, B->meta, sizeof(m), hipMemcpyDeviceToHost, ctx->stream), "meta copy")))
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "point write sync"))) return rc;
    B->n_pts = n;
    for (int a = 0; a < 3; ++a) B->pbar[a] = m.pbar[a];
    B->pts_version = B->version;
    return COVOX_OK;
}

int run_summaries(covox_ctx *ctx, const SummaryReq *reqs, int n)
{
    if (n <= 0) return COVOX_OK;
    int rc;
    const size_t bytes = sizeof(SummaryReq) * n;
    if ((rc = ensure_buffer(ctx, &ctx->sum_dev, &ctx->sum_cap, (int64_t)bytes, 1, "summary requests"))) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->sum_dev, reqs, bytes, hipMemcpyHostToDevice, ctx->stream),
                        "summary upload")))
        return rc;
    {
        TimedLaunch tl(ctx, COVOX_K_SUMMARY);
        const int64_t total = (int64_t)n * 32768;
        hipLaunchKernelGGL(k_summary, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 1 << 20)), dim3(256), 0,
                           ctx->stream, (const SummaryReq *)ctx->sum_dev, n, (float)ctx->p.voxel_size,
                           (float)ctx->p.d_max);
    }
    return hip_check(ctx, hipGetLastError(), "summary launch");
}

AlignLaunch align_launch_of(const covox_ctx *ctx)
{
    AlignLaunch L;
    L.vs = (float)ctx->p.voxel_size;
    L.tol_rho = ctx->p.tol_rho;
    L.tol_theta = ctx->p.tol_theta;
    L.n_min = ctx->p.n_min;
    L.dof = ctx->p.align_dof;
    L.lm = ctx->p.align_solver == COVOX_LEVENBERG_MARQUARDT;
    L.threads = ctx->tune.align_threads == 512 ? 512 : 256;
    L.pps = ctx->tune.align_points_per_step == 2 ? 2 : 1;
    return L;
}

void align_order(const AlignProblem *probs, int n, int32_t *order)
{
    // longest problems first so that the hardware dispatches them early
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order, order + n, [&](int a, int b) { return probs[a].n_pts > probs[b].n_pts; });
}

int launch_alignment(covox_ctx *ctx, const AlignProblem *dprob, const int32_t *dorder, int n, AlignResult *dres,
                     const AlignLaunch &L)
{
    if (n <= 0) return COVOX_OK;
    {
        TimedLaunch tl(ctx, COVOX_K_ALIGN);
        const int shape = (L.threads == 512 ? 4 : 0) + (L.pps == 2 ? 2 : 0) + (L.lm ? 1 : 0);
        switch (shape) {
#define COVOX_ALIGN_LAUNCH(S, NT, U, LM)                                                                       \
    case S:                                                                                                    \
        hipLaunchKernelGGL((k_align<NT, U, LM>), dim3(n), dim3(NT), 0, ctx->stream, dprob, dorder, dres, L.vs, \
                           L.tol_rho, L.tol_theta, L.n_min, L.dof);                                            \
        break;
            COVOX_ALIGN_LAUNCH(0, 256, 1, false)
            COVOX_ALIGN_LAUNCH(1, 256, 1, true)
            COVOX_ALIGN_LAUNCH(2, 256, 2, false)
            COVOX_ALIGN_LAUNCH(3, 256, 2, true)
            COVOX_ALIGN_LAUNCH(4, 512, 1, false)
            COVOX_ALIGN_LAUNCH(5, 512, 1, true)
            COVOX_ALIGN_LAUNCH(6, 512, 2, false)
            COVOX_ALIGN_LAUNCH(7, 512, 2, true)
#undef COVOX_ALIGN_LAUNCH
        }
    }
    return hip_check(ctx, hipGetLastError(), "align launch");
}

int run_alignment(covox_ctx *ctx, const AlignProblem *probs, int n, AlignResult *res)
{
    if (n <= 0) return COVOX_OK;
    int rc;
    const size_t pbytes = sizeof(AlignProblem) * n + sizeof(int32_t) * n;
    if ((rc = ensure_buffer(ctx, &ctx->prob_dev, &ctx->prob_cap, (int64_t)pbytes, 1, "problems"))) return rc;
    if ((rc = ensure_buffer(ctx, &ctx->res_dev, &ctx->res_cap, (int64_t)(sizeof(AlignResult) * n), 1, "results")))
        return rc;
    std::vector<char> stage(pbytes);
    ::memcpy(stage.data(), probs, sizeof(AlignProblem) * n);
    align_order(probs, n, (int32_t *)(stage.data() + sizeof(AlignProblem) * n));
    if ((rc = hip_check(ctx, hipMemcpyAsync(ctx->prob_dev, stage.data(), pbytes, hipMemcpyHostToDevice, ctx->stream),
                        "problem upload")))
        return rc;
    const AlignProblem *dprob = (const AlignProblem *)ctx->prob_dev;
    const int32_t *dorder = (const int32_t *)((const char *)ctx->prob_dev + sizeof(AlignProblem) * n);
    if ((rc = launch_alignment(ctx, dprob, dorder, n, (AlignResult *)ctx->res_dev, align_launch_of(ctx)))) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(res, ctx->res_dev, sizeof(AlignResult) * n, hipMemcpyDeviceToHost,
                                            ctx->stream),
                        "result copy")))
        return rc;
    return hip_check(ctx, hipStreamSynchronize(ctx->stream), "align sync");
}

}  // namespace covox
