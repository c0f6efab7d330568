/*
 * covox oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of what the GPU library computes, used by
 * the tests, the smoke check and the CPU-baseline leg of the benchmark.  It
 * shares no code with the GPU library and is never called by it.
 *
 * Paper: Hoss and De Cristoforis, "coVoxSLAM: GPU accelerated globally
 * consistent dense SLAM" (arXiv 2410.21149).
 *
 *   integrate   Sec. III-C (projection mapping: a voxel's distance is the
 *               depth value minus the voxel depth; blocks of n^3 voxels
 *               indexed by 3-D position), Sec. III-D (count new blocks,
 *               allocate them from a pre-allocated buffer, then update; the
 *               weight/distance update is commutative).
 *   raycast     Sec. III-C (rays from the optical centre through every
 *               observed point; all voxels crossed up to the truncation
 *               distance behind the point are updated; every point counts),
 *               Sec. III-D (count and allocate new blocks, then reduce all
 *               contributions of the frame per voxel in address order).
 *   esdf        Sec. I and Sec. III-E (Euclidean distance to the nearest
 *               obstacle built from the TSDF, reusing the distances inside the
 *               truncation band; exact EDT in the PBA lineage).
 *   wavefront   Sec. III-E (incremental update: newly occupied and freed
 *               voxels seed per-block work, each block is swept along every
 *               axis, block faces pass better distances to the neighbours,
 *               repeated until nothing changes).
 *   align       Sec. I and Sec. III-F, Eq. (1) registration term
 *               (correspondence-free ESDF alignment, registration points
 *               chosen by weight, least squares on residuals/Jacobians;
 *               Gauss-Newton, or Levenberg-Marquardt with a trust region
 *               as Sec. III-F names for the backend).
 *   hash        Sec. III-B (blocks indexed by their 3-D position through a
 *               hash table with open addressing) and the hash-table stress
 *               test of Sec. IV: keys inserted one after another, each in
 *               the first empty slot from its home slot upwards (linear
 *               probing, wrapping at the end).
 *
 * Two numeric modes:
 *   binary32  every arithmetic step rounded to binary32 in the pinned
 *             operation order (no FMA contraction; build with
 *             -ffp-contract=off and without fast-math), sums of the
 *             normal equations in binary64;
 *   binary64  the same definitions in binary64 (for error statements).
 * Optional binary16 storage of distance and weight (binary32 arithmetic).
 *
 * Threads: the loops over independent items -- the voxels of the frustum
 * box, the valid voxels of a frame, the lines of an EDT pass, the blocks of
 * the final values -- run under OpenMP (orc_set_threads); every item writes
 * its own outputs and the per-thread lists are joined in sequential order,
 * so the results are bit-identical for any thread count.
 *
 * Every function is a direct transcription of a definition: brute-force
 * voxel enumeration over a box that contains the camera frustum, sorted key
 * arrays with binary search, the Felzenszwalb-Huttenlocher lower-envelope
 * exact EDT (a textbook algorithm, Theory of Computing 8, 2012), dense
 * Cholesky.  Nothing here is tuned.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EDEGENERATE (-5)
#define ORC_NOT_CONVERGED 1

typedef struct {
    double vs;         /* voxel edge (m) */
    int trunc_vox;     /* truncation distance in voxels */
    double max_range;  /* depth values above this are ignored (m) */
    double d_max;      /* ESDF range (m) */
    double w_reg;      /* minimum weight of registration-point endpoints */
    int fp64;          /* 0: binary32 mode, 1: binary64 mode */
    int fp16;          /* binary16 storage of D and W (binary32 mode only) */
    int max_iter;      /* Gauss-Newton iteration cap */
    int n_min;         /* minimum number of residuals */
    double tol_rho;    /* Gauss-Newton stop: |step translation| below this (m) ... */
    double tol_theta;  /* ... and |step rotation| below this (rad) */
    int align_dof;     /* 6, or 4: translation and yaw only (gravity-aligned submaps) */
    int weight_mode;   /* 0: weight 1 per observation; 1: weight 1 / d^2 (d = measured depth, m) */
    int integrator;    /* 0: projection mapping; 1: raycasting */
    int ray_carve;     /* raycasting: 1 = rays start at the optical centre; 0 = at tau before the point */
    int esdf_mode;     /* 0: exact EDT recomputed; 1: incremental wavefront (nearest-site propagation) */
    int align_solver;  /* 0: Gauss-Newton; 1: Levenberg-Marquardt with the gain-ratio trust region */
} orc_params;

typedef struct {
    orc_params p;
    double T_ws[16];
    int64_t n, cap;
    uint64_t *keys;     /* buffer order */
    uint64_t *skeys;    /* sorted keys */
    int64_t *sidx;      /* buffer index of skeys[j] */
    float *D, *W;       /* binary32 values (binary16-rounded when fp16) */
    double *D64, *W64;  /* binary64 mode */
    float *phi;
    double *phi64;
    int32_t *ksq;       /* squared EDT distance in voxels^2; -1 in band / unobserved */
    /* wavefront ESDF state (esdf_mode 1) */
    int32_t *wk;        /* squared distance to the parent site (voxels^2), or WF_INF */
    int32_t *wpar;      /* parent site as a packed offset from the voxel, or WF_NONE */
    uint8_t *wsite;     /* site flag at the last update */
    int64_t wn;         /* blocks at the last update */
    /* raycasting: voxels next to fragile walk steps (x, y, z triples), all frames */
    int64_t *frag;
    int64_t n_frag, frag_cap;
} orc_submap;

/* ------------------------------------------------------------ keys */

#define KEY_OFF 1048576LL /* 2^20 */

static uint64_t pack_key(int64_t bx, int64_t by, int64_t bz)
{
    return ((uint64_t)(bx + KEY_OFF) << 42) | ((uint64_t)(by + KEY_OFF) << 21) |
           (uint64_t)(bz + KEY_OFF);
}

static void unpack_key(uint64_t k, int64_t b[3])
{
    b[0] = (int64_t)((k >> 42) & 0x1FFFFF) - KEY_OFF;
    b[1] = (int64_t)((k >> 21) & 0x1FFFFF) - KEY_OFF;
    b[2] = (int64_t)(k & 0x1FFFFF) - KEY_OFF;
}

/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y ? 1 : 0;
}

/* Buffer index of block key k, or -1 (binary search in the sorted copy). */
static int64_t find_block(const orc_submap *s, uint64_t k)
{
    int64_t lo = 0, hi = s->n - 1;
    while (lo <= hi) {
        int64_t m = lo + (hi - lo) / 2;
        if (s->skeys[m] == k) return s->sidx[m];
        if (s->skeys[m] < k) lo = m + 1; else hi = m - 1;
    }
    return -1;
}

static void rebuild_sorted(orc_submap *s)
{
    /* sort (key, idx) pairs by key: plain insertion of indices then qsort on
     * a combined array */
    typedef struct { uint64_t k; int64_t i; } kv;
    kv *tmp = (kv *)malloc(sizeof(kv) * (size_t)(s->n > 0 ? s->n : 1));
    for (int64_t i = 0; i < s->n; ++i) { tmp[i].k = s->keys[i]; tmp[i].i = i; }
    qsort(tmp, (size_t)s->n, sizeof(kv), cmp_u64); /* k is the first member */
    for (int64_t i = 0; i < s->n; ++i) { s->skeys[i] = tmp[i].k; s->sidx[i] = tmp[i].i; }
    free(tmp);
}

/* -------------------------------------------------------- binary16 */

/* binary32 -> binary16, round to nearest even (IEEE 754). */
uint16_t orc_f2h(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    uint32_t sign = (x >> 16) & 0x8000u;
    uint32_t e = (x >> 23) & 0xFFu;
    uint32_t m = x & 0x7FFFFFu;
    if (e == 0xFFu) return (uint16_t)(sign | 0x7C00u | (m ? 0x200u : 0u));
    int32_t E = (int32_t)e - 127 + 15;
    if (E >= 31) return (uint16_t)(sign | 0x7C00u);
    if (E <= 0) {
        /* subnormal half (or zero): value = m_full * 2^(e-150); half
         * subnormal unit is 2^-24 */
        if (E < -10) return (uint16_t)sign;
        uint32_t mf = m | 0x800000u;       /* 24-bit significand */
        int shift = 14 - E;                /* bits to drop: (e-150) - (-24) negated */
        uint32_t q = mf >> shift;
        uint32_t rem = mf & ((1u << shift) - 1u);
        uint32_t half = 1u << (shift - 1);
        if (rem > half || (rem == half && (q & 1u))) q += 1u;
        return (uint16_t)(sign | q);
    }
    uint32_t q = ((uint32_t)E << 10) | (m >> 13);
    uint32_t rem = m & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (q & 1u))) q += 1u; /* may carry into exponent */
    return (uint16_t)(sign | q);
}

float orc_h2f(uint16_t h)
{
    uint32_t sign = ((uint32_t)h & 0x8000u) << 16;
    uint32_t e = (h >> 10) & 0x1Fu;
    uint32_t m = h & 0x3FFu;
    float v;
    if (e == 0) {
        v = (float)m * 5.9604644775390625e-08f; /* m * 2^-24, exact */
        uint32_t x;
        memcpy(&x, &v, 4);
        x |= sign;
        memcpy(&v, &x, 4);
        return v;
    }
    uint32_t x;
    if (e == 31) x = sign | 0x7F800000u | (m << 13);
    else x = sign | ((e - 15 + 127) << 23) | (m << 13);
    memcpy(&v, &x, 4);
    return v;
}

static float round_store(const orc_submap *s, float v)
{
    return s->p.fp16 ? orc_h2f(orc_f2h(v)) : v;
}

/* ------------------------------------------------------ rigid poses */

/* Rigid inverse of a row-major 4x4 [R t; 0 1]: [R^T, -R^T t]. */
static void rigid_inverse(const double *T, double *O)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) O[4 * r + c] = T[4 * c + r];
    for (int r = 0; r < 3; ++r)
        O[4 * r + 3] = -((O[4 * r + 0] * T[3] + O[4 * r + 1] * T[7]) + O[4 * r + 2] * T[11]);
    O[12] = 0; O[13] = 0; O[14] = 0; O[15] = 1;
}

/* Product of two rigid transforms, fixed summation order. */
static void rigid_mul(const double *A, const double *B, double *O)
{
    double t[16];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            t[4 * r + c] = (A[4 * r + 0] * B[c] + A[4 * r + 1] * B[4 + c]) + A[4 * r + 2] * B[8 + c];
        t[4 * r + 3] = ((A[4 * r + 0] * B[3] + A[4 * r + 1] * B[7]) + A[4 * r + 2] * B[11]) + A[4 * r + 3];
    }
    t[12] = 0; t[13] = 0; t[14] = 0; t[15] = 1;
    memcpy(O, t, sizeof(t));
}

void orc_pose_cam_sub(const double *T_wc, const double *T_ws, double *T_cs)
{
    double inv[16];
    rigid_inverse(T_wc, inv);
    rigid_mul(inv, T_ws, T_cs);
}

/* ------------------------------------------------------- submap */

orc_submap *orc_submap_create(const orc_params *p, const double *T_ws)
{
    orc_submap *s = (orc_submap *)calloc(1, sizeof(orc_submap));
    s->p = *p;
    memcpy(s->T_ws, T_ws, sizeof(s->T_ws));
    return s;
}

/* Replaces the alignment solver's parameters (max_iter, n_min, tol_rho,
 * tol_theta, align_dof, align_solver); the map is untouched. */
void orc_set_solver(orc_submap *s, const orc_params *p)
{
    s->p.max_iter = p->max_iter;
    s->p.n_min = p->n_min;
    s->p.tol_rho = p->tol_rho;
    s->p.tol_theta = p->tol_theta;
    s->p.align_dof = p->align_dof;
    s->p.align_solver = p->align_solver;
}

void orc_submap_destroy(orc_submap *s)
{
    if (!s) return;
    free(s->keys); free(s->skeys); free(s->sidx);
    free(s->D); free(s->W); free(s->D64); free(s->W64);
    free(s->phi); free(s->phi64); free(s->ksq);
    free(s->wk); free(s->wpar); free(s->wsite); free(s->frag);
    free(s);
}

static void grow(orc_submap *s, int64_t need)
{
    if (need <= s->cap) return;
    int64_t nc = s->cap ? s->cap : 256;
    while (nc < need) nc *= 2;
    s->keys = (uint64_t *)realloc(s->keys, sizeof(uint64_t) * nc);
    s->skeys = (uint64_t *)realloc(s->skeys, sizeof(uint64_t) * nc);
    s->sidx = (int64_t *)realloc(s->sidx, sizeof(int64_t) * nc);
    if (s->p.fp64) {
        s->D64 = (double *)realloc(s->D64, sizeof(double) * 512 * nc);
        s->W64 = (double *)realloc(s->W64, sizeof(double) * 512 * nc);
        s->phi64 = (double *)realloc(s->phi64, sizeof(double) * 512 * nc);
    } else {
        s->D = (float *)realloc(s->D, sizeof(float) * 512 * nc);
        s->W = (float *)realloc(s->W, sizeof(float) * 512 * nc);
        s->phi = (float *)realloc(s->phi, sizeof(float) * 512 * nc);
    }
    s->ksq = (int32_t *)realloc(s->ksq, sizeof(int32_t) * 512 * nc);
    s->wk = (int32_t *)realloc(s->wk, sizeof(int32_t) * 512 * nc);
    s->wpar = (int32_t *)realloc(s->wpar, sizeof(int32_t) * 512 * nc);
    s->wsite = (uint8_t *)realloc(s->wsite, 512 * nc);
    s->cap = nc;
}

int64_t orc_n_blocks(const orc_submap *s) { return s->n; }

/* Threads of the parallel loops (n < 1: all cores); returns the count now in use. */
int orc_set_threads(int n)
{
    omp_set_num_threads(n >= 1 ? n : omp_get_num_procs());
    return omp_get_max_threads();
}

static int64_t floordiv8(int64_t v) { return v >= 0 ? v / 8 : -((-v + 7) / 8); }

static int lin_index(int64_t ix, int64_t iy, int64_t iz)
{
    return (int)((ix & 7) + 8 * (iy & 7) + 64 * (iz & 7));
}

/* ------------------------------------------------------- integrate */

typedef struct { int64_t i[3]; double sdf, d; } valid_vox;

/* Projective validity of voxel i under camera pose T_cs (Sec. III-C),
 * binary32 pinned order.  Returns 1 and the signed distance when valid. */
static int valid32(const float R[9], const float t[3], float vs_f, float tau_f, float maxr_f,
                   const float K[4], const float *depth, int H, int W, const int64_t i[3],
                   float *sdf_out, float *d_out)
{
    float c[3], p[3];
    for (int a = 0; a < 3; ++a) c[a] = ((float)i[a] + 0.5f) * vs_f;
    for (int k = 0; k < 3; ++k) p[k] = ((R[3 * k + 0] * c[0] + R[3 * k + 1] * c[1]) + R[3 * k + 2] * c[2]) + t[k];
    if (!(p[2] > 0.0f)) return 0;
    float u = ((K[0] * p[0]) / p[2]) + K[2];
    float v = ((K[1] * p[1]) / p[2]) + K[3];
    float uf = floorf(u + 0.5f);
    float vf = floorf(v + 0.5f);
    if (!(uf >= 0.0f && uf < (float)W && vf >= 0.0f && vf < (float)H)) return 0;
    int col = (int)uf, row = (int)vf;
    float d = depth[(size_t)row * W + col];
    if (!(d > 0.0f && d <= maxr_f)) return 0;
    float sdf = d - p[2];
    if (!(sdf >= -tau_f)) return 0;
    *sdf_out = sdf;
    *d_out = d;
    return 1;
}

/* The same test in binary64. */
static int valid64(const double R[9], const double t[3], double vs, double tau, double maxr,
                   const float K[4], const float *depth, int H, int W, const int64_t i[3],
                   double *sdf_out, double *d_out)
{
    double c[3], p[3];
    for (int a = 0; a < 3; ++a) c[a] = ((double)i[a] + 0.5) * vs;
    for (int k = 0; k < 3; ++k) p[k] = ((R[3 * k + 0] * c[0] + R[3 * k + 1] * c[1]) + R[3 * k + 2] * c[2]) + t[k];
    if (!(p[2] > 0.0)) return 0;
    double u = ((K[0] * p[0]) / p[2]) + K[2];
    double v = ((K[1] * p[1]) / p[2]) + K[3];
    double uf = floor(u + 0.5);
    double vf = floor(v + 0.5);
    if (!(uf >= 0.0 && uf < (double)W && vf >= 0.0 && vf < (double)H)) return 0;
    int col = (int)uf, row = (int)vf;
    double d = depth[(size_t)row * W + col];
    if (!(d > 0.0 && d <= maxr)) return 0;
    double sdf = d - p[2];
    if (!(sdf >= -tau)) return 0;
    *sdf_out = sdf;
    *d_out = d;
    return 1;
}

/* Voxel index box that contains every voxel centre inside the viewing
 * frustum cut at depth max_range + tau: the bounding box of the camera
 * centre and the four far-plane corners through the image's outer pixel
 * edges, widened by one voxel. */
static void frustum_box(const orc_submap *s, const float K[4], int H, int W, const double *T_wc,
                        int64_t lo[3], int64_t hi[3])
{
    double inv_ws[16], T_sc[16];
    rigid_inverse(s->T_ws, inv_ws);
    rigid_mul(inv_ws, T_wc, T_sc);
    double zf = s->p.max_range + s->p.trunc_vox * s->p.vs;
    double us[2] = {-0.5, W - 0.5}, vsv[2] = {-0.5, H - 0.5};
    double mn[3], mx[3];
    for (int a = 0; a < 3; ++a) { mn[a] = T_sc[4 * a + 3]; mx[a] = T_sc[4 * a + 3]; }
    for (int iu = 0; iu < 2; ++iu)
        for (int iv = 0; iv < 2; ++iv) {
            double pc[3] = {(us[iu] - K[2]) / K[0] * zf, (vsv[iv] - K[3]) / K[1] * zf, zf};
            for (int a = 0; a < 3; ++a) {
                double w = T_sc[4 * a + 0] * pc[0] + T_sc[4 * a + 1] * pc[1] + T_sc[4 * a + 2] * pc[2] + T_sc[4 * a + 3];
                if (w < mn[a]) mn[a] = w;
                if (w > mx[a]) mx[a] = w;
            }
        }
    for (int a = 0; a < 3; ++a) {
        lo[a] = (int64_t)floor(mn[a] / s->p.vs - 0.5) - 1;
        hi[a] = (int64_t)ceil(mx[a] / s->p.vs - 0.5) + 1;
    }
}

/* Blocks touched by a frame: keys tk[0..n) (any order, duplicates allowed)
 * are sorted and deduplicated in place; blocks not yet allocated get buffer
 * indices n + rank in ascending key order (Sec. III-D: count, then allocate
 * from the pre-allocated buffer).  Returns the number of new blocks and sets
 * *n_touched. */
static int64_t allocate_touched(orc_submap *s, uint64_t *tk, size_t n, size_t *n_touched)
{
    qsort(tk, n, sizeof(uint64_t), cmp_u64);
    size_t nt = 0;
    for (size_t j = 0; j < n; ++j)
        if (nt == 0 || tk[nt - 1] != tk[j]) tk[nt++] = tk[j];
    int64_t n_new = 0;
    int64_t n0 = s->n;
    grow(s, s->n + (int64_t)nt);
    for (size_t j = 0; j < nt; ++j) {  /* tk is ascending: ranks follow key order */
        if (find_block(s, tk[j]) >= 0) continue;
        int64_t idx = n0 + n_new;
        s->keys[idx] = tk[j];
        for (int l = 0; l < 512; ++l) {
            if (s->p.fp64) { s->D64[512 * idx + l] = 0.0; s->W64[512 * idx + l] = 0.0; }
            else { s->D[512 * idx + l] = 0.0f; s->W[512 * idx + l] = 0.0f; }
            s->ksq[512 * idx + l] = -1;
            if (s->p.fp64) s->phi64[512 * idx + l] = NAN; else s->phi[512 * idx + l] = NAN;
        }
        ++n_new;
    }
    s->n = n0 + n_new;
    rebuild_sorted(s);
    *n_touched = nt;
    return n_new;
}

/*
 * Integrate one depth frame (Sec. III-C projection mapping; Sec. III-D
 * count / allocate / update).
 *   1. every voxel i of the frustum box is tested with valid(i);
 *   2. Touched = blocks holding a valid voxel; New = Touched minus the
 *      allocated blocks; new blocks get buffer indices n + rank in
 *      ascending packed-key order;
 *   3. each valid voxel: t = min(sdf, tau); W' = W + 1; D' = (D W + t) / W'.
 * stats (nullable): [n_new, n_touched, n_valid, n_valid].
 */
int orc_integrate_raycast(orc_submap *s, const float *depth, int H, int W, const float K[4],
                          const double *T_wc, int64_t *stats);

int orc_integrate(orc_submap *s, const float *depth, int H, int W, const float K[4],
                  const double *T_wc, int64_t *stats)
{
    if (H <= 0 || W <= 0 || !(K[0] > 0) || !(K[1] > 0)) return ORC_EINVAL;
    if (s->p.integrator == 1) return orc_integrate_raycast(s, depth, H, W, K, T_wc, stats);
    double T_cs[16];
    orc_pose_cam_sub(T_wc, s->T_ws, T_cs);
    int64_t lo[3], hi[3];
    frustum_box(s, K, H, W, T_wc, lo, hi);

    float R32[9], t32[3];
    double R64[9], t64[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) { R32[3 * r + c] = (float)T_cs[4 * r + c]; R64[3 * r + c] = T_cs[4 * r + c]; }
        t32[r] = (float)T_cs[4 * r + 3];
        t64[r] = T_cs[4 * r + 3];
    }
    const double tau = s->p.trunc_vox * s->p.vs;
    const float vs_f = (float)s->p.vs, tau_f = (float)tau, maxr_f = (float)s->p.max_range;

    /* 1. brute-force validity over the box: each thread scans a contiguous
     * range of x slices into a list of its own; the lists are joined in
     * thread order, which is the sequential (x, y, z) order */
    const int nthr = omp_get_max_threads();
    valid_vox **tv = (valid_vox **)calloc((size_t)nthr, sizeof(valid_vox *));
    size_t *tn = (size_t *)calloc((size_t)nthr, sizeof(size_t));
#pragma omp parallel num_threads(nthr)
    {
        const int th = omp_get_thread_num(), nt_ = omp_get_num_threads();
        const int64_t nx = hi[0] - lo[0] + 1;
        const int64_t x0 = lo[0] + nx * th / nt_, x1 = lo[0] + nx * (th + 1) / nt_;
        size_t nv_t = 0, cap_t = 1 << 12;
        valid_vox *vt = (valid_vox *)malloc(sizeof(valid_vox) * cap_t);
        int64_t i[3];
        for (i[0] = x0; i[0] < x1; ++i[0])
            for (i[1] = lo[1]; i[1] <= hi[1]; ++i[1])
                for (i[2] = lo[2]; i[2] <= hi[2]; ++i[2]) {
                    int ok;
                    double sdf, dd;
                    if (s->p.fp64) {
                        ok = valid64(R64, t64, s->p.vs, tau, s->p.max_range, K, depth, H, W, i, &sdf, &dd);
                    } else {
                        float sf, df;
                        ok = valid32(R32, t32, vs_f, tau_f, maxr_f, K, depth, H, W, i, &sf, &df);
                        sdf = sf;
                        dd = df;
                    }
                    if (!ok) continue;
                    if (nv_t == cap_t) { cap_t *= 2; vt = (valid_vox *)realloc(vt, sizeof(valid_vox) * cap_t); }
                    vt[nv_t].i[0] = i[0]; vt[nv_t].i[1] = i[1]; vt[nv_t].i[2] = i[2];
                    vt[nv_t].sdf = sdf;
                    vt[nv_t].d = dd;
                    ++nv_t;
                }
        tv[th] = vt;
        tn[th] = nv_t;
    }
    size_t nv = 0;
    for (int th = 0; th < nthr; ++th) nv += tn[th];
    valid_vox *vv = (valid_vox *)malloc(sizeof(valid_vox) * (nv ? nv : 1));
    size_t o = 0;
    for (int th = 0; th < nthr; ++th) {
        if (tn[th]) memcpy(vv + o, tv[th], sizeof(valid_vox) * tn[th]);
        o += tn[th];
        free(tv[th]);
    }
    free(tv);
    free(tn);

    /* 2. touched and new blocks */
    uint64_t *tk = (uint64_t *)malloc(sizeof(uint64_t) * (nv ? nv : 1));
    for (size_t j = 0; j < nv; ++j)
        tk[j] = pack_key(floordiv8(vv[j].i[0]), floordiv8(vv[j].i[1]), floordiv8(vv[j].i[2]));
    size_t nt = 0;
    const int64_t n_new = allocate_touched(s, tk, nv, &nt);

    /* 3. update every valid voxel (each voxel of the box appears at most
     * once, so the updates are independent) */
#pragma omp parallel for schedule(static)
    for (size_t j = 0; j < nv; ++j) {
        const int64_t *v = vv[j].i;
        int64_t idx = find_block(s, pack_key(floordiv8(v[0]), floordiv8(v[1]), floordiv8(v[2])));
        size_t o = (size_t)512 * idx + lin_index(v[0], v[1], v[2]);
        /* observation weight (Sec. III-C: weights may follow the sensor's
         * performance curve): 1, or 1 / d^2 for a depth noise that grows with
         * the distance */
        if (s->p.fp64) {
            double t = vv[j].sdf < tau ? vv[j].sdf : tau;
            double w = s->p.weight_mode ? 1.0 / (vv[j].d * vv[j].d) : 1.0;
            double Wn = s->W64[o] + w;
            s->D64[o] = ((s->D64[o] * s->W64[o]) + (t * w)) / Wn;
            s->W64[o] = Wn;
        } else {
            float t = fminf((float)vv[j].sdf, tau_f);
            const float df = (float)vv[j].d;
            float w = s->p.weight_mode ? 1.0f / (df * df) : 1.0f;
            float Wold = s->W[o], Dold = s->D[o];
            float Wn = Wold + w;
            float Dn = ((Dold * Wold) + (t * w)) / Wn;
            s->D[o] = round_store(s, Dn);
            s->W[o] = round_store(s, Wn);
        }
    }
    if (stats) { stats[0] = n_new; stats[1] = (int64_t)nt; stats[2] = (int64_t)nv; stats[3] = (int64_t)nv; }
    free(tk);
    free(vv);
    return ORC_OK;
}

/* ---------------------------------------------------------- raycast */

/*
 * Voxels crossed by the segment o + s u, s in [s0, s1], of a ray with unit
 * direction u: the grid traversal of Amanatides and Woo (Eurographics 1987).
 * The walk starts in the voxel holding o + s0 u.  In voxel i the ray leaves
 * through the boundary plane of axis a at the parameter that solves
 * o_a + s u_a = (i_a + [u_a > 0]) vs, that is
 *   s_a = ((i_a + [u_a > 0]) vs - o_a) / u_a
 * (one correctly rounded division; infinite when u_a = 0).  The smallest s_a
 * (x before y before z on ties) moves axis a by one voxel; the walk ends once
 * that smallest s_a is not below s1.  At most max_out voxels (3 ceil((s1 -
 * s0) / vs) + 6 bounds the walk) are written to out as (x, y, z) triples;
 * returns the number written.
 *
 * Fragile steps.  A different but still faithful rounding of the crossing
 * parameters (each within eps/2 of the exact quotient, relative) can change a
 * step only where two candidates are that close.  With m the smallest s_a
 * and eps = 2^-21 (binary32; 2^-50 in binary64), axis a is in doubt when
 * s_a - m <= eps |s_a|, and the end test when |m - s1| <= eps max(|m|, |s1|).
 * At a step where two or more axes are in doubt, or the end test is, every
 * voxel another choice could enter next is appended to frag (nullable; at
 * most max_frag triples, *n_frag counts them all): i moved along a subset of
 * the axes in doubt -- the proper non-empty subsets, or all non-empty subsets
 * when the end test is in doubt too (then the walk may stop before any).
 */
static void walk_frag(const int64_t i[3], const int step[3], const int doubt[3], int end_doubt, int64_t *frag,
                      int64_t max_frag, int64_t *n_frag)
{
    int nd = doubt[0] + doubt[1] + doubt[2];
    if (nd < 2 && !end_doubt) return;
    for (int mask = 1; mask < 8; ++mask) {
        int ok = 1, full = 1;
        for (int a = 0; a < 3; ++a) {
            if ((mask >> a) & 1) ok &= doubt[a];
            else if (doubt[a]) full = 0;
        }
        if (!ok || (full && !end_doubt)) continue;
        if (frag && *n_frag < max_frag)
            for (int a = 0; a < 3; ++a) frag[3 * *n_frag + a] = i[a] + (((mask >> a) & 1) ? step[a] : 0);
        ++*n_frag;
    }
}

static int64_t ray_walk32_frag(const float o[3], const float u[3], float s0, float s1, float vs, int64_t *out,
                               int64_t max_out, int64_t *frag, int64_t max_frag, int64_t *n_frag)
{
    const float eps = 0x1p-21f;
    int64_t i[3];
    int step[3];
    float sn[3];
    for (int a = 0; a < 3; ++a) {
        const float e = o[a] + s0 * u[a];
        i[a] = (int64_t)floorf(e / vs);
        step[a] = u[a] > 0.0f ? 1 : (u[a] < 0.0f ? -1 : 0);
    }
    int64_t n = 0;
    while (n < max_out) {
        out[3 * n + 0] = i[0]; out[3 * n + 1] = i[1]; out[3 * n + 2] = i[2];
        ++n;
        for (int a = 0; a < 3; ++a)
            sn[a] = step[a] ? (((float)(i[a] + (step[a] > 0)) * vs) - o[a]) / u[a] : INFINITY;
        int a = 0;
        if (sn[1] < sn[a]) a = 1;
        if (sn[2] < sn[a]) a = 2;
        const float m = sn[a];
        int doubt[3];
        for (int b = 0; b < 3; ++b) doubt[b] = step[b] && sn[b] - m <= eps * fabsf(sn[b]);
        const int end_doubt = fabsf(m - s1) <= eps * fmaxf(fabsf(m), fabsf(s1));
        if (n_frag) walk_frag(i, step, doubt, end_doubt, frag, max_frag, n_frag);
        if (!(m < s1)) break;
        i[a] += step[a];
    }
    return n;
}

int64_t orc_ray_walk32(const float o[3], const float u[3], float s0, float s1, float vs, int64_t *out,
                       int64_t max_out)
{
    return ray_walk32_frag(o, u, s0, s1, vs, out, max_out, NULL, 0, NULL);
}

/* The walk with its fragile steps (frag: max_frag triples; returns the
 * voxel count, *n_frag the fragile voxels). */
int64_t orc_ray_walk32_fragile(const float o[3], const float u[3], float s0, float s1, float vs, int64_t *out,
                               int64_t max_out, int64_t *frag, int64_t max_frag, int64_t *n_frag)
{
    *n_frag = 0;
    return ray_walk32_frag(o, u, s0, s1, vs, out, max_out, frag, max_frag, n_frag);
}

/* The same walk in binary64. */
static int64_t ray_walk64(const double o[3], const double u[3], double s0, double s1, double vs, int64_t *out,
                          int64_t max_out, int64_t *frag, int64_t max_frag, int64_t *n_frag)
{
    const double eps = 0x1p-50;
    int64_t i[3];
    int step[3];
    double sn[3];
    for (int a = 0; a < 3; ++a) {
        const double e = o[a] + s0 * u[a];
        i[a] = (int64_t)floor(e / vs);
        step[a] = u[a] > 0.0 ? 1 : (u[a] < 0.0 ? -1 : 0);
    }
    int64_t n = 0;
    while (n < max_out) {
        out[3 * n + 0] = i[0]; out[3 * n + 1] = i[1]; out[3 * n + 2] = i[2];
        ++n;
        for (int a = 0; a < 3; ++a)
            sn[a] = step[a] ? (((double)(i[a] + (step[a] > 0)) * vs) - o[a]) / u[a] : INFINITY;
        int a = 0;
        if (sn[1] < sn[a]) a = 1;
        if (sn[2] < sn[a]) a = 2;
        const double m = sn[a];
        int doubt[3];
        for (int b = 0; b < 3; ++b) doubt[b] = step[b] && sn[b] - m <= eps * fabs(sn[b]);
        const int end_doubt = fabs(m - s1) <= eps * fmax(fabs(m), fabs(s1));
        if (n_frag) walk_frag(i, step, doubt, end_doubt, frag, max_frag, n_frag);
        if (!(m < s1)) break;
        i[a] += step[a];
    }
    return n;
}

static void frag_append(orc_submap *s, const int64_t *v, int64_t n)
{
    if (n <= 0) return;
    if (s->n_frag + n > s->frag_cap) {
        s->frag_cap = 2 * (s->n_frag + n);
        s->frag = (int64_t *)realloc(s->frag, sizeof(int64_t) * 3 * s->frag_cap);
    }
    memcpy(s->frag + 3 * s->n_frag, v, sizeof(int64_t) * 3 * n);
    s->n_frag += n;
}

/* Voxels next to fragile walk steps of all raycast frames so far (with
 * repeats), up to cap triples; returns the count. */
int64_t orc_fragile_voxels(const orc_submap *s, int64_t *out, int64_t cap)
{
    if (out) memcpy(out, s->frag, sizeof(int64_t) * 3 * (s->n_frag < cap ? s->n_frag : cap));
    return s->n_frag;
}

typedef struct { uint64_t bkey; int64_t lin, pix; double t, w; } ray_contrib;

static int cmp_contrib(const void *a, const void *b)
{
    const ray_contrib *x = (const ray_contrib *)a, *y = (const ray_contrib *)b;
    if (x->bkey != y->bkey) return x->bkey < y->bkey ? -1 : 1;
    if (x->lin != y->lin) return x->lin < y->lin ? -1 : 1;
    return x->pix < y->pix ? -1 : (x->pix > y->pix ? 1 : 0);
}

/*
 * Raycast integration of one depth frame (Sec. III-C: a ray from the optical
 * centre through every observed point updates the voxels it crosses up to the
 * truncation distance behind the point; Sec. III-D: count and allocate the
 * new blocks, then merge all of the frame's contributions per voxel, the
 * weight and distance update being commutative, with the voxels in address
 * order).
 *   ray of pixel (col, row) with valid depth z (0 < z <= max_range):
 *     q = ((col - cx) z / fx, (row - cy) z / fy, z) in the camera frame,
 *     d = R_sc q, r = |d|, u = d / r, origin o = t_sc (submap frame);
 *   segment s in [s0, r + tau], s0 = 0 with ray_carve (from the optical
 *     centre), else max(0, r - tau);
 *   each crossed voxel (the walk above; its fragile steps are recorded for
 *     orc_fragile_voxels) with centre c: sdf = r - (c - o).u;
 *     it contributes t = min(sdf, tau) with the weight w (1, or 1/z^2) when
 *     sdf >= -tau;
 *   blocks holding a contribution are touched; new ones get buffer indices
 *     n + rank in ascending key order;
 *   per voxel, over its contributions in pixel (raster) order:
 *     sw = sum w, stw = sum t w, both in binary64 (the products of binary32
 *     t and w are exact there); then in binary32 W' = W + sw,
 *     D' = (D W + stw) / W' (sw and stw rounded once).
 * stats (nullable): [n_new, n_touched, n_contributions, n_voxels_updated].
 */
int orc_integrate_raycast(orc_submap *s, const float *depth, int H, int W, const float K[4],
                          const double *T_wc, int64_t *stats)
{
    double inv_ws[16], T_sc[16];
    rigid_inverse(s->T_ws, inv_ws);
    rigid_mul(inv_ws, T_wc, T_sc);
    float R32[9], o32[3];
    double R64[9], o64[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) { R32[3 * r + c] = (float)T_sc[4 * r + c]; R64[3 * r + c] = T_sc[4 * r + c]; }
        o32[r] = (float)T_sc[4 * r + 3];
        o64[r] = T_sc[4 * r + 3];
    }
    const double tau = s->p.trunc_vox * s->p.vs;
    const float vs_f = (float)s->p.vs, tau_f = (float)tau, maxr_f = (float)s->p.max_range;

    size_t nc = 0, capc = 1 << 16;
    ray_contrib *L = (ray_contrib *)malloc(sizeof(ray_contrib) * capc);
    int64_t walk_cap = 0, *walk = NULL;
    int64_t fcap = 0, *fbuf = NULL, nf = 0;
    for (int row = 0; row < H; ++row)
        for (int col = 0; col < W; ++col) {
            const float z = depth[(size_t)row * W + col];
            if (!(z > 0.0f && z <= maxr_f)) continue;
            const int64_t pix = (int64_t)row * W + col;
            int64_t nvox, guard;
            double r, u[3], o[3], w;
            if (!s->p.fp64) {
                const float xc = (((float)col - K[2]) * z) / K[0];
                const float yc = (((float)row - K[3]) * z) / K[1];
                float d[3], uf[3];
                for (int k = 0; k < 3; ++k) d[k] = (R32[3 * k] * xc + R32[3 * k + 1] * yc) + R32[3 * k + 2] * z;
                const float rf = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                for (int k = 0; k < 3; ++k) uf[k] = d[k] / rf;
                const float s1 = rf + tau_f;
                const float s0 = s->p.ray_carve ? 0.0f : fmaxf(rf - tau_f, 0.0f);
                guard = 3 * (int64_t)ceilf((s1 - s0) / vs_f) + 6;
                if (guard > walk_cap) {
                    walk_cap = guard;
                    walk = (int64_t *)realloc(walk, sizeof(int64_t) * 3 * walk_cap);
                    fcap = 7 * walk_cap;
                    fbuf = (int64_t *)realloc(fbuf, sizeof(int64_t) * 3 * fcap);
                }
                nf = 0;
                nvox = ray_walk32_frag(o32, uf, s0, s1, vs_f, walk, guard, fbuf, fcap, &nf);
                frag_append(s, fbuf, nf < fcap ? nf : fcap);
                const float wf = s->p.weight_mode ? 1.0f / (z * z) : 1.0f;
                for (int64_t k = 0; k < nvox; ++k) {
                    float c[3];
                    for (int a = 0; a < 3; ++a) c[a] = ((float)walk[3 * k + a] + 0.5f) * vs_f;
                    const float proj = ((c[0] - o32[0]) * uf[0] + (c[1] - o32[1]) * uf[1]) + (c[2] - o32[2]) * uf[2];
                    const float sdf = rf - proj;
                    if (!(sdf >= -tau_f)) continue;
                    if (nc == capc) { capc *= 2; L = (ray_contrib *)realloc(L, sizeof(ray_contrib) * capc); }
                    const int64_t *v = walk + 3 * k;
                    L[nc].bkey = pack_key(floordiv8(v[0]), floordiv8(v[1]), floordiv8(v[2]));
                    L[nc].lin = lin_index(v[0], v[1], v[2]);
                    L[nc].pix = pix;
                    L[nc].t = fminf(sdf, tau_f);
                    L[nc].w = wf;
                    ++nc;
                }
            } else {
                const double zd = z;
                const double xc = (((double)col - K[2]) * zd) / K[0];
                const double yc = (((double)row - K[3]) * zd) / K[1];
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = (R64[3 * k] * xc + R64[3 * k + 1] * yc) + R64[3 * k + 2] * zd;
                r = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
                for (int k = 0; k < 3; ++k) { u[k] = d[k] / r; o[k] = o64[k]; }
                const double s1 = r + tau;
                const double s0 = s->p.ray_carve ? 0.0 : fmax(r - tau, 0.0);
                guard = 3 * (int64_t)ceil((s1 - s0) / s->p.vs) + 6;
                if (guard > walk_cap) {
                    walk_cap = guard;
                    walk = (int64_t *)realloc(walk, sizeof(int64_t) * 3 * walk_cap);
                    fcap = 7 * walk_cap;
                    fbuf = (int64_t *)realloc(fbuf, sizeof(int64_t) * 3 * fcap);
                }
                nf = 0;
                nvox = ray_walk64(o, u, s0, s1, s->p.vs, walk, guard, fbuf, fcap, &nf);
                frag_append(s, fbuf, nf < fcap ? nf : fcap);
                w = s->p.weight_mode ? 1.0 / (zd * zd) : 1.0;
                for (int64_t k = 0; k < nvox; ++k) {
                    double c[3];
                    for (int a = 0; a < 3; ++a) c[a] = ((double)walk[3 * k + a] + 0.5) * s->p.vs;
                    const double proj = ((c[0] - o[0]) * u[0] + (c[1] - o[1]) * u[1]) + (c[2] - o[2]) * u[2];
                    const double sdf = r - proj;
                    if (!(sdf >= -tau)) continue;
                    if (nc == capc) { capc *= 2; L = (ray_contrib *)realloc(L, sizeof(ray_contrib) * capc); }
                    const int64_t *v = walk + 3 * k;
                    L[nc].bkey = pack_key(floordiv8(v[0]), floordiv8(v[1]), floordiv8(v[2]));
                    L[nc].lin = lin_index(v[0], v[1], v[2]);
                    L[nc].pix = pix;
                    L[nc].t = sdf < tau ? sdf : tau;
                    L[nc].w = w;
                    ++nc;
                }
            }
        }
    free(walk);
    free(fbuf);

    /* count and allocate */
    uint64_t *tk = (uint64_t *)malloc(sizeof(uint64_t) * (nc ? nc : 1));
    for (size_t j = 0; j < nc; ++j) tk[j] = L[j].bkey;
    size_t nt = 0;
    const int64_t n_new = allocate_touched(s, tk, nc, &nt);
    free(tk);

    /* merge per voxel: contributions sorted by (voxel, pixel) */
    qsort(L, nc, sizeof(ray_contrib), cmp_contrib);
    int64_t n_vox = 0;
    for (size_t j = 0; j < nc;) {
        size_t e = j;
        while (e < nc && L[e].bkey == L[j].bkey && L[e].lin == L[j].lin) ++e;
        const size_t o = (size_t)512 * find_block(s, L[j].bkey) + (size_t)L[j].lin;
        if (s->p.fp64) {
            double sw = 0.0, stw = 0.0;
            for (size_t k = j; k < e; ++k) { sw = sw + L[k].w; stw = stw + L[k].t * L[k].w; }
            const double Wn = s->W64[o] + sw;
            s->D64[o] = ((s->D64[o] * s->W64[o]) + stw) / Wn;
            s->W64[o] = Wn;
        } else {
            /* t and w are binary32 values; their products are exact in
             * binary64, and the sums are kept in binary64 */
            double sw = 0.0, stw = 0.0;
            for (size_t k = j; k < e; ++k) { sw = sw + L[k].w; stw = stw + L[k].t * L[k].w; }
            const float Wold = s->W[o], Dold = s->D[o];
            const float Wn = Wold + (float)sw;
            const float Dn = ((Dold * Wold) + (float)stw) / Wn;
            s->D[o] = round_store(s, Dn);
            s->W[o] = round_store(s, Wn);
        }
        ++n_vox;
        j = e;
    }
    free(L);
    if (stats) { stats[0] = n_new; stats[1] = (int64_t)nt; stats[2] = (int64_t)nc; stats[3] = n_vox; }
    return ORC_OK;
}

/* --------------------------------------------------------------- ESDF */

/* 1-D squared distance transform of f (INF = no site) by the lower envelope
 * of parabolas (Felzenszwalb and Huttenlocher).  Exact on integers: the
 * breakpoints are compared as correctly rounded quotients of integers. */
#define EDT_INF ((int64_t)1 << 50)

static void edt1d(const int64_t *f, int64_t *d, int n, int *v, double *z)
{
    int k = -1; /* index of the rightmost parabola of the envelope */
    for (int q = 0; q < n; ++q) {
        if (f[q] >= EDT_INF) continue;
        if (k < 0) { k = 0; v[0] = q; z[0] = -INFINITY; z[1] = INFINITY; continue; }
        double s;
        for (;;) {
            int p = v[k];
            s = (double)((f[q] + (int64_t)q * q) - (f[p] + (int64_t)p * p)) / (double)(2 * q - 2 * p);
            if (s <= z[k]) { --k; continue; } /* z[0] = -inf ends the loop at k = 0 */
            break;
        }
        ++k;
        v[k] = q;
        z[k] = s;
        z[k + 1] = INFINITY;
    }
    if (k < 0) {
        for (int q = 0; q < n; ++q) d[q] = EDT_INF;
        return;
    }
    int j = 0;
    for (int q = 0; q < n; ++q) {
        while (z[j + 1] < (double)q) ++j;
        int64_t dq = (int64_t)(q - v[j]);
        d[q] = dq * dq + f[v[j]];
    }
}

/* The band: |D| below the truncation distance by more than tau / 1024.  A
 * voxel that was clamped in every observation holds D = tau up to the
 * rounding of the running average (and of binary16 storage); it carries no
 * distance information and must not count as in-band whatever the precision. */
static double band_limit(const orc_params *p) { return p->trunc_vox * p->vs * (1.0 - 1.0 / 1024.0); }

/* Voxel value helpers for either mode. */
static double Dval(const orc_submap *s, size_t o) { return s->p.fp64 ? s->D64[o] : (double)s->D[o]; }
static double Wval(const orc_submap *s, size_t o) { return s->p.fp64 ? s->W64[o] : (double)s->W[o]; }

/*
 * ESDF of the whole submap.
 *   Obs  = {W > 0};  Band = Obs and |D| < tau (1 - 2^-10);  Sites = Obs and
 *   |D| <= vs.
 *   Band voxels copy D.  Other observed voxels: k = min over sites of the
 *   squared voxel distance (exact EDT on the dense block box);
 *   phi = sign * min(d_max, vs * sqrt(k)) for k <= R^2 with R = round(d_max /
 *   vs), else sign * d_max; sign = +1 when D > 0.  Unobserved: NaN.
 */
int orc_esdf_wavefront(orc_submap *s, int64_t *stats);

int orc_update_esdf(orc_submap *s)
{
    if (s->p.esdf_mode == 1) return orc_esdf_wavefront(s, NULL);
    if (s->n == 0) return ORC_OK;
    const int fp64 = s->p.fp64;
    const double tau = band_limit(&s->p);
    const float vs_f = (float)s->p.vs, tau_f = (float)tau, dmax_f = (float)s->p.d_max;
    const int64_t Rv = llround(s->p.d_max / s->p.vs);
    const int64_t R2 = Rv * Rv;

    int64_t bmin[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, bmax[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int64_t j = 0; j < s->n; ++j) {
        int64_t b[3];
        unpack_key(s->keys[j], b);
        for (int a = 0; a < 3; ++a) {
            if (b[a] < bmin[a]) bmin[a] = b[a];
            if (b[a] > bmax[a]) bmax[a] = b[a];
        }
    }
    int64_t o0[3], dim[3];
    for (int a = 0; a < 3; ++a) { o0[a] = 8 * bmin[a]; dim[a] = 8 * (bmax[a] - bmin[a] + 1); }
    size_t N = (size_t)(dim[0] * dim[1] * dim[2]);
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * N);
    for (size_t q = 0; q < N; ++q) g[q] = EDT_INF;
#define GI(x, y, z) ((size_t)(((z) * dim[1] + (y)) * dim[0] + (x)))
    /* sites */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < s->n; ++j) {
        int64_t b[3];
        unpack_key(s->keys[j], b);
        for (int l = 0; l < 512; ++l) {
            size_t o = (size_t)512 * j + l;
            double Wv = Wval(s, o), Dv = Dval(s, o);
            int site = fp64 ? (Wv > 0 && fabs(Dv) <= s->p.vs)
                            : ((float)Wv > 0.0f && fabsf((float)Dv) <= vs_f);
            if (!site) continue;
            int64_t x = 8 * b[0] + (l & 7) - o0[0];
            int64_t y = 8 * b[1] + ((l >> 3) & 7) - o0[1];
            int64_t z = 8 * b[2] + (l >> 6) - o0[2];
            g[GI(x, y, z)] = 0;
        }
    }
    /* separable passes x, y, z (the lines of a pass are independent) */
    int64_t L = dim[0] > dim[1] ? dim[0] : dim[1];
    if (dim[2] > L) L = dim[2];
    for (int axis = 0; axis < 3; ++axis) {
        int64_t n = dim[axis];
        int64_t a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
#pragma omp parallel
        {
            int64_t *fin = (int64_t *)malloc(sizeof(int64_t) * L), *fout = (int64_t *)malloc(sizeof(int64_t) * L);
            int *v = (int *)malloc(sizeof(int) * (L + 1));
            double *zz = (double *)malloc(sizeof(double) * (L + 2));
#pragma omp for schedule(static)
            for (int64_t u = 0; u < dim[a1]; ++u)
                for (int64_t w = 0; w < dim[a2]; ++w) {
                    for (int64_t q = 0; q < n; ++q) {
                        int64_t c[3];
                        c[axis] = q; c[a1] = u; c[a2] = w;
                        fin[q] = g[GI(c[0], c[1], c[2])];
                    }
                    edt1d(fin, fout, (int)n, v, zz);
                    for (int64_t q = 0; q < n; ++q) {
                        int64_t c[3];
                        c[axis] = q; c[a1] = u; c[a2] = w;
                        g[GI(c[0], c[1], c[2])] = fout[q] >= EDT_INF ? EDT_INF : fout[q];
                    }
                }
            free(fin); free(fout); free(v); free(zz);
        }
    }
    /* values */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < s->n; ++j) {
        int64_t b[3];
        unpack_key(s->keys[j], b);
        for (int l = 0; l < 512; ++l) {
            size_t o = (size_t)512 * j + l;
            int64_t x = 8 * b[0] + (l & 7) - o0[0];
            int64_t y = 8 * b[1] + ((l >> 3) & 7) - o0[1];
            int64_t z = 8 * b[2] + (l >> 6) - o0[2];
            int64_t k = g[GI(x, y, z)];
            s->ksq[o] = -1;
            if (fp64) {
                double Wv = s->W64[o], Dv = s->D64[o];
                if (!(Wv > 0)) { s->phi64[o] = NAN; continue; }
                if (fabs(Dv) < tau) { s->phi64[o] = Dv; continue; }
                double sg = Dv > 0 ? 1.0 : -1.0;
                if (k > R2) { s->ksq[o] = (int32_t)(R2 + 1); s->phi64[o] = sg * s->p.d_max; continue; }
                s->ksq[o] = (int32_t)k;
                double r = s->p.vs * sqrt((double)k);
                s->phi64[o] = sg * (r < s->p.d_max ? r : s->p.d_max);
            } else {
                float Wv = s->W[o], Dv = s->D[o];
                if (!(Wv > 0.0f)) { s->phi[o] = NAN; continue; }
                if (fabsf(Dv) < tau_f) { s->phi[o] = Dv; continue; }
                float sg = Dv > 0.0f ? 1.0f : -1.0f;
                if (k > R2) { s->ksq[o] = (int32_t)(R2 + 1); s->phi[o] = sg * dmax_f; continue; }
                s->ksq[o] = (int32_t)k;
                float r = vs_f * sqrtf((float)k);
                s->phi[o] = sg * fminf(dmax_f, r);
            }
        }
    }
#undef GI
    free(g);
    return ORC_OK;
}

/* ----------------------------------------------------- ESDF wavefront */

#define WF_INF INT32_MAX
#define WF_NONE (-1)

static int32_t wf_pack(int dx, int dy, int dz) { return (dx + 128) | ((dy + 128) << 8) | ((dz + 128) << 16); }

static void wf_unpack(int32_t p, int d[3])
{
    d[0] = (p & 255) - 128;
    d[1] = ((p >> 8) & 255) - 128;
    d[2] = ((p >> 16) & 255) - 128;
}

/* Voxel v takes the parent site of its face neighbour u (parent offset pu,
 * e = u - v) when that site is nearer than its own and within R. */
static int wf_offer(int32_t *kv, int32_t *pv, int32_t ku, int32_t pu, const int e[3], int64_t R2)
{
    if (ku == WF_INF) return 0;
    int d[3];
    wf_unpack(pu, d);
    const int o[3] = {d[0] + e[0], d[1] + e[1], d[2] + e[2]};
    const int64_t k = (int64_t)o[0] * o[0] + (int64_t)o[1] * o[1] + (int64_t)o[2] * o[2];
    if (k > R2 || k >= *kv) return 0;
    *kv = (int32_t)k;
    *pv = wf_pack(o[0], o[1], o[2]);
    return 1;
}

/* Buffer index of the block next to block j in direction dir (0 -x, 1 +x,
 * 2 -y, 3 +y, 4 -z, 5 +z), or -1. */
static int64_t wf_neighbour(const orc_submap *s, int64_t j, int dir)
{
    int64_t b[3];
    unpack_key(s->keys[j], b);
    b[dir >> 1] += (dir & 1) ? 1 : -1;
    return find_block(s, pack_key(b[0], b[1], b[2]));
}

static int site_of(const orc_submap *s, size_t o)
{
    if (s->p.fp64) return s->W64[o] > 0 && fabs(s->D64[o]) <= s->p.vs;
    return s->W[o] > 0.0f && fabsf(s->D[o]) <= (float)s->p.vs;
}

/*
 * Incremental ESDF (Sec. III-E).  Every voxel of an allocated block keeps
 * its nearest known site (parent, as an offset) and the squared distance k
 * to it in voxels^2 (k <= R^2, else none), R = round(d_max / vs).
 *   1. sites: observed voxels with |D| <= vs (as for the exact EDT);
 *   2. seeds: voxels of new blocks start with no parent; a site takes
 *      itself (k = 0); a voxel whose parent is no longer a site loses it
 *      (raise); every block with such a change is queued;
 *   3. rounds, until the queue is empty; each queued block, from the state
 *      of the previous round: its face voxels take the parents of the
 *      neighbouring blocks' face voxels when nearer (faces -x, +x, -y, +y,
 *      -z, +z in turn), then each axis x, y, z is swept forward and
 *      backward, every voxel taking its predecessor's parent when nearer;
 *      a block that changed queues itself and its six neighbours;
 *   4. phi of every observed voxel as for the exact EDT, with k from 3.
 * stats (nullable): [rounds, block-rounds processed, blocks queued first].
 */
int orc_esdf_wavefront(orc_submap *s, int64_t *stats)
{
    const int64_t n = s->n, n0 = s->wn;
    const int64_t Rv = llround(s->p.d_max / s->p.vs), R2 = Rv * Rv;
    uint8_t *site = (uint8_t *)malloc((size_t)512 * (n ? n : 1));
    uint8_t *q = (uint8_t *)calloc((size_t)(n ? n : 1), 1);
    for (int64_t j = 0; j < n; ++j)
        for (int l = 0; l < 512; ++l) site[512 * j + l] = (uint8_t)site_of(s, (size_t)512 * j + l);
    int64_t n_dirty = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t b[3];
        unpack_key(s->keys[j], b);
        for (int l = 0; l < 512; ++l) {
            const size_t o = (size_t)512 * j + l;
            if (j >= n0) { s->wk[o] = WF_INF; s->wpar[o] = WF_NONE; q[j] = 1; }
            if (site[o]) {
                if (s->wk[o] != 0) { s->wk[o] = 0; s->wpar[o] = wf_pack(0, 0, 0); q[j] = 1; }
            } else if (s->wk[o] != WF_INF) {
                int d[3];
                wf_unpack(s->wpar[o], d);
                const int64_t v[3] = {8 * b[0] + (l & 7), 8 * b[1] + ((l >> 3) & 7), 8 * b[2] + (l >> 6)};
                const int64_t st[3] = {v[0] + d[0], v[1] + d[1], v[2] + d[2]};
                const int64_t sb = find_block(s, pack_key(floordiv8(st[0]), floordiv8(st[1]), floordiv8(st[2])));
                if (sb < 0 || !site[512 * sb + lin_index(st[0], st[1], st[2])]) {
                    s->wk[o] = WF_INF;
                    s->wpar[o] = WF_NONE;
                    q[j] = 1;
                }
            }
        }
        n_dirty += q[j];
    }
    int32_t *nk = (int32_t *)malloc(sizeof(int32_t) * 512 * (n ? n : 1));
    int32_t *np = (int32_t *)malloc(sizeof(int32_t) * 512 * (n ? n : 1));
    uint8_t *changed = (uint8_t *)malloc((size_t)(n ? n : 1));
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    int64_t rounds = 0, work = 0;
    for (;;) {
        int64_t m = 0;
        for (int64_t j = 0; j < n; ++j)
            if (q[j]) list[m++] = j;
        if (m == 0) break;
        for (int64_t t = 0; t < m; ++t) {
            const int64_t j = list[t];
            int32_t *K = nk + 512 * j, *P = np + 512 * j;
            memcpy(K, s->wk + 512 * j, sizeof(int32_t) * 512);
            memcpy(P, s->wpar + 512 * j, sizeof(int32_t) * 512);
            for (int dir = 0; dir < 6; ++dir) {
                const int64_t nb = wf_neighbour(s, j, dir);
                if (nb < 0) continue;
                const int a = dir >> 1, side = (dir & 1) ? 7 : 0;
                int e[3] = {0, 0, 0};
                e[a] = (dir & 1) ? 1 : -1;
                for (int u1 = 0; u1 < 8; ++u1)
                    for (int u2 = 0; u2 < 8; ++u2) {
                        int c[3], cn[3];
                        c[a] = side;
                        c[a == 0 ? 1 : 0] = u1;
                        c[a == 2 ? 1 : 2] = u2;
                        memcpy(cn, c, sizeof(c));
                        cn[a] = 7 - side;
                        const int lv = c[0] + 8 * c[1] + 64 * c[2], lu = cn[0] + 8 * cn[1] + 64 * cn[2];
                        wf_offer(&K[lv], &P[lv], s->wk[512 * nb + lu], s->wpar[512 * nb + lu], e, R2);
                    }
            }
            for (int a = 0; a < 3; ++a)
                for (int u1 = 0; u1 < 8; ++u1)
                    for (int u2 = 0; u2 < 8; ++u2) {
                        int c[3];
                        c[a == 0 ? 1 : 0] = u1;
                        c[a == 2 ? 1 : 2] = u2;
                        int e[3] = {0, 0, 0};
                        e[a] = -1;
                        for (int x = 1; x < 8; ++x) {  /* forward: from x - 1 */
                            c[a] = x;
                            const int lv = c[0] + 8 * c[1] + 64 * c[2];
                            c[a] = x - 1;
                            const int lu = c[0] + 8 * c[1] + 64 * c[2];
                            wf_offer(&K[lv], &P[lv], K[lu], P[lu], e, R2);
                        }
                        e[a] = 1;
                        for (int x = 6; x >= 0; --x) {  /* backward: from x + 1 */
                            c[a] = x;
                            const int lv = c[0] + 8 * c[1] + 64 * c[2];
                            c[a] = x + 1;
                            const int lu = c[0] + 8 * c[1] + 64 * c[2];
                            wf_offer(&K[lv], &P[lv], K[lu], P[lu], e, R2);
                        }
                    }
            changed[j] = memcmp(K, s->wk + 512 * j, sizeof(int32_t) * 512) != 0 ||
                         memcmp(P, s->wpar + 512 * j, sizeof(int32_t) * 512) != 0;
        }
        memset(q, 0, (size_t)n);
        for (int64_t t = 0; t < m; ++t) {
            const int64_t j = list[t];
            memcpy(s->wk + 512 * j, nk + 512 * j, sizeof(int32_t) * 512);
            memcpy(s->wpar + 512 * j, np + 512 * j, sizeof(int32_t) * 512);
        }
        for (int64_t t = 0; t < m; ++t) {
            const int64_t j = list[t];
            if (!changed[j]) continue;
            q[j] = 1;
            for (int dir = 0; dir < 6; ++dir) {
                const int64_t nb = wf_neighbour(s, j, dir);
                if (nb >= 0) q[nb] = 1;
            }
        }
        ++rounds;
        work += m;
    }
    /* phi as for the exact EDT */
    const double tau = band_limit(&s->p);
    const float vs_f = (float)s->p.vs, tau_f = (float)tau, dmax_f = (float)s->p.d_max;
    for (int64_t j = 0; j < n; ++j)
        for (int l = 0; l < 512; ++l) {
            const size_t o = (size_t)512 * j + l;
            const int64_t k = s->wk[o] == WF_INF ? R2 + 1 : s->wk[o];
            s->ksq[o] = -1;
            if (s->p.fp64) {
                double Wv = s->W64[o], Dv = s->D64[o];
                if (!(Wv > 0)) { s->phi64[o] = NAN; continue; }
                if (fabs(Dv) < tau) { s->phi64[o] = Dv; continue; }
                double sg = Dv > 0 ? 1.0 : -1.0;
                s->ksq[o] = (int32_t)k;
                if (k > R2) { s->phi64[o] = sg * s->p.d_max; continue; }
                double r = s->p.vs * sqrt((double)k);
                s->phi64[o] = sg * (r < s->p.d_max ? r : s->p.d_max);
            } else {
                float Wv = s->W[o], Dv = s->D[o];
                if (!(Wv > 0.0f)) { s->phi[o] = NAN; continue; }
                if (fabsf(Dv) < tau_f) { s->phi[o] = Dv; continue; }
                float sg = Dv > 0.0f ? 1.0f : -1.0f;
                s->ksq[o] = (int32_t)k;
                if (k > R2) { s->phi[o] = sg * dmax_f; continue; }
                float r = vs_f * sqrtf((float)k);
                s->phi[o] = sg * fminf(dmax_f, r);
            }
        }
    memcpy(s->wsite, site, (size_t)512 * n);
    s->wn = n;
    if (stats) { stats[0] = rounds; stats[1] = work; stats[2] = n_dirty; }
    free(site); free(q); free(nk); free(np); free(changed); free(list);
    return ORC_OK;
}

/* ------------------------------------------------------------ export */

void orc_export(const orc_submap *s, uint64_t *keys, double *D, double *W, double *phi, int32_t *ksq)
{
    for (int64_t j = 0; j < s->n; ++j) {
        if (keys) keys[j] = s->keys[j];
        for (int l = 0; l < 512; ++l) {
            size_t o = (size_t)512 * j + l;
            if (D) D[o] = Dval(s, o);
            if (W) W[o] = Wval(s, o);
            if (phi) phi[o] = s->p.fp64 ? s->phi64[o] : (double)s->phi[o];
            if (ksq) ksq[o] = s->ksq[o];
        }
    }
}

/* Overwrite the voxel state (used by tests that build fields directly). */
int orc_import(orc_submap *s, int64_t n, const uint64_t *keys, const double *D, const double *W)
{
    s->n = 0;
    grow(s, n);
    for (int64_t j = 0; j < n; ++j) {
        s->keys[j] = keys[j];
        for (int l = 0; l < 512; ++l) {
            size_t o = (size_t)512 * j + l;
            if (s->p.fp64) { s->D64[o] = D[o]; s->W64[o] = W[o]; s->phi64[o] = NAN; }
            else { s->D[o] = round_store(s, (float)D[o]); s->W[o] = round_store(s, (float)W[o]); s->phi[o] = NAN; }
            s->ksq[o] = -1;
        }
    }
    s->n = n;
    s->wn = 0;  /* the wavefront state starts over */
    rebuild_sorted(s);
    return ORC_OK;
}

/* ------------------------------------------------- registration points */

/*
 * Registration points of a submap (Sec. III-F: points chosen by weight):
 * zero crossings of D along voxel edges (i, i + e_a) whose two endpoints are
 * both in the band (|D| < tau (1 - 2^-10)) and both have W >= w_reg.  p = c(i) with
 * p_a = c_a(i) + s vs,  s = D(i) / (D(i) - D(i + e_a)).
 * Order: (block buffer index, in-block index l, axis a).
 * out: 3 floats per point (binary32 mode) or 3 doubles (binary64 mode).
 * Returns the number of points (written up to cap).
 */
int64_t orc_iso_points(const orc_submap *s, void *out, int64_t cap)
{
    const double tau = band_limit(&s->p);
    const float vs_f = (float)s->p.vs, tau_f = (float)tau, wreg_f = (float)s->p.w_reg;
    int64_t n = 0;
    for (int64_t j = 0; j < s->n; ++j) {
        int64_t b[3];
        unpack_key(s->keys[j], b);
        for (int l = 0; l < 512; ++l) {
            int64_t i[3] = {8 * b[0] + (l & 7), 8 * b[1] + ((l >> 3) & 7), 8 * b[2] + (l >> 6)};
            size_t o = (size_t)512 * j + l;
            for (int a = 0; a < 3; ++a) {
                int64_t nb[3] = {i[0], i[1], i[2]};
                nb[a] += 1;
                int64_t jn = find_block(s, pack_key(floordiv8(nb[0]), floordiv8(nb[1]), floordiv8(nb[2])));
                if (jn < 0) continue;
                size_t on = (size_t)512 * jn + lin_index(nb[0], nb[1], nb[2]);
                if (s->p.fp64) {
                    double Wi = s->W64[o], Wn = s->W64[on], Di = s->D64[o], Dn = s->D64[on];
                    if (!(Wi >= s->p.w_reg && Wn >= s->p.w_reg)) continue;
                    if (!(fabs(Di) < tau && fabs(Dn) < tau)) continue;
                    if ((Di < 0) == (Dn < 0)) continue;
                    if (n < cap) {
                        double *p = (double *)out + 3 * n;
                        double sfr = Di / (Di - Dn);
                        for (int c = 0; c < 3; ++c) p[c] = ((double)i[c] + 0.5) * s->p.vs;
                        p[a] = p[a] + sfr * s->p.vs;
                    }
                } else {
                    float Wi = s->W[o], Wn = s->W[on], Di = s->D[o], Dn = s->D[on];
                    if (!(Wi >= wreg_f && Wn >= wreg_f)) continue;
                    if (!(fabsf(Di) < tau_f && fabsf(Dn) < tau_f)) continue;
                    if ((Di < 0.0f) == (Dn < 0.0f)) continue;
                    if (n < cap) {
                        float *p = (float *)out + 3 * n;
                        float sfr = Di / (Di - Dn);
                        for (int c = 0; c < 3; ++c) p[c] = ((float)i[c] + 0.5f) * vs_f;
                        p[a] = p[a] + sfr * vs_f;
                    }
                }
                ++n;
            }
        }
    }
    return n;
}

/* ------------------------------------------------ residual and NE */

/* phi of submap A at voxel index j, NaN when unallocated. */
static double phi_at(const orc_submap *A, const int64_t j[3])
{
    int64_t idx = find_block(A, pack_key(floordiv8(j[0]), floordiv8(j[1]), floordiv8(j[2])));
    if (idx < 0) return NAN;
    size_t o = (size_t)512 * idx + lin_index(j[0], j[1], j[2]);
    return A->p.fp64 ? A->phi64[o] : (double)A->phi[o];
}

/* phi of voxel (x, y, z) of submap s, NaN when unallocated (for the
 * summary oracle). */
double orc_phi_at_voxel(const orc_submap *s, int64_t x, int64_t y, int64_t z)
{
    int64_t j[3] = {x, y, z};
    return phi_at(s, j);
}

/*
 * Residual r = phi_A(T p) by trilinear interpolation, gradient g of the
 * interpolant, Jacobian J = [g ; q x g] for the left perturbation
 * T <- Exp(xi) T with xi = (rho, theta).  Points whose eight cell corners
 * are not all observed are skipped.  Sums over the points (binary64):
 *   out[0..20]  H = sum J J^T, upper triangle row by row
 *   out[21..26] b = sum J r
 *   out[27]     c = sum r^2
 *   out[28]     n = number of points used
 * Binary32 mode: per-point arithmetic in binary32 (T rounded to binary32),
 * products and sums in binary64.
 */
void orc_normal_eq(const orc_submap *A, const void *pts, int64_t n_pts, const double *T, double out[29])
{
    memset(out, 0, sizeof(double) * 29);
    const int fp64 = A->p.fp64;
    const float vs_f = (float)A->p.vs;
    float R32[9], t32[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) R32[3 * r + c] = (float)T[4 * r + c];
        t32[r] = (float)T[4 * r + 3];
    }
    for (int64_t k = 0; k < n_pts; ++k) {
        double Jd[6], rd;
        int64_t j0[3];
        double cor[8];
        if (fp64) {
            const double *p = (const double *)pts + 3 * k;
            double q[3], g[3], f[3];
            for (int a = 0; a < 3; ++a)
                q[a] = ((T[4 * a + 0] * p[0] + T[4 * a + 1] * p[1]) + T[4 * a + 2] * p[2]) + T[4 * a + 3];
            for (int a = 0; a < 3; ++a) {
                g[a] = q[a] / A->p.vs - 0.5;
                double fl = floor(g[a]);
                j0[a] = (int64_t)fl;
                f[a] = g[a] - fl;
            }
            int ok = 1;
            for (int c = 0; c < 8 && ok; ++c) {
                int64_t jj[3] = {j0[0] + (c & 1), j0[1] + ((c >> 1) & 1), j0[2] + ((c >> 2) & 1)};
                cor[c] = phi_at(A, jj);
                if (isnan(cor[c])) ok = 0;
            }
            if (!ok) continue;
            double wx0 = 1.0 - f[0], wx1 = f[0], wy0 = 1.0 - f[1], wy1 = f[1], wz0 = 1.0 - f[2], wz1 = f[2];
            double c00 = cor[0] * wx0 + cor[1] * wx1, c10 = cor[2] * wx0 + cor[3] * wx1;
            double c01 = cor[4] * wx0 + cor[5] * wx1, c11 = cor[6] * wx0 + cor[7] * wx1;
            double c0 = c00 * wy0 + c10 * wy1, c1 = c01 * wy0 + c11 * wy1;
            rd = c0 * wz0 + c1 * wz1;
            double dx = ((cor[1] - cor[0]) * wy0 + (cor[3] - cor[2]) * wy1) * wz0 +
                        ((cor[5] - cor[4]) * wy0 + (cor[7] - cor[6]) * wy1) * wz1;
            double dy = (c10 - c00) * wz0 + (c11 - c01) * wz1;
            double dz = c1 - c0;
            double gr[3] = {dx / A->p.vs, dy / A->p.vs, dz / A->p.vs};
            Jd[0] = gr[0]; Jd[1] = gr[1]; Jd[2] = gr[2];
            Jd[3] = q[1] * gr[2] - q[2] * gr[1];
            Jd[4] = q[2] * gr[0] - q[0] * gr[2];
            Jd[5] = q[0] * gr[1] - q[1] * gr[0];
        } else {
            const float *p = (const float *)pts + 3 * k;
            float q[3], g[3], f[3];
            for (int a = 0; a < 3; ++a)
                q[a] = ((R32[3 * a + 0] * p[0] + R32[3 * a + 1] * p[1]) + R32[3 * a + 2] * p[2]) + t32[a];
            for (int a = 0; a < 3; ++a) {
                g[a] = (q[a] / vs_f) - 0.5f;
                float fl = floorf(g[a]);
                j0[a] = (int64_t)fl;
                f[a] = g[a] - fl;
            }
            int ok = 1;
            for (int c = 0; c < 8 && ok; ++c) {
                int64_t jj[3] = {j0[0] + (c & 1), j0[1] + ((c >> 1) & 1), j0[2] + ((c >> 2) & 1)};
                cor[c] = phi_at(A, jj);
                if (isnan(cor[c])) ok = 0;
            }
            if (!ok) continue;
            float cf[8];
            for (int c = 0; c < 8; ++c) cf[c] = (float)cor[c];
            float wx0 = 1.0f - f[0], wx1 = f[0], wy0 = 1.0f - f[1], wy1 = f[1], wz0 = 1.0f - f[2], wz1 = f[2];
            float c00 = cf[0] * wx0 + cf[1] * wx1, c10 = cf[2] * wx0 + cf[3] * wx1;
            float c01 = cf[4] * wx0 + cf[5] * wx1, c11 = cf[6] * wx0 + cf[7] * wx1;
            float c0 = c00 * wy0 + c10 * wy1, c1 = c01 * wy0 + c11 * wy1;
            float r = c0 * wz0 + c1 * wz1;
            float dx = ((cf[1] - cf[0]) * wy0 + (cf[3] - cf[2]) * wy1) * wz0 +
                       ((cf[5] - cf[4]) * wy0 + (cf[7] - cf[6]) * wy1) * wz1;
            float dy = (c10 - c00) * wz0 + (c11 - c01) * wz1;
            float dz = c1 - c0;
            float gr[3] = {dx / vs_f, dy / vs_f, dz / vs_f};
            float J[6];
            J[0] = gr[0]; J[1] = gr[1]; J[2] = gr[2];
            J[3] = q[1] * gr[2] - q[2] * gr[1];
            J[4] = q[2] * gr[0] - q[0] * gr[2];
            J[5] = q[0] * gr[1] - q[1] * gr[0];
            for (int a = 0; a < 6; ++a) Jd[a] = (double)J[a];
            rd = (double)r;
        }
        int m = 0;
        for (int a = 0; a < 6; ++a)
            for (int b2 = a; b2 < 6; ++b2) out[m++] += Jd[a] * Jd[b2];
        for (int a = 0; a < 6; ++a) out[21 + a] += Jd[a] * rd;
        out[27] += rd * rd;
        out[28] += 1.0;
    }
}

/* ------------------------------------------------------ SE(3), solve */

/* Exp of xi = (rho, theta) in se(3) as a 4x4 (Rodrigues rotation and the
 * left Jacobian V applied to rho). */
void orc_se3_exp(const double xi[6], double *E)
{
    const double *rho = xi, *w = xi + 3;
    double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        double sh = sin(0.5 * th);
        A = sin(th) / th;
        B = 2.0 * sh * sh / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            K2[3 * r + c] = K[3 * r + 0] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
    double Rm[9], V[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double I = r == c ? 1.0 : 0.0;
            Rm[3 * r + c] = I + A * K[3 * r + c] + B * K2[3 * r + c];
            V[3 * r + c] = I + B * K[3 * r + c] + C * K2[3 * r + c];
        }
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) E[4 * r + c] = Rm[3 * r + c];
        E[4 * r + 3] = V[3 * r + 0] * rho[0] + V[3 * r + 1] * rho[1] + V[3 * r + 2] * rho[2];
    }
    E[12] = 0; E[13] = 0; E[14] = 0; E[15] = 1;
}

/* Solve (H + mu diag(H)) x = -b for the 6x6 symmetric H (upper triangle
 * packed) by Cholesky; mu = 0 is the Gauss-Newton step.  Returns 0, or -1
 * when the matrix is not positive definite. */
int orc_solve6_damped(const double *ne, double mu, double x[6])
{
    double H[36], L[36];
    int m = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b) { H[6 * a + b] = ne[m]; H[6 * b + a] = ne[m]; ++m; }
    if (mu != 0.0)
        for (int j = 0; j < 6; ++j) H[6 * j + j] = H[6 * j + j] + mu * H[6 * j + j];
    memset(L, 0, sizeof(L));
    for (int j = 0; j < 6; ++j) {
        double s = H[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0)) return -1;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double t = H[6 * i + j];
            for (int k = 0; k < j; ++k) t -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = t / L[6 * j + j];
        }
    }
    double y[6];
    for (int i = 0; i < 6; ++i) {
        double t = -ne[21 + i];
        for (int k = 0; k < i; ++k) t -= L[6 * i + k] * y[k];
        y[i] = t / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 6; ++k) t -= L[6 * k + i] * x[k];
        x[i] = t / L[6 * i + i];
    }
    return 0;
}

int orc_solve6(const double *ne, double x[6]) { return orc_solve6_damped(ne, 0.0, x); }

/*
 * The 4-DoF step (translation and yaw, for submaps whose gravity direction
 * is known): the Jacobian is the 6-DoF one restricted to (rho_x, rho_y,
 * rho_z, theta_z), so its normal equations are rows and columns 0, 1, 2, 5 of
 * the 6-DoF ones.  Solved by the same Cholesky; d = (rho, 0, 0, theta_z).
 */
int orc_solve_xyz_yaw_damped(const double ne[29], double mu, double d[6])
{
    static const int sel[4] = {0, 1, 2, 5};
    double H[4][4], b[4];
    for (int a = 0; a < 4; ++a) {
        for (int c = 0; c < 4; ++c) {
            int r = sel[a], q = sel[c];
            if (r > q) { int t = r; r = q; q = t; }
            H[a][c] = ne[r * 6 - r * (r - 1) / 2 + (q - r)];
        }
        b[a] = ne[21 + sel[a]];
    }
    if (mu != 0.0)
        for (int a = 0; a < 4; ++a) H[a][a] = H[a][a] + mu * H[a][a];
    double L[4][4] = {{0}};
    for (int j = 0; j < 4; ++j) {
        double sj = H[j][j];
        for (int k = 0; k < j; ++k) sj -= L[j][k] * L[j][k];
        if (!(sj > 0.0)) return -1;
        L[j][j] = sqrt(sj);
        for (int i = j + 1; i < 4; ++i) {
            double t = H[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    double y[4], x[4];
    for (int i = 0; i < 4; ++i) {
        double t = -b[i];
        for (int k = 0; k < i; ++k) t -= L[i][k] * y[k];
        y[i] = t / L[i][i];
    }
    for (int i = 3; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < 4; ++k) t -= L[k][i] * x[k];
        x[i] = t / L[i][i];
    }
    d[0] = x[0]; d[1] = x[1]; d[2] = x[2];
    d[3] = 0.0; d[4] = 0.0; d[5] = x[3];
    return 0;
}

int orc_solve_xyz_yaw(const double ne[29], double d[6]) { return orc_solve_xyz_yaw_damped(ne, 0.0, d); }

/*
 * Levenberg-Marquardt alignment (Sec. III-F solves the backend's least
 * squares by LM with a trust region; here the same rule serves one pair).
 * At the current pose T with normal equations (H, b, c, n), cost c / n:
 *   solve (H + mu diag(H)) delta = -b (4-DoF: rows and columns 0, 1, 2, 5);
 *   if |delta_rho| < tol_rho and |delta_theta| < tol_theta: converged, the
 *     step is not taken;
 *   trial T' = Exp(delta) T with normal equations (H', b', c', n');
 *   predicted decrease of the mean cost L = -(2 delta.b + delta.H.delta) / n;
 *   gain ratio rho = (c / n - c' / n') / L when n' >= n_min and L > 0,
 *     else -1;
 *   rho > 0: T = T', mu *= max(1/3, 1 - (2 rho - 1)^3), nu = 2;
 *   otherwise mu *= nu, nu *= 2.
 * mu starts at 1e-4 (relative to diag(H), Marquardt's scaling), nu at 2
 * (the rule of Madsen, Nielsen and Tingleff, 2004).  max_iter caps the
 * solves; fewer than n_min residuals at the start is EDEGENERATE, as is a
 * damped matrix that is not positive definite.
 * Rounding-noise floor: a residual computed in a format of unit roundoff u
 * is off by at most about 16 u Q, Q the distance from A's origin of the
 * farthest corner of A's block box (every point with a residual lies in
 * it): the transform, the grid coordinate and the interpolation each add a
 * few roundings of quantities up to Q.  Independent errors add in
 * root-sum-square, so c = sum r^2 is uncertain by up to 2 * 16 u Q sqrt(c).
 * A step whose predicted decrease L n is within that is converged (not
 * taken): beyond it the gain ratio compares rounding noise.  u = 2^-24 for
 * binary32 residuals, 2^-53 for binary64.
 * info[0] = steps taken, info[1] = n at the returned T, info[2] = solves.
 */
static double lm_predicted(const double *ne, const double d[6])
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

static int align_lm(const orc_submap *A, const void *pts, int64_t n_pts, const double *T_init, double *T_out,
                    double *cost, int64_t *info)
{
    double T[16], Tt[16], ne[29], nt[29];
    memcpy(T, T_init, sizeof(T));
    int status = ORC_NOT_CONVERGED;
    int64_t taken = 0;
    orc_normal_eq(A, pts, n_pts, T, ne);
    if (A->p.max_iter > 0 && ne[28] < A->p.n_min) status = ORC_EDEGENERATE;
    double mu = 1e-4, nu = 2.0;
    /* Q from the block box of A (block edge 8 voxels) */
    int64_t bmin[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, bmax[3] = {INT64_MIN, INT64_MIN, INT64_MIN};
    for (int64_t j = 0; j < A->n; ++j) {
        int64_t b[3];
        unpack_key(A->keys[j], b);
        for (int a = 0; a < 3; ++a) {
            if (b[a] < bmin[a]) bmin[a] = b[a];
            if (b[a] > bmax[a]) bmax[a] = b[a];
        }
    }
    const double edge = 8.0 * (A->p.fp64 ? A->p.vs : (double)(float)A->p.vs);
    double q2 = 0.0;
    for (int a = 0; a < 3 && A->n > 0; ++a) {
        const double lo = fabs(edge * (double)bmin[a]), hi = fabs(edge * (double)(bmax[a] + 1));
        const double m = lo > hi ? lo : hi;
        q2 += m * m;
    }
    const double u = A->p.fp64 ? ldexp(1.0, -53) : ldexp(1.0, -24);
    const double noise = 2.0 * 16.0 * u * sqrt(q2);
    int64_t solves = 0;
    for (int it = 0; it < A->p.max_iter && status == ORC_NOT_CONVERGED; ++it) {
        double d[6];
        if ((A->p.align_dof == 4 ? orc_solve_xyz_yaw_damped(ne, mu, d) : orc_solve6_damped(ne, mu, d)) != 0) {
            status = ORC_EDEGENERATE;
            break;
        }
        ++solves;
        double nr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double nth = sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
        if (nr < A->p.tol_rho && nth < A->p.tol_theta) { status = ORC_OK; break; }
        if (lm_predicted(ne, d) <= noise * sqrt(ne[27])) { status = ORC_OK; break; }
        double E[16];
        orc_se3_exp(d, E);
        rigid_mul(E, T, Tt);
        orc_normal_eq(A, pts, n_pts, Tt, nt);
        const double pred = lm_predicted(ne, d);
        double rho = -1.0;
        if (nt[28] >= A->p.n_min && pred > 0.0) rho = (ne[27] / ne[28] - nt[27] / nt[28]) / (pred / ne[28]);
        if (rho > 0.0) {
            memcpy(T, Tt, sizeof(T));
            memcpy(ne, nt, sizeof(ne));
            ++taken;
            const double s = 2.0 * rho - 1.0, f = 1.0 - s * s * s;
            mu *= f > 1.0 / 3.0 ? f : 1.0 / 3.0;
            nu = 2.0;
        } else {
            mu *= nu;
            nu *= 2.0;
        }
    }
    *cost = ne[28] > 0 ? ne[27] / ne[28] : INFINITY;
    memcpy(T_out, T, sizeof(T));
    if (info) { info[0] = taken; info[1] = (int64_t)ne[28]; info[2] = solves; }
    return status;
}

/*
 * Gauss-Newton alignment of B's registration points to A's ESDF.
 * T maps B coordinates to A coordinates.  Each iteration: normal equations
 * at T; stop with EDEGENERATE when fewer than n_min residuals or H is not
 * positive definite; delta = -H^-1 b; T <- Exp(delta) T; stop when
 * |delta_rho| < 1e-7 m and |delta_theta| < 1e-8 rad (converged) or after
 * max_iter iterations.  cost = c / n at the returned T.
 * info[0] = pose updates applied, info[1] = n used at the returned T,
 * info[2] = solves (Gauss-Newton: = info[0]).
 */
int orc_align_points(const orc_submap *A, const void *pts, int64_t n_pts, const double *T_init,
                     double *T_out, double *cost, int64_t *info)
{
    if (A->p.align_solver == 1) return align_lm(A, pts, n_pts, T_init, T_out, cost, info);
    double T[16];
    memcpy(T, T_init, sizeof(T));
    int status = ORC_NOT_CONVERGED;
    int64_t n_upd = 0;
    double ne[29];
    for (int it = 0; it < A->p.max_iter; ++it) {
        orc_normal_eq(A, pts, n_pts, T, ne);
        if (ne[28] < A->p.n_min) { status = ORC_EDEGENERATE; break; }
        double d[6];
        if ((A->p.align_dof == 4 ? orc_solve_xyz_yaw(ne, d) : orc_solve6(ne, d)) != 0) {
            status = ORC_EDEGENERATE;
            break;
        }
        double E[16];
        orc_se3_exp(d, E);
        rigid_mul(E, T, T);
        ++n_upd;
        double nr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double nt = sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
        if (nr < A->p.tol_rho && nt < A->p.tol_theta) { status = ORC_OK; break; }
    }
    orc_normal_eq(A, pts, n_pts, T, ne);
    *cost = ne[28] > 0 ? ne[27] / ne[28] : INFINITY;
    memcpy(T_out, T, sizeof(T));
    if (info) { info[0] = n_upd; info[1] = (int64_t)ne[28]; info[2] = n_upd; }
    return status;
}

/*
 * Multi-start alignment: start k (0 <= k < n_starts) is
 *   T_k = T_init Trans(pbar) Rz(2 pi k / n_starts) Trans(-pbar)
 * with pbar the binary64 centroid of the points (summed in order).  The
 * answer is the start of least cost among those with n_k >= n_max / 2 and a
 * status other than EDEGENERATE; ties go to the smallest k.
 * starts_out (nullable): 16 doubles per start.  best_k: chosen start.
 */
int orc_align_multistart(const orc_submap *A, const void *pts, int64_t n_pts, const double *T_init,
                         int n_starts, double *T_out, double *cost, int64_t *info, int *best_k,
                         double *starts_out)
{
    double pbar[3] = {0, 0, 0};
    for (int64_t k = 0; k < n_pts; ++k)
        for (int a = 0; a < 3; ++a)
            pbar[a] += A->p.fp64 ? ((const double *)pts)[3 * k + a] : (double)((const float *)pts)[3 * k + a];
    for (int a = 0; a < 3; ++a) pbar[a] /= (double)(n_pts > 0 ? n_pts : 1);
    double *Ts = (double *)malloc(sizeof(double) * 16 * n_starts);
    double *cs = (double *)malloc(sizeof(double) * n_starts);
    int64_t *ns = (int64_t *)malloc(sizeof(int64_t) * n_starts);
    int64_t *its = (int64_t *)malloc(sizeof(int64_t) * n_starts);
    int64_t *sol = (int64_t *)malloc(sizeof(int64_t) * n_starts);
    int *st = (int *)malloc(sizeof(int) * n_starts);
    int64_t nmax = 0;
    for (int k = 0; k < n_starts; ++k) {
        double a = 2.0 * M_PI * (double)k / (double)n_starts;
        double P[16] = {1, 0, 0, pbar[0], 0, 1, 0, pbar[1], 0, 0, 1, pbar[2], 0, 0, 0, 1};
        double Pm[16] = {1, 0, 0, -pbar[0], 0, 1, 0, -pbar[1], 0, 0, 1, -pbar[2], 0, 0, 0, 1};
        double Rz[16] = {cos(a), -sin(a), 0, 0, sin(a), cos(a), 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
        double S[16];
        rigid_mul(T_init, P, S);
        rigid_mul(S, Rz, S);
        rigid_mul(S, Pm, S);
        if (starts_out) memcpy(starts_out + 16 * k, S, sizeof(S));
        int64_t inf[3];
        st[k] = orc_align_points(A, pts, n_pts, S, Ts + 16 * k, &cs[k], inf);
        its[k] = inf[0];
        ns[k] = inf[1];
        sol[k] = inf[2];
        if (st[k] != ORC_EDEGENERATE && ns[k] > nmax) nmax = ns[k];
    }
    int best = -1;
    for (int k = 0; k < n_starts; ++k) {
        if (st[k] == ORC_EDEGENERATE) continue;
        if (2 * ns[k] < nmax) continue;
        if (best < 0 || cs[k] < cs[best]) best = k;
    }
    int status = ORC_EDEGENERATE;
    if (best >= 0) {
        memcpy(T_out, Ts + 16 * best, sizeof(double) * 16);
        *cost = cs[best];
        if (info) { info[0] = its[best]; info[1] = ns[best]; info[2] = sol[best]; }
        status = st[best];
    } else {
        memcpy(T_out, T_init, sizeof(double) * 16);
        *cost = INFINITY;
        if (info) { info[0] = 0; info[1] = 0; info[2] = 0; }
    }
    if (best_k) *best_k = best;
    free(Ts); free(cs); free(ns); free(its); free(sol); free(st);
    return status;
}

/* ------------------------------------------------------------- hash table */

/*
 * Inserts keys[0..n) in this order into the open-addressing table
 * tkeys/tvals of `cap` slots (a power of two; empty = all ones): each key
 * goes to the first empty slot at or after its home slot mix64(key) &
 * (cap - 1), wrapping at the end; the slot's value becomes val_base + i
 * (modulo 2^32).  probe[i] (nullable) receives the number of slots passed
 * over.  stats[0] = max probe, stats[1] += probe sum, stats[2] += keys that
 * found no empty slot (the table was full).
 */
void orc_hash_insert(uint64_t *tkeys, uint32_t *tvals, int64_t cap, const uint64_t *keys, int64_t n,
                     uint32_t val_base, int64_t *probe, int64_t stats[3])
{
    const uint64_t EMPTY = ~(uint64_t)0;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t h = orc_mix64(keys[i]) & (uint64_t)(cap - 1);
        int64_t p = 0;
        while (p < cap && tkeys[h] != EMPTY) {
            h = (h + 1) & (uint64_t)(cap - 1);
            ++p;
        }
        if (p == cap) {
            stats[2] += 1;
            if (probe) probe[i] = -1;
            continue;
        }
        tkeys[h] = keys[i];
        tvals[h] = val_base + (uint32_t)i;
        if (probe) probe[i] = p;
        if (p > stats[0]) stats[0] = p;
        stats[1] += p;
    }
}
