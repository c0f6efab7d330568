/*
 * Seeded synthetic depth renderer (input generation only).
 *
 * This file produces the depth frames that both the oracle and
 * the GPU path consume.  It contains no part of the mapping method: only
 * ray/primitive intersection, a counter-based random number generator and
 * the sensor noise model of the synthetic workloads.
 *
 * Camera convention: pinhole, x right, y down, z forward.  Pixel (c, r) is
 * the ray through its centre with camera-frame direction
 * ((c - cx) / fx, (r - cy) / fy, 1), so the ray parameter of a hit equals
 * its depth z.  A depth of 0 means "no measurement".
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), keyed by the scene seed and
 * indexed by (frame, pixel).  Gaussian noise uses the Box-Muller transform.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC (plain host C).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox */

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* One Philox4x32 round on the counter with the given key. */
static inline void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(0xD2511F53u, c[0], &hi0, &lo0);
    mulhilo32(0xCD9E8D57u, c[2], &hi1, &lo1);
    uint32_t o0 = hi1 ^ c[1] ^ k[0];
    uint32_t o1 = lo1;
    uint32_t o2 = hi0 ^ c[3] ^ k[1];
    uint32_t o3 = lo0;
    c[0] = o0; c[1] = o1; c[2] = o2; c[3] = o3;
}

/* Philox4x32 with ten rounds; the key is bumped by the Weyl constants
 * between rounds. */
void sg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof(c));
}

/* Uniform in the open interval (0, 1) from 32 random bits. */
static inline double u01_open(uint32_t x)
{
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

/* Draw for one pixel: a standard normal variate (Box-Muller on words 0, 1)
 * and a uniform in (0, 1) (word 2) for the invalid-pixel Bernoulli test. */
static inline void pixel_draws(uint32_t seed, uint32_t frame, uint32_t pixel,
                               double *gauss, double *unif)
{
    const uint32_t key[2] = {seed, 0x636f7678u};
    const uint32_t ctr[4] = {pixel, frame, 0x64657074u, 0u};
    uint32_t o[4];
    sg_philox4x32_10(ctr, key, o);
    double u1 = u01_open(o[0]);
    double u2 = u01_open(o[1]);
    *gauss = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
    *unif = u01_open(o[2]);
}

void sg_pixel_draws(uint32_t seed, uint32_t frame, uint32_t pixel, double out[2])
{
    pixel_draws(seed, frame, pixel, &out[0], &out[1]);
}

/* ------------------------------------------------------------ primitives */

/* Ray o + s d, s > 0.  Returns the smallest hit parameter > eps or INFINITY. */

static double hit_room_interior(const double o[3], const double d[3], const double lo[3],
                                const double hi[3])
{
    /* From inside an axis-aligned box the ray leaves through the nearest
     * exit plane. */
    double s = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] > 0.0) {
            double t = (hi[a] - o[a]) / d[a];
            if (t < s) s = t;
        } else if (d[a] < 0.0) {
            double t = (lo[a] - o[a]) / d[a];
            if (t < s) s = t;
        }
    }
    return s > 1e-9 ? s : INFINITY;
}

static double hit_sphere(const double o[3], const double d[3], const double c[3], double r)
{
    double oc[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
    double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double b = oc[0] * d[0] + oc[1] * d[1] + oc[2] * d[2];
    double cc = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - r * r;
    double disc = b * b - a * cc;
    if (disc < 0.0) return INFINITY;
    double sq = sqrt(disc);
    double t0 = (-b - sq) / a;
    if (t0 > 1e-9) return t0;
    double t1 = (-b + sq) / a;
    if (t1 > 1e-9) return t1;
    return INFINITY;
}

/* Solid axis-aligned box seen from outside (slab method). */
static double hit_box_solid(const double o[3], const double d[3], const double lo[3],
                            const double hi[3])
{
    double tmin = -INFINITY, tmax = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double t1 = (lo[a] - o[a]) / d[a];
            double t2 = (hi[a] - o[a]) / d[a];
            if (t1 > t2) { double tt = t1; t1 = t2; t2 = tt; }
            if (t1 > tmin) tmin = t1;
            if (t2 < tmax) tmax = t2;
        } else if (o[a] < lo[a] || o[a] > hi[a]) {
            return INFINITY;
        }
    }
    if (tmax < tmin) return INFINITY;
    if (tmin > 1e-9) return tmin;
    if (tmax > 1e-9) return tmax; /* origin inside the solid */
    return INFINITY;
}

/* Heightfield z = h(x, y): bilinear interpolation of a regular grid of
 * nx * ny samples with spacing `step` starting at (x0, y0).  Intersection by
 * marching with a step bounded by the height gap over the maximum slope,
 * followed by bisection to 1e-6 m. */
typedef struct {
    const double *h;
    int nx, ny;
    double x0, y0, step, slope;
} hfield_t;

static double hf_eval(const hfield_t *f, double x, double y)
{
    double gx = (x - f->x0) / f->step, gy = (y - f->y0) / f->step;
    if (gx < 0) gx = 0;
    if (gy < 0) gy = 0;
    if (gx > f->nx - 1) gx = f->nx - 1;
    if (gy > f->ny - 1) gy = f->ny - 1;
    int ix = (int)floor(gx), iy = (int)floor(gy);
    if (ix > f->nx - 2) ix = f->nx - 2;
    if (iy > f->ny - 2) iy = f->ny - 2;
    double fx = gx - ix, fy = gy - iy;
    const double *r0 = f->h + (size_t)iy * f->nx;
    const double *r1 = r0 + f->nx;
    double a = r0[ix] * (1 - fx) + r0[ix + 1] * fx;
    double b = r1[ix] * (1 - fx) + r1[ix + 1] * fx;
    return a * (1 - fy) + b * fy;
}

static double hit_hfield(const hfield_t *f, const double o[3], const double d[3], double smax)
{
    /* gap(s) = z(s) - h(x(s), y(s)); |d gap / ds| <= |dz| + slope * |dxy|. */
    double dxy = sqrt(d[0] * d[0] + d[1] * d[1]);
    double lip = fabs(d[2]) + f->slope * dxy + 1e-12;
    double s = 1e-6;
    double gap = o[2] + s * d[2] - hf_eval(f, o[0] + s * d[0], o[1] + s * d[1]);
    if (gap <= 0) return INFINITY; /* starting below the ground */
    while (s < smax) {
        double stepv = gap / lip;
        if (stepv < 1e-4) stepv = 1e-4;
        double s2 = s + stepv;
        double g2 = o[2] + s2 * d[2] - hf_eval(f, o[0] + s2 * d[0], o[1] + s2 * d[1]);
        if (g2 <= 0) {
            double a = s, b = s2;
            while (b - a > 1e-6) {
                double m = 0.5 * (a + b);
                double gm = o[2] + m * d[2] - hf_eval(f, o[0] + m * d[0], o[1] + m * d[1]);
                if (gm > 0) a = m; else b = m;
            }
            return 0.5 * (a + b);
        }
        s = s2;
        gap = g2;
    }
    return INFINITY;
}

/* ------------------------------------------------------------------ render */

/*
 * Render one depth frame.
 *   room[6]        interior box lo, hi (ignored when has_room == 0)
 *   sph[4 * n_sph] centre, radius
 *   box[6 * n_box] solid boxes lo, hi
 *   hf, hf_nx...   optional heightfield (hf == NULL: none)
 *   T_world_cam    4x4 row-major, maps camera coordinates to world
 *   noise_model    0: none, 1: sigma = noise_a, 2: sigma = noise_a * z^2
 *   invalid_frac   probability that a pixel is set to 0
 */
void sg_render(int has_room, const double *room, int n_sph, const double *sph, int n_box,
               const double *box, const double *hf, int hf_nx, int hf_ny, double hf_x0,
               double hf_y0, double hf_step, double hf_slope, int H, int W, double fx,
               double fy, double cx, double cy, const double *T, double max_range,
               int noise_model, double noise_a, double invalid_frac, uint32_t seed,
               uint32_t frame, float *out)
{
    hfield_t hfs = {hf, hf_nx, hf_ny, hf_x0, hf_y0, hf_step, hf_slope};
    const double o[3] = {T[3], T[7], T[11]};
#pragma omp parallel for schedule(static)
    for (int r = 0; r < H; ++r) {
        for (int c = 0; c < W; ++c) {
            double dc[3] = {((double)c - cx) / fx, ((double)r - cy) / fy, 1.0};
            double d[3];
            for (int k = 0; k < 3; ++k)
                d[k] = T[4 * k + 0] * dc[0] + T[4 * k + 1] * dc[1] + T[4 * k + 2] * dc[2];
            double s = INFINITY;
            if (has_room) {
                double t = hit_room_interior(o, d, room, room + 3);
                if (t < s) s = t;
            }
            for (int i = 0; i < n_sph; ++i) {
                double t = hit_sphere(o, d, sph + 4 * i, sph[4 * i + 3]);
                if (t < s) s = t;
            }
            for (int i = 0; i < n_box; ++i) {
                double t = hit_box_solid(o, d, box + 6 * i, box + 6 * i + 3);
                if (t < s) s = t;
            }
            if (hf) {
                double lim = s < max_range ? s : max_range;
                double t = hit_hfield(&hfs, o, d, lim);
                if (t < s) s = t;
            }
            double z = (s <= max_range) ? s : 0.0;
            uint32_t pix = (uint32_t)(r * W + c);
            if (z > 0.0 && (noise_model != 0 || invalid_frac > 0.0)) {
                double g, u;
                pixel_draws(seed, frame, pix, &g, &u);
                double sigma = noise_model == 1 ? noise_a
                             : noise_model == 2 ? noise_a * z * z : 0.0;
                z += sigma * g;
                if (z <= 0.0) z = 0.0;
                if (u < invalid_frac) z = 0.0;
            }
            out[(size_t)r * W + c] = (float)z;
        }
    }
}

/* Height of the heightfield at (x, y) (for scene construction and tests). */
double sg_hfield_eval(const double *hf, int nx, int ny, double x0, double y0, double step,
                      double x, double y)
{
    hfield_t f = {hf, nx, ny, x0, y0, step, 0.0};
    return hf_eval(&f, x, y);
}

/* ------------------------------------------------------------ outdoor scene
 *
 * Ground: bilinear heightfield on a regular grid (spacing hs, origin x0, y0,
 * nx * ny samples); a ray is walked cell by cell (2-D DDA) and intersected
 * exactly with each cell's bilinear patch (a quadratic in the ray
 * parameter).  Buildings: solid axis-aligned boxes listed in a coarse 2-D
 * grid (cell gs) that the ray also walks.  Everything in binary64.
 */

typedef struct {
    const double *h;
    int nx, ny;
    double x0, y0, hs;
} hgrid_t;

/* smallest root of a + b t + c t^2 = 0 in [t0, t1], or INFINITY */
static double quad_first_root(double a, double b, double c, double t0, double t1)
{
    double r[2];
    int n = 0;
    if (fabs(c) < 1e-14) {
        if (fabs(b) > 1e-300) r[n++] = -a / b;
    } else {
        double disc = b * b - 4 * a * c;
        if (disc >= 0) {
            double sq = sqrt(disc);
            double q = -0.5 * (b + (b >= 0 ? sq : -sq));
            double x1 = q / c;
            double x2 = q != 0 ? a / q : x1;
            r[n++] = x1 < x2 ? x1 : x2;
            r[n++] = x1 < x2 ? x2 : x1;
        }
    }
    for (int i = 0; i < n; ++i)
        if (r[i] >= t0 && r[i] <= t1) return r[i];
    return INFINITY;
}

static double hit_hgrid(const hgrid_t *g, const double o[3], const double d[3], double tmax)
{
    /* grid coordinates of the ray */
    double gx = (o[0] - g->x0) / g->hs, gy = (o[1] - g->y0) / g->hs;
    double dx = d[0] / g->hs, dy = d[1] / g->hs;
    int ix = (int)floor(gx), iy = (int)floor(gy);
    int sx = dx > 0 ? 1 : -1, sy = dy > 0 ? 1 : -1;
    double tdx = dx != 0 ? fabs(1.0 / dx) : INFINITY, tdy = dy != 0 ? fabs(1.0 / dy) : INFINITY;
    double tnx = dx != 0 ? ((dx > 0 ? (ix + 1 - gx) : (gx - ix)) * tdx) : INFINITY;
    double tny = dy != 0 ? ((dy > 0 ? (iy + 1 - gy) : (gy - iy)) * tdy) : INFINITY;
    double t0 = 0.0;
    while (t0 <= tmax) {
        double t1 = tnx < tny ? tnx : tny;
        if (t1 > tmax) t1 = tmax;
        if (ix >= 0 && iy >= 0 && ix < g->nx - 1 && iy < g->ny - 1) {
            const double *r0 = g->h + (size_t)iy * g->nx + ix;
            const double *r1 = r0 + g->nx;
            double A = r0[0], B = r0[1] - r0[0], C = r1[0] - r0[0], E = r0[0] - r0[1] - r1[0] + r1[1];
            double u0 = gx - ix, v0 = gy - iy;
            double a0 = o[2] - A - B * u0 - C * v0 - E * u0 * v0;
            double a1 = d[2] - B * dx - C * dy - E * (u0 * dy + v0 * dx);
            double a2 = -E * dx * dy;
            double t = quad_first_root(a0, a1, a2, t0, t1);
            if (t < INFINITY) return t;
        }
        if (t1 >= tmax) break;
        t0 = t1;
        if (tnx < tny) { ix += sx; tnx += tdx; } else { iy += sy; tny += tdy; }
    }
    return INFINITY;
}

typedef struct {
    const double *box;      /* 6 per box */
    const int32_t *start;   /* cell -> first entry in items (ncx * ncy + 1) */
    const int32_t *items;   /* box indices */
    int ncx, ncy;
    double x0, y0, gs;
} bgrid_t;

static double hit_bgrid(const bgrid_t *g, const double o[3], const double d[3], double tmax)
{
    double gx = (o[0] - g->x0) / g->gs, gy = (o[1] - g->y0) / g->gs;
    double dx = d[0] / g->gs, dy = d[1] / g->gs;
    int ix = (int)floor(gx), iy = (int)floor(gy);
    int sx = dx > 0 ? 1 : -1, sy = dy > 0 ? 1 : -1;
    double tdx = dx != 0 ? fabs(1.0 / dx) : INFINITY, tdy = dy != 0 ? fabs(1.0 / dy) : INFINITY;
    double tnx = dx != 0 ? ((dx > 0 ? (ix + 1 - gx) : (gx - ix)) * tdx) : INFINITY;
    double tny = dy != 0 ? ((dy > 0 ? (iy + 1 - gy) : (gy - iy)) * tdy) : INFINITY;
    double best = INFINITY, t0 = 0.0;
    while (t0 <= tmax && t0 < best) {
        double t1 = tnx < tny ? tnx : tny;
        if (ix >= 0 && iy >= 0 && ix < g->ncx && iy < g->ncy) {
            int c = iy * g->ncx + ix;
            for (int k = g->start[c]; k < g->start[c + 1]; ++k) {
                double t = hit_box_solid(o, d, g->box + 6 * g->items[k], g->box + 6 * g->items[k] + 3);
                if (t < best) best = t;
            }
        }
        if (t1 > tmax) break;
        t0 = t1;
        if (tnx < tny) { ix += sx; tnx += tdx; } else { iy += sy; tny += tdy; }
    }
    return best;
}

void sg_render_outdoor(const double *hf, int hnx, int hny, double hx0, double hy0, double hs, const double *box,
                       const int32_t *bstart, const int32_t *bitems, int ncx, int ncy, double bx0, double by0,
                       double bgs, int H, int W, double fx, double fy, double cx, double cy, const double *T,
                       double max_range, int noise_model, double noise_a, double invalid_frac, uint32_t seed,
                       uint32_t frame, float *out)
{
    hgrid_t hg = {hf, hnx, hny, hx0, hy0, hs};
    bgrid_t bg = {box, bstart, bitems, ncx, ncy, bx0, by0, bgs};
    const double o[3] = {T[3], T[7], T[11]};
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < H; ++r) {
        for (int c = 0; c < W; ++c) {
            double dc[3] = {((double)c - cx) / fx, ((double)r - cy) / fy, 1.0};
            double d[3];
            for (int k = 0; k < 3; ++k)
                d[k] = T[4 * k + 0] * dc[0] + T[4 * k + 1] * dc[1] + T[4 * k + 2] * dc[2];
            double s = hit_hgrid(&hg, o, d, max_range);
            double lim = s < max_range ? s : max_range;
            double tb = hit_bgrid(&bg, o, d, lim);
            if (tb < s) s = tb;
            double z = (s <= max_range) ? s : 0.0;
            uint32_t pix = (uint32_t)(r * W + c);
            if (z > 0.0 && (noise_model != 0 || invalid_frac > 0.0)) {
                double gn, u;
                pixel_draws(seed, frame, pix, &gn, &u);
                double sigma = noise_model == 1 ? noise_a : noise_model == 2 ? noise_a * z * z : 0.0;
                z += sigma * gn;
                if (z <= 0.0) z = 0.0;
                if (u < invalid_frac) z = 0.0;
            }
            out[(size_t)r * W + c] = (float)z;
        }
    }
}
