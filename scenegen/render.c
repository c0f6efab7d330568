/*
 * Seeded synthetic depth renderer (input generation only).
 *
 * This file produces the depth frames that both the reference checker and
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
