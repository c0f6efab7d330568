/*
 * covox oracle, learned-proposal part -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain loops for the coarse ESDF summaries and for the small 3-D
 * convolutional network (forward, loss, backward) that the GPU library runs
 * on its matrix cores.  Shares no code with the library.
 *
 * Network: layers of 3x3x3 convolutions with zero padding 1 and a stride,
 * each followed by ReLU; global mean over the last layer's positions; a fully
 * connected layer to 5 outputs.  Tensors are NDHWC.  Parameter vector:
 * for each convolution w[cout][((kd * 3 + kh) * 3 + kw) * cin + ci] then
 * b[cout]; then fc w[5][feat] and b[5].
 *
 * bf16 mode follows the library's rounding points: inputs and convolution
 * weights rounded to bfloat16 (nearest even), products accumulated in
 * binary32 in ascending k order, bias added and ReLU applied in binary32,
 * layer outputs rounded to bfloat16; mean and head in binary32.  The
 * binary64 mode does the same arithmetic in binary64 without rounding (for
 * the finite-difference gradient check).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int cin, cout, din, dout, stride;
} orc_conv;

typedef struct orc_submap orc_submap;
double orc_phi_at_voxel(const orc_submap *s, int64_t x, int64_t y, int64_t z); /* covox_oracle.c */

float orc_bf16_round(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7F800000u) == 0x7F800000u) {
        if (x & 0x7FFFFFu) x |= 0x400000u; /* quiet NaN */
        x &= 0xFFFF0000u;
    } else {
        uint32_t lsb = (x >> 16) & 1u;
        x += 0x7FFFu + lsb;
        x &= 0xFFFF0000u;
    }
    float r;
    memcpy(&r, &x, 4);
    return r;
}

static int64_t conv_params(const orc_conv *c) { return (int64_t)c->cout * 27 * c->cin + c->cout; }

int64_t orc_net_num_params(const orc_conv *L, int nl, int feat)
{
    int64_t n = 0;
    for (int l = 0; l < nl; ++l) n += conv_params(&L[l]);
    return n + 5 * feat + 5;
}

/* One convolution layer.  x: n * din^3 * cin, y: n * dout^3 * cout. */
static void conv_forward(const orc_conv *c, int n, const double *w, const double *b, const double *x, double *y,
                         int bf16)
{
    const int K = 27 * c->cin;
    for (int nb = 0; nb < n; ++nb)
        for (int oz = 0; oz < c->dout; ++oz)
            for (int oy = 0; oy < c->dout; ++oy)
                for (int ox = 0; ox < c->dout; ++ox) {
                    int64_t o = (((int64_t)nb * c->dout + oz) * c->dout + oy) * c->dout + ox;
                    for (int co = 0; co < c->cout; ++co) {
                        double acc64 = 0.0;
                        float acc32 = 0.0f;
                        for (int k = 0; k < K; ++k) {
                            int off = k / c->cin, ci = k % c->cin;
                            int kd = off / 9, kh = (off / 3) % 3, kw = off % 3;
                            int iz = oz * c->stride + kd - 1, iy = oy * c->stride + kh - 1, ix = ox * c->stride + kw - 1;
                            if (iz < 0 || iy < 0 || ix < 0 || iz >= c->din || iy >= c->din || ix >= c->din) continue;
                            double xv = x[((((int64_t)nb * c->din + iz) * c->din + iy) * c->din + ix) * c->cin + ci];
                            double wv = w[(int64_t)co * K + k];
                            if (bf16) acc32 += (float)xv * (float)wv;
                            else acc64 += xv * wv;
                        }
                        double v;
                        if (bf16) {
                            float t = acc32 + (float)b[co];
                            t = t > 0.0f ? t : 0.0f;
                            v = orc_bf16_round(t);
                        } else {
                            v = acc64 + b[co];
                            v = v > 0.0 ? v : 0.0;
                        }
                        y[o * c->cout + co] = v;
                    }
                }
}

static int64_t act_size(const orc_conv *c, int n) { return (int64_t)n * c->dout * c->dout * c->dout * c->cout; }

/* Forward pass; acts (nullable) receives every layer output back to back,
 * pooled the means (n * feat). */
static void net_forward(const orc_conv *L, int nl, int feat, const float *params, const float *x, int n, int bf16,
                        double *out, double **acts_out, double *pooled)
{
    int64_t np = orc_net_num_params(L, nl, feat);
    double *P = (double *)malloc(sizeof(double) * np);
    /* weights as used by the forward pass */
    int64_t o = 0;
    for (int l = 0; l < nl; ++l) {
        int64_t nw = (int64_t)L[l].cout * 27 * L[l].cin;
        for (int64_t i = 0; i < nw; ++i) P[o + i] = bf16 ? orc_bf16_round(params[o + i]) : params[o + i];
        o += nw;
        for (int i = 0; i < L[l].cout; ++i) P[o + i] = params[o + i];
        o += L[l].cout;
    }
    for (int64_t i = o; i < np; ++i) P[i] = params[i];
    int64_t nx = (int64_t)n * L[0].din * L[0].din * L[0].din * L[0].cin;
    double *in = (double *)malloc(sizeof(double) * nx);
    for (int64_t i = 0; i < nx; ++i) in[i] = bf16 ? orc_bf16_round(x[i]) : x[i];
    o = 0;
    for (int l = 0; l < nl; ++l) {
        int64_t nw = (int64_t)L[l].cout * 27 * L[l].cin;
        conv_forward(&L[l], n, P + o, P + o + nw, in, acts_out[l], bf16);
        o += nw + L[l].cout;
        free(in);
        in = NULL;
        /* next layer reads acts_out[l] */
        if (l + 1 < nl) {
            in = (double *)malloc(sizeof(double) * act_size(&L[l], n));
            memcpy(in, acts_out[l], sizeof(double) * act_size(&L[l], n));
        }
    }
    const orc_conv *last = &L[nl - 1];
    int npos = last->dout * last->dout * last->dout;
    const double *fw = P + o, *fb = P + o + 5 * feat;
    for (int b = 0; b < n; ++b) {
        for (int c = 0; c < feat; ++c) {
            if (bf16) {
                float s = 0.0f;
                for (int p = 0; p < npos; ++p) s += (float)acts_out[nl - 1][((int64_t)b * npos + p) * feat + c];
                pooled[b * feat + c] = s * (1.0f / (float)npos);
            } else {
                double s = 0.0;
                for (int p = 0; p < npos; ++p) s += acts_out[nl - 1][((int64_t)b * npos + p) * feat + c];
                pooled[b * feat + c] = s / npos;
            }
        }
        for (int k = 0; k < 5; ++k) {
            if (bf16) {
                float t = (float)fb[k];
                for (int c = 0; c < feat; ++c) t += (float)fw[k * feat + c] * (float)pooled[b * feat + c];
                out[b * 5 + k] = t;
            } else {
                double t = fb[k];
                for (int c = 0; c < feat; ++c) t += fw[k * feat + c] * pooled[b * feat + c];
                out[b * 5 + k] = t;
            }
        }
    }
    free(P);
}

int orc_net_forward(const orc_conv *L, int nl, int feat, const float *params, const float *x, int n, int bf16,
                    double *out)
{
    double **acts = (double **)malloc(sizeof(double *) * nl);
    for (int l = 0; l < nl; ++l) acts[l] = (double *)malloc(sizeof(double) * act_size(&L[l], n));
    double *pooled = (double *)malloc(sizeof(double) * n * feat);
    net_forward(L, nl, feat, params, x, n, bf16, out, acts, pooled);
    for (int l = 0; l < nl; ++l) free(acts[l]);
    free(acts);
    free(pooled);
    return 0;
}

/*
 * Loss = (1/n) sum_b [ sum_{k<3} (o - y)^2 / s^2 + sum_{k>=3} (o - y)^2 ] and
 * its gradient with respect to every parameter, by backpropagation in
 * binary64 through the forward values of the chosen mode (ReLU derivative:
 * 1 where the layer output is positive).
 */
int orc_net_loss_grad(const orc_conv *L, int nl, int feat, const float *params, const float *x, const float *y, int n,
                      int bf16, double trans_scale, double *grad, double *loss)
{
    int64_t np = orc_net_num_params(L, nl, feat);
    double **acts = (double **)malloc(sizeof(double *) * nl);
    for (int l = 0; l < nl; ++l) acts[l] = (double *)malloc(sizeof(double) * act_size(&L[l], n));
    double *pooled = (double *)malloc(sizeof(double) * n * feat);
    double *out = (double *)malloc(sizeof(double) * n * 5);
    net_forward(L, nl, feat, params, x, n, bf16, out, acts, pooled);
    memset(grad, 0, sizeof(double) * np);
    /* offsets */
    int64_t *ow = (int64_t *)malloc(sizeof(int64_t) * nl), *ob = (int64_t *)malloc(sizeof(int64_t) * nl);
    int64_t o = 0;
    for (int l = 0; l < nl; ++l) {
        ow[l] = o;
        o += (int64_t)L[l].cout * 27 * L[l].cin;
        ob[l] = o;
        o += L[l].cout;
    }
    int64_t ofw = o, ofb = o + 5 * feat;
    double inv2 = 1.0 / (trans_scale * trans_scale);
    double *dout = (double *)malloc(sizeof(double) * n * 5);
    double ls = 0.0;
    for (int b = 0; b < n; ++b)
        for (int k = 0; k < 5; ++k) {
            double wk = k < 3 ? inv2 : 1.0;
            double d = out[b * 5 + k] - y[b * 5 + k];
            ls += wk * d * d / n;
            dout[b * 5 + k] = 2.0 * wk * d / n;
        }
    *loss = ls;
    const orc_conv *last = &L[nl - 1];
    int npos = last->dout * last->dout * last->dout;
    /* head */
    double *dact = (double *)calloc(act_size(last, n), sizeof(double));
    for (int b = 0; b < n; ++b)
        for (int k = 0; k < 5; ++k) {
            grad[ofb + k] += dout[b * 5 + k];
            for (int c = 0; c < feat; ++c) grad[ofw + k * feat + c] += dout[b * 5 + k] * pooled[b * feat + c];
        }
    for (int b = 0; b < n; ++b)
        for (int c = 0; c < feat; ++c) {
            double dp = 0.0;
            for (int k = 0; k < 5; ++k) dp += dout[b * 5 + k] * params[ofw + k * feat + c];
            for (int p = 0; p < npos; ++p) {
                int64_t q = ((int64_t)b * npos + p) * feat + c;
                dact[q] = acts[nl - 1][q] > 0.0 ? dp / npos : 0.0; /* through ReLU */
            }
        }
    /* convolutions, last to first; dact holds d loss / d pre-activation */
    for (int l = nl - 1; l >= 0; --l) {
        const orc_conv *c = &L[l];
        const int K = 27 * c->cin;
        double *xin;
        int64_t nx = (int64_t)n * c->din * c->din * c->din * c->cin;
        xin = (double *)malloc(sizeof(double) * nx);
        if (l == 0)
            for (int64_t i = 0; i < nx; ++i) xin[i] = bf16 ? orc_bf16_round(x[i]) : x[i];
        else
            memcpy(xin, acts[l - 1], sizeof(double) * nx);
        double *dx = (l > 0) ? (double *)calloc(nx, sizeof(double)) : NULL;
        for (int nb = 0; nb < n; ++nb)
            for (int oz = 0; oz < c->dout; ++oz)
                for (int oy = 0; oy < c->dout; ++oy)
                    for (int ox = 0; ox < c->dout; ++ox) {
                        int64_t op = (((int64_t)nb * c->dout + oz) * c->dout + oy) * c->dout + ox;
                        for (int co = 0; co < c->cout; ++co) {
                            double g = dact[op * c->cout + co];
                            if (g == 0.0) continue;
                            grad[ob[l] + co] += g;
                            for (int k = 0; k < K; ++k) {
                                int off = k / c->cin, ci = k % c->cin;
                                int kd = off / 9, kh = (off / 3) % 3, kw = off % 3;
                                int iz = oz * c->stride + kd - 1, iy = oy * c->stride + kh - 1, ix = ox * c->stride + kw - 1;
                                if (iz < 0 || iy < 0 || ix < 0 || iz >= c->din || iy >= c->din || ix >= c->din) continue;
                                int64_t xi = ((((int64_t)nb * c->din + iz) * c->din + iy) * c->din + ix) * c->cin + ci;
                                grad[ow[l] + (int64_t)co * K + k] += g * xin[xi];
                                if (dx) dx[xi] += g * params[ow[l] + (int64_t)co * K + k];
                            }
                        }
                    }
        free(dact);
        dact = NULL;
        if (dx) {
            /* through the ReLU of the layer that produced x */
            for (int64_t i = 0; i < nx; ++i)
                if (!(xin[i] > 0.0)) dx[i] = 0.0;
            dact = dx;
        }
        free(xin);
    }
    free(dact);
    for (int l = 0; l < nl; ++l) free(acts[l]);
    free(acts);
    free(pooled);
    free(out);
    free(dout);
    free(ow);
    free(ob);
    return 0;
}

/*
 * Coarse summary of a submap (binary64): for cell c = (x, y, z) of the 32^3
 * grid (x fastest), the point ((c + 0.5) - 16) * cell in grid coordinates is
 * mapped into the submap by T; phi is interpolated trilinearly from the 8
 * voxel corners of its cell (g = q / vs - 0.5) when all are observed:
 * out[2c] = clamp(phi / d_max, -1, 1), out[2c + 1] = 1, else 0 and 0.
 */
int orc_summary(const orc_submap *s, double vs, double dmax, const double *T, double cell, double *out)
{
    for (int c = 0; c < 32768; ++c) {
        int cx = c & 31, cy = (c >> 5) & 31, cz = c >> 10;
        double g[3] = {((cx + 0.5) - 16.0) * cell, ((cy + 0.5) - 16.0) * cell, ((cz + 0.5) - 16.0) * cell};
        double q[3], f[3];
        int64_t j0[3];
        for (int a = 0; a < 3; ++a) q[a] = T[4 * a] * g[0] + T[4 * a + 1] * g[1] + T[4 * a + 2] * g[2] + T[4 * a + 3];
        for (int a = 0; a < 3; ++a) {
            double u = q[a] / vs - 0.5;
            double fl = floor(u);
            j0[a] = (int64_t)fl;
            f[a] = u - fl;
        }
        double cor[8];
        int ok = 1;
        for (int k = 0; k < 8 && ok; ++k) {
            cor[k] = orc_phi_at_voxel(s, j0[0] + (k & 1), j0[1] + ((k >> 1) & 1), j0[2] + ((k >> 2) & 1));
            if (isnan(cor[k])) ok = 0;
        }
        if (!ok) {
            out[2 * c] = 0.0;
            out[2 * c + 1] = 0.0;
            continue;
        }
        double c00 = cor[0] * (1 - f[0]) + cor[1] * f[0], c10 = cor[2] * (1 - f[0]) + cor[3] * f[0];
        double c01 = cor[4] * (1 - f[0]) + cor[5] * f[0], c11 = cor[6] * (1 - f[0]) + cor[7] * f[0];
        double c0 = c00 * (1 - f[1]) + c10 * f[1], c1 = c01 * (1 - f[1]) + c11 * f[1];
        double r = c0 * (1 - f[2]) + c1 * f[2];
        double v = r / dmax;
        out[2 * c] = v < -1.0 ? -1.0 : (v > 1.0 ? 1.0 : v);
        out[2 * c + 1] = 1.0;
    }
    return 0;
}
