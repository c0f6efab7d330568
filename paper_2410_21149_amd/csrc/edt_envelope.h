// Lower envelope of the parabolas f_q(y) = f(q) + (y - q)^2 along one line
// (Felzenszwalb and Huttenlocher, "Distance transforms of sampled
// functions"), in exact integer arithmetic.  Shared by the y and z passes of
// the ESDF; host-callable so the logic can be checked on the CPU.
//
// Breakpoint of parabolas p < q: s(p, q) = N / D with
//   N = (f_q - f_p) + (q - p)(q + p),  D = 2 (q - p) > 0.
// Positions are < 256 and f <= 56^2, so |N| < 2^18, D < 2^9 and every
// cross-product fits in 32 bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace covox {

// Envelope stack: entry k of the stack of line `lane` is stk[k * stride +
// lane]; the top two entries are cached.
struct Envelope {
    int k;        // top index, -1 = empty
    int p, fp;    // top entry
    int pp, fpp;  // entry below the top (valid when k >= 1)
};

__host__ __device__ inline void env_clear(Envelope &e)
{
    e.k = -1;
    e.p = e.fp = e.pp = e.fpp = 0;
}

// Appends parabola (q, fq); positions must arrive in increasing order.
template <typename GetF>
__host__ __device__ inline void env_push(Envelope &e, uint8_t *stk, int stride, int lane, int q, int fq, GetF getf)
{
    while (e.k >= 1) {
        const int N1 = (fq - e.fp) + (q - e.p) * (q + e.p), D1 = 2 * (q - e.p);
        const int N2 = (e.fp - e.fpp) + (e.p - e.pp) * (e.p + e.pp), D2 = 2 * (e.p - e.pp);
        if (N1 * D2 > N2 * D1) break;
        // s(top, q) <= s(below, top): the top parabola is nowhere lowest
        --e.k;
        e.p = e.pp;
        e.fp = e.fpp;
        if (e.k >= 1) {
            e.pp = stk[(e.k - 1) * stride + lane];
            e.fpp = getf(e.pp);
        }
    }
    ++e.k;
    stk[e.k * stride + lane] = (uint8_t)q;
    e.pp = e.p;
    e.fpp = e.fp;
    e.p = q;
    e.fp = fq;
}

// Walks the envelope left to right.
struct Walker {
    int kk, cur, fcur, nxt, fnxt;
};

template <typename GetF>
__host__ __device__ inline void walk_init(Walker &w, const Envelope &e, const uint8_t *stk, int stride, int lane,
                                          GetF getf)
{
    w.kk = 0;
    w.cur = stk[lane];
    w.fcur = getf(w.cur);
    w.nxt = 0;
    w.fnxt = 0;
    if (e.k >= 1) {
        w.nxt = stk[stride + lane];
        w.fnxt = getf(w.nxt);
    }
}

// Value of the envelope at y; queries must come in non-decreasing y.
template <typename GetF>
__host__ __device__ inline int walk_at(Walker &w, const Envelope &e, const uint8_t *stk, int stride, int lane, int y,
                                       GetF getf)
{
    while (w.kk < e.k) {
        const int N = (w.fnxt - w.fcur) + (w.nxt - w.cur) * (w.nxt + w.cur), D = 2 * (w.nxt - w.cur);
        if (N >= y * D) break;
        ++w.kk;
        w.cur = w.nxt;
        w.fcur = w.fnxt;
        if (w.kk < e.k) {
            w.nxt = stk[(w.kk + 1) * stride + lane];
            w.fnxt = getf(w.nxt);
        }
    }
    const int dy = y - w.cur;
    return dy * dy + w.fcur;
}

}  // namespace covox
