// The fill of one front pixel by a group of G lanes (Guidefill, arXiv
// 1611.05319): Algorithm 1's weighted average over the readable points of the
// rotated ball of ghost pixels (Sec. 3.1, 3.3, eqn:weight, eqn:bilinearDef),
// with onion order or the smart-order test (Sec. 3.4, eqn:confidence,
// eqn:ready).  The state and colours are read through a view: the frame in
// global memory, or a tile window staged in LDS.
#pragma once

#include "device_common.h"

namespace gfk {

// frame in global memory (state = shell map)
template <typename TS> struct GlobalView {
    const int32_t *S;
    const TS *U;
    int W, H, C;
    __device__ bool inside(int x0, int y0, int x1, int y1) const {
        return x0 >= 0 && y0 >= 0 && x1 < W && y1 < H;
    }
    __device__ int32_t state(int x, int y) const { return S[y * W + x]; }
    __device__ double colour(int x, int y, int c) const {
        return load_px(U + (long long)(y * W + x) * C + c);
    }
};

// tile window in LDS (state = window codes; pixels outside the frame are
// bystander-coded, so they are never readable)
template <typename TS> struct LdsView {
    const int32_t *st;
    const TS *col;
    int WW, WH, C;
    __device__ bool inside(int x0, int y0, int x1, int y1) const {
        return x0 >= 0 && y0 >= 0 && x1 < WW && y1 < WH;
    }
    __device__ int32_t state(int x, int y) const { return st[y * WW + x]; }
    __device__ double colour(int x, int y, int c) const {
        return load_px(col + (y * WW + x) * C + c);
    }
};

// Weights are exp(-(q - q_min)) / |(n, m)|: relative to the largest readable
// weight (the quotient is unchanged, nothing underflows), with the exact
// distance of the unrotated offset.
// Returns true (on every lane of the group) when the pixel is ready; then
// out[0..C) holds its new colour (FP64, before storage rounding).
// (X, Y): the pixel in the view's coordinates; k: the shell used by the
// readable test (s in [-1, k-1]); a = mu^2 / (2 eps^2); c < 0: onion order.
template <typename TS, int G, typename V>
__device__ bool fill_core(const V &v, int X, int Y, double gx, double gy, bool ghost,
                          const short2 *off, const double *rinv, int T, int k, int l, double a,
                          double c, double out[4]) {
    const bool rot = ghost && (gx != 0.0 || gy != 0.0);
    double cs = 0.0, sn = 0.0;
    if (rot) {
        double L = sqrt(gx * gx + gy * gy);
        cs = gx / L;
        sn = gy / L;
    }
    // pass 1: readable set and exponents q = a (g_perp . o)^2
    double q[kPerLaneMax];
    unsigned rmask = 0;
    double qmin_r = INFINITY, qmin_all = INFINITY;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        q[r] = INFINITY;
        const int t = l + r * G;
        if (t < T) {
            const short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            const Support s = support_of(X, Y, ox, oy);
            bool rd = false;
            if (v.inside(s.x0, s.y0, s.x1, s.y1)) {
                const int32_t a0 = v.state(s.x0, s.y0), a1 = v.state(s.x1, s.y0);
                const int32_t a2 = v.state(s.x0, s.y1), a3 = v.state(s.x1, s.y1);
                rd = ((int)readable(a0, k) & (int)readable(a1, k) & (int)readable(a2, k) &
                      (int)readable(a3, k)) != 0;
            }
            const double tp = (-gy) * ox + gx * oy;
            q[r] = a * tp * tp;
            qmin_all = fmin(qmin_all, q[r]);
            if (rd) {
                rmask |= 1u << r;
                qmin_r = fmin(qmin_r, q[r]);
            }
        }
    }
    qmin_r = gmin<G>(qmin_r);
    if (!(qmin_r < INFINITY)) return false;  // no readable point: the pixel waits
    if (c >= 0.0) {                          // smart order
        qmin_all = gmin<G>(qmin_all);
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int r = 0; r < kPerLaneMax; ++r) {
            const int t = l + r * G;
            if (t < T) {
                const double w = exp(-(q[r] - qmin_all)) * rinv[t];
                den += w;
                if (rmask & (1u << r)) num += w;
            }
        }
        num = gsum<G>(num);
        den = gsum<G>(den);
        if (!(num / den > c)) return false;
    }
    // pass 2: weighted average of the readable ghost values
    double Ssum = 0.0, acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int C = v.C;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        if (rmask & (1u << r)) {
            const int t = l + r * G;
            const short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            const Support s = support_of(X, Y, ox, oy);
            const double w = exp(-(q[r] - qmin_r)) * rinv[t];
            Ssum += w;
            const double b00 = s.wx0 * s.wy0, b10 = s.wx1 * s.wy0, b01 = s.wx0 * s.wy1,
                         b11 = s.wx1 * s.wy1;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch < C) {
                    const double val = b00 * v.colour(s.x0, s.y0, ch) + b10 * v.colour(s.x1, s.y0, ch) +
                                       b01 * v.colour(s.x0, s.y1, ch) + b11 * v.colour(s.x1, s.y1, ch);
                    acc[ch] += w * val;
                }
            }
        }
    }
    Ssum = gsum<G>(Ssum);
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
        if (ch < C) out[ch] = gsum<G>(acc[ch]) / Ssum;
    return true;
}

}  // namespace gfk
