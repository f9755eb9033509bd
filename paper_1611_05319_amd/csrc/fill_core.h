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
    __device__ int index(int x, int y) const { return y * W + x; }
    __device__ int pitch() const { return W; }
    __device__ int32_t state_at(int i) const { return S[i]; }
    __device__ double colour_at(int i, int c) const { return load_px(U + (long long)i * C + c); }
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
    __device__ int index(int x, int y) const { return y * WW + x; }
    __device__ int pitch() const { return WW; }
    __device__ int32_t state_at(int i) const { return st[i]; }
    __device__ double colour_at(int i, int c) const { return load_px(col + i * C + c); }
};

// Weights are exp(-(q - q_min)) / |(n, m)|: relative to the largest readable
// weight (the quotient is unchanged, nothing underflows), with the exact
// distance of the unrotated offset.  With the rotated ball the exponent is
// q = a |g|^2 n^2 (g_perp . R(n, m) = -|g| n), so it takes at most R + 1
// values: lane |n| of the group evaluates exp once and the others read it by
// a shuffle.
// Returns true (on every lane of the group) when the pixel is ready; then
// out[0..C) holds its new colour (FP64, before storage rounding).
// (X, Y): the pixel in the view's coordinates; k: the shell used by the
// readable test (s in [-1, k-1]); a = mu^2 / (2 eps^2); c < 0: onion order;
// R = floor(eps) < G.
template <typename TS, int G, typename V>
__device__ bool fill_core(const V &v, int X, int Y, double gx, double gy, bool ghost,
                          const short2 *off, const double *rinv, int T, int R, int k, int l,
                          double a, double c, double out[4]) {
    const bool rot = ghost && (gx != 0.0 || gy != 0.0);
    const double L2 = gx * gx + gy * gy;
    double cs = 0.0, sn = 0.0;
    if (rot) {
        const double L = sqrt(L2);
        cs = gx / L;
        sn = gy / L;
    }
    const double aL2 = a * L2;
    // pass 1: readable set, exponents, bilinear supports (kept for pass 2)
    double q[kPerLaneMax], fxs[kPerLaneMax], fys[kPerLaneMax];
    int base[kPerLaneMax];
    unsigned rmask = 0, exmask = 0, eymask = 0;
    double qmin_r = INFINITY, qmin_all = INFINITY;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        q[r] = INFINITY;
        fxs[r] = 0.0;
        fys[r] = 0.0;
        base[r] = 0;
        const int t = l + r * G;
        if (t < T) {
            const short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            const double fx0 = floor(ox), fy0 = floor(oy);
            const bool ex = (ox == fx0), ey = (oy == fy0);
            const int x0 = X + (int)fx0, y0 = Y + (int)fy0;
            const int x1 = x0 + (ex ? 0 : 1), y1 = y0 + (ey ? 0 : 1);
            fxs[r] = ox - fx0;
            fys[r] = oy - fy0;
            exmask |= ex ? (1u << r) : 0u;
            eymask |= ey ? (1u << r) : 0u;
            bool rd = false;
            if (v.inside(x0, y0, x1, y1)) {
                const int b = v.index(x0, y0), P = v.pitch();
                base[r] = b;
                const int dx = ex ? 0 : 1, dy = ey ? 0 : P;
                const int32_t a0 = v.state_at(b), a1 = v.state_at(b + dx);
                const int32_t a2 = v.state_at(b + dy), a3 = v.state_at(b + dy + dx);
                rd = ((int)readable(a0, k) & (int)readable(a1, k) & (int)readable(a2, k) &
                      (int)readable(a3, k)) != 0;
            }
            if (rot) {
                q[r] = aL2 * (double)(nm.x * nm.x);
            } else {
                const double tp = (-gy) * ox + gx * oy;
                q[r] = a * tp * tp;
            }
            qmin_all = fmin(qmin_all, q[r]);
            if (rd) {
                rmask |= 1u << r;
                qmin_r = fmin(qmin_r, q[r]);
            }
        }
    }
    qmin_r = gmin<G>(qmin_r);
    if (!(qmin_r < INFINITY)) return false;  // no readable point: the pixel waits
    // exponentials: shared by |n| with the rotated ball, one per offset otherwise
    double e_r = 0.0, e_all = 0.0;
    if (rot && l <= R) {
        e_r = exp(-(aL2 * (double)(l * l) - qmin_r));
        e_all = exp(-(aL2 * (double)(l * l)));  // q_min over the whole ball is 0 (n = 0)
    }
    if (c >= 0.0) {  // smart order
        if (!rot) qmin_all = gmin<G>(qmin_all);
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int r = 0; r < kPerLaneMax; ++r) {
            const int t = l + r * G;
            double w = 0.0;
            if (rot) {
                const int an = t < T ? abs((int)off[t].x) : 0;
                w = __shfl(e_all, an, G) * (t < T ? rinv[t] : 0.0);
            } else if (t < T) {
                w = exp(-(q[r] - qmin_all)) * rinv[t];
            }
            den += w;
            if (rmask & (1u << r)) num += w;
        }
        num = gsum<G>(num);
        den = gsum<G>(den);
        if (!(num / den > c)) return false;
    }
    // pass 2: weighted average of the readable ghost values
    double Ssum = 0.0, acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int C = v.C, P = v.pitch();
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        const int t = l + r * G;
        double w = 0.0;
        if (rot) {  // every lane takes part in the shuffle
            const int an = t < T ? abs((int)off[t].x) : 0;
            w = __shfl(e_r, an, G);
        }
        if (rmask & (1u << r)) {
            w = (rot ? w : exp(-(q[r] - qmin_r))) * rinv[t];
            Ssum += w;
            const bool ex = (exmask >> r) & 1u, ey = (eymask >> r) & 1u;
            const double wx1 = ex ? 0.0 : fxs[r], wy1 = ey ? 0.0 : fys[r];
            const double wx0 = 1.0 - wx1, wy0 = 1.0 - wy1;
            const double b00 = wx0 * wy0, b10 = wx1 * wy0, b01 = wx0 * wy1, b11 = wx1 * wy1;
            const int i00 = base[r], i10 = i00 + (ex ? 0 : 1), i01 = i00 + (ey ? 0 : P),
                      i11 = i01 + (ex ? 0 : 1);
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch < C) {
                    const double val = b00 * v.colour_at(i00, ch) + b10 * v.colour_at(i10, ch) +
                                       b01 * v.colour_at(i01, ch) + b11 * v.colour_at(i11, ch);
                    acc[ch] += w * val;
                }
            }
        }
    }
    Ssum = gsum<G>(Ssum);
    const double inv = 1.0 / Ssum;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
        if (ch < C) out[ch] = gsum<G>(acc[ch]) * inv;
    return true;
}

}  // namespace gfk
