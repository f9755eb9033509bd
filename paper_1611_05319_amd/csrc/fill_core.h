// The fill of one front pixel by a group of G lanes (Guidefill, arXiv
// 1611.05319): Algorithm 1's weighted average over the readable points of the
// rotated ball of ghost pixels (Sec. 3.1, 3.3, eqn:weight, eqn:bilinearDef),
// with onion order or the smart-order test (Sec. 3.4, eqn:confidence,
// eqn:ready).  The state and colours are read from a window staged in LDS: a
// tile window (tiled engine) or one pixel's neighbourhood (global-front
// engine, adjoint).
//
// Precision: every quantity that decides a shell (the ghost offsets, their
// floors and lattice-line tests, the smart-order confidence) is FP64 with no
// contraction, as the reference computes it.  The weights and the weighted
// sum are FP64; the bilinear value of one ghost point is interpolated in FP32
// from binary32 colours (exact on lattice lines and for constant data) and in
// FP64 from binary16 colours.
#pragma once

#include <type_traits>

#include "device_common.h"

namespace gfk {

// colours as FP32
__device__ inline float px_f32(float v) { return v; }
__device__ inline float px_f32(__half v) { return __half2float(v); }

// channels of a pixel in an LDS window: always 4 (padding never read into a
// result), so a pixel's colours are one vector load
__host__ __device__ inline int padded_channels(int) { return 4; }

template <typename TS> __device__ inline void lds_colours(const TS *p, float o[4]);
template <> __device__ inline void lds_colours<float>(const float *p, float o[4]) {
    const float4 v = *reinterpret_cast<const float4 *>(__builtin_assume_aligned(p, 16));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <> __device__ inline void lds_colours<__half>(const __half *p, float o[4]) {
    const uint2 v = *reinterpret_cast<const uint2 *>(__builtin_assume_aligned(p, 8));
    o[0] = __half2float(__ushort_as_half((unsigned short)(v.x & 0xffffu)));
    o[1] = __half2float(__ushort_as_half((unsigned short)(v.x >> 16)));
    o[2] = __half2float(__ushort_as_half((unsigned short)(v.y & 0xffffu)));
    o[3] = __half2float(__ushort_as_half((unsigned short)(v.y >> 16)));
}

// tile window in LDS (state = window codes; pixels outside the frame are
// bystander-coded, so they are never readable); CP channels per pixel
template <typename TS> struct LdsView {
    const int32_t *st;
    const TS *col;
    int WW, WH, C, CP;
    __device__ bool inside(int x0, int y0, int x1, int y1) const {
        return x0 >= 0 && y0 >= 0 && x1 < WW && y1 < WH;
    }
    __device__ int index(int x, int y) const { return y * WW + x; }
    __device__ int pitch() const { return WW; }
    __device__ int32_t state_at(int i) const { return st[i]; }
    __device__ void colours(int i, float o[4]) const { lds_colours<TS>(col + i * 4, o); }
};

// Weights are exp(-(q - q_min)) / |(n, m)|: relative to the largest readable
// weight (the quotient is unchanged, nothing underflows), with the exact
// distance of the unrotated offset.  With the rotated ball the exponent is
// q = a |g|^2 n^2 (g_perp . R(n, m) = -|g| n), so it takes at most R + 1
// values: lane |n| of the group evaluates exp once and the others read it by
// a shuffle; q_min is a |g|^2 times the smallest readable n^2.  The lattice
// ball (no ghost pixels, or g = 0) evaluates exp per offset; that code runs
// only in wavefronts that hold such a pixel.
// The geometry pass is branch-free: the offset table is padded with entries
// that are never readable and weigh 0, and every load stays inside the view.
// Returns true (on every lane of the group) when the pixel is ready; then
// out[0..C) holds its new colour (FP64, before storage rounding).
// (X, Y): the pixel in the view's coordinates; k: the shell used by the
// readable test (s in [-1, k-1]); a = mu^2 / (2 eps^2); c < 0: onion order;
// R = floor(eps) < G; off / rinv: the padded offset table (per_lane<G>() * G
// entries).
template <typename TS, int G, typename V>
__device__ __attribute__((always_inline)) bool fill_core(const V &v, int X, int Y, double gx, double gy, bool ghost,
                          const short2 *off, const double *rinv, int T, int R, int k, int l,
                          double a, double c, double out[4]) {
    const bool rot = ghost && (gx != 0.0 || gy != 0.0);
    const bool lattice_here = __any(!rot);  // wavefront-uniform
    const double L2 = gx * gx + gy * gy;
    // R takes (0, 1) to g/|g|; the lattice ball is R = identity, (c, s) = (0, 1),
    // which the same products give exactly (n * 1 + m * 0 = n, m * 1 - n * 0 = m)
    double cs = 0.0, sn = 1.0;
    if (rot) {
        const double L = sqrt(L2);
        cs = gx / L;
        sn = gy / L;
    }
    const double aL2 = a * L2;
    const int P = v.pitch();
    // pass 1: readable set and bilinear supports (kept for pass 2)
    constexpr int PL = per_lane<G>();
    // binary16 storage: the ghost values are interpolated in FP64 (see pass 2)
    constexpr bool kF64Values = std::is_same<TS, __half>::value;
    using FT = typename std::conditional<kF64Values, double, float>::type;
    FT fxs[PL], fys[PL];
    int base[PL];
    unsigned rmask = 0, exmask = 0, eymask = 0;
    int n2min = 0x7fffffff;    // rotated ball: smallest readable n^2
    double qmin_r = INFINITY;  // lattice ball: smallest readable exponent
#pragma unroll
    for (int r = 0; r < PL; ++r) {
        const int t = l + r * G;
        const short2 nm = off[t];
        double ox, oy;
        rot_offset(true, cs, sn, nm.x, nm.y, ox, oy);
        const double fx0 = floor(ox), fy0 = floor(oy);
        const bool ex = (ox == fx0), ey = (oy == fy0);
        const int x0 = X + (int)fx0, y0 = Y + (int)fy0;
        const int x1 = x0 + (ex ? 0 : 1), y1 = y0 + (ey ? 0 : 1);
        fxs[r] = (FT)(ox - fx0);
        fys[r] = (FT)(oy - fy0);
        const bool ins = v.inside(x0, y0, x1, y1);
        const int b = ins ? v.index(x0, y0) : 0;
        const int dx = (ex || !ins) ? 0 : 1, dy = (ey || !ins) ? 0 : P;
        const int32_t a0 = v.state_at(b), a1 = v.state_at(b + dx);
        const int32_t a2 = v.state_at(b + dy), a3 = v.state_at(b + dy + dx);
        const bool rd = ins && (((int)readable(a0, k) & (int)readable(a1, k) &
                                 (int)readable(a2, k) & (int)readable(a3, k)) != 0);
        base[r] = b;
        rmask |= rd ? (1u << r) : 0u;
        exmask |= (ex || !rd) ? (1u << r) : 0u;  // unreadable points read one pixel
        eymask |= (ey || !rd) ? (1u << r) : 0u;
        n2min = min(n2min, rd ? (int)nm.x * (int)nm.x : 0x7fffffff);
        if (lattice_here) {
            const double tp = (-gy) * ox + gx * oy;
            qmin_r = fmin(qmin_r, rd ? a * tp * tp : INFINITY);
        }
    }
    // exponentials of the readable weights
    n2min = gmin_i<G>(n2min);
    if (lattice_here) qmin_r = gmin<G>(qmin_r);
    if (rot) {
        if (n2min == 0x7fffffff) return false;  // no readable point: the pixel waits
        qmin_r = aL2 * (double)n2min;
    } else if (!(qmin_r < INFINITY)) {
        return false;
    }
    const double e_r = exp(-(aL2 * (double)(l * l) - qmin_r));  // used by lanes l <= R
    if (c >= 0.0) {  // smart order: confidence over the whole ball, shifted by its q_min
        double e_all = 0.0, qmin_all = 0.0;  // rotated ball: q_min over the ball is 0 (n = 0)
        if (rot) {
            if (l <= R) e_all = exp(-(aL2 * (double)(l * l)));
        } else {
            double qm = INFINITY;
#pragma unroll
            for (int r = 0; r < PL; ++r) {
                const int t = l + r * G;
                if (t < T) {
                    const short2 nm = off[t];
                    const double tp = (-gy) * (double)nm.x + gx * (double)nm.y;
                    qm = fmin(qm, a * tp * tp);
                }
            }
            qmin_all = gmin<G>(qm);
        }
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int r = 0; r < PL; ++r) {
            const int t = l + r * G;
            const short2 nm = off[t];
            double w = 0.0;
            if (rot) {
                w = __shfl(e_all, t < T ? abs((int)nm.x) : 0, G) * rinv[t];
            } else if (t < T) {
                const double tp = (-gy) * (double)nm.x + gx * (double)nm.y;
                w = exp(-(a * tp * tp - qmin_all)) * rinv[t];
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
    const int C = v.C;
#pragma unroll
    for (int r = 0; r < PL; ++r) {
        const int t = l + r * G;
        const short2 nm = off[t];
        double e = __shfl(e_r, abs((int)nm.x) & (G - 1), G);  // every lane takes part
        if (lattice_here && !rot) {
            const double tp = (-gy) * (double)nm.x + gx * (double)nm.y;
            e = exp(-(a * tp * tp - qmin_r));
        }
        // neighbouring front pixels see the same side of the hole, so an offset
        // is often unreadable for every pixel of a wavefront: the branch is
        // then skipped as a whole
        if ((rmask >> r) & 1u) {
            const double w = e * rinv[t];
            Ssum += w;
            const bool ex = (exmask >> r) & 1u, ey = (eymask >> r) & 1u;
            const int i00 = base[r], i10 = i00 + (ex ? 0 : 1), i01 = i00 + (ey ? 0 : P),
                      i11 = i01 + (ex ? 0 : 1);
            float c00[4], c10[4], c01[4], c11[4];
            v.colours(i00, c00);
            v.colours(i10, c10);
            v.colours(i01, c01);
            v.colours(i11, c11);
            // channels past C carry padding or zeros: their sums are never used,
            // so three are interpolated without a test
            if constexpr (kF64Values) {
                // binary16 storage: each stored value is an exact binary64, and
                // the value is the tensor-product form sum_b sum_a bx_a by_b u
                // in FP64 (a zero fraction adds exact zeros), so the filled
                // value differs from an FP64 evaluation only by the order of
                // the weighted sum; rounding to binary16 then agrees except
                // within ~1e-16 of a rounding midpoint.  (An FP32 value here
                // could round a fill to the neighbouring binary16 number, and
                // later shells carry that step on.)
                const double fx = fxs[r], fy = fys[r];
                const double bx0 = 1.0 - fx, by0 = 1.0 - fy;
                const double b00 = bx0 * by0, b10 = fx * by0, b01 = bx0 * fy, b11 = fx * fy;
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) {
                    if (ch < 3 || C == 4) {
                        double val = b00 * (double)c00[ch];
                        val = val + b10 * (double)c10[ch];
                        val = val + b01 * (double)c01[ch];
                        val = val + b11 * (double)c11[ch];
                        acc[ch] = fma(w, val, acc[ch]);
                    }
                }
            } else {
                const float fx = fxs[r], fy = fys[r];
#pragma unroll
                for (int ch = 0; ch < 4; ++ch) {
                    if (ch < 3 || C == 4) {
                        const float top = fmaf(fx, c10[ch] - c00[ch], c00[ch]);
                        const float bot = fmaf(fx, c11[ch] - c01[ch], c01[ch]);
                        const float val = fmaf(fy, bot - top, top);
                        acc[ch] = fma(w, (double)val, acc[ch]);
                    }
                }
            }
        }
        // one offset's loads at a time: fewer registers live (no spills)
        __builtin_amdgcn_sched_barrier(0);
    }
    Ssum = gsum<G>(Ssum);
    const double inv = 1.0 / Ssum;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
        if (ch < C) out[ch] = gsum<G>(acc[ch]) * inv;
    return true;
}

}  // namespace gfk
