// Guide field of Guidefill (arXiv 1611.05319, Sec. 3.2) on the device: for
// every inpaint pixel x, the spline nearest to x and
//     g(x) = g_Gamma exp(-d(x, Gamma)^2 / (2 eta^2)),
// 0 beyond the cutoff distance and on every other pixel.  A spline is a
// polyline of segments, each carrying its spline's direction; the nearest
// spline holds the nearest segment (equal distances keep the first).  The
// distances and the argmin are FP64 with no contraction, so the choice of
// spline and the cutoff test are exact; the result is rounded to binary32.
//
// One workgroup per 32 x 32 tile.  A segment whose bounding box stays more
// than the cutoff away from the tile's box cannot come within the cutoff of
// any of its pixels; if it were nevertheless a pixel's nearest segment, the
// pixel would get 0 either way.  So each tile keeps only the segments near it
// (in their original order, which the tie rule needs), staged in LDS in
// batches, and its hole pixels scan those.
#pragma once

#include "device_common.h"

namespace gfk {

struct GuideArgs {
    const uint8_t *label;
    const float *seg;       // nseg x (x0, y0, x1, y1, gx, gy)
    const int32_t *seg_off; // B + 1
    float *guide;           // B x H x W x 2
    long long HW;
    int B, H, W;
    int tiles_x, tiles_y;
    double eta, cutoff;
};

constexpr int kGuideTile = 32;                          // tile edge (pixels)
constexpr int kGuideSlots = kGuideTile * kGuideTile / kBlock;  // pixels per thread
constexpr int kGuideBatch = 1024;                       // segments staged per batch

__global__ __launch_bounds__(kBlock) void guide_kernel(GuideArgs A) {
    __shared__ int s_pix[kGuideTile * kGuideTile];
    __shared__ float s_seg[kGuideBatch * 6];
    __shared__ int s_idx[kGuideBatch];
    __shared__ int s_wave[kBlock / 64];
    __shared__ int s_n, s_kept;
    const int tid = threadIdx.x;
    const int per_frame = A.tiles_x * A.tiles_y;
    const int f = (int)blockIdx.x / per_frame;
    const int t = (int)blockIdx.x - f * per_frame;
    const int x0 = (t % A.tiles_x) * kGuideTile, y0 = (t / A.tiles_x) * kGuideTile;
    const long long base = (long long)f * A.HW;
    float2 *out = reinterpret_cast<float2 *>(A.guide) + base;
    const uint8_t *lab = A.label + base;
    if (tid == 0) s_n = 0;
    __syncthreads();
    // the tile's pixels: 0 off the hole, the hole pixels listed
    for (int i = tid; i < kGuideTile * kGuideTile; i += kBlock) {  // uniform trip count
        const int x = x0 + (i & (kGuideTile - 1)), y = y0 + i / kGuideTile;
        const bool in = x < A.W && y < A.H;
        const long long q = (long long)y * A.W + x;
        const bool hole = in && lab[q] == 1;
        if (in && !hole) out[q] = make_float2(0.0f, 0.0f);
        const int slot = wave_append(hole, &s_n);
        if (hole) s_pix[slot] = i;
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0) return;

    const double cut = A.cutoff;
    const double cut2 = cut * cut;
    // the tile's box of pixel centres, widened by the cutoff and a margin
    // far above the rounding of the comparisons
    const double bx0 = x0 - cut - 1e-3, by0 = y0 - cut - 1e-3;
    const double bx1 = min(x0 + kGuideTile - 1, A.W - 1) + cut + 1e-3;
    const double by1 = min(y0 + kGuideTile - 1, A.H - 1) + cut + 1e-3;
    double best[kGuideSlots];
    int arg[kGuideSlots];
#pragma unroll
    for (int e = 0; e < kGuideSlots; ++e) {
        best[e] = INFINITY;
        arg[e] = -1;
    }
    const int s0 = A.seg_off[f], s1 = A.seg_off[f + 1];
    const int lane = tid & 63, wave = tid >> 6;
    for (int b0 = s0; b0 < s1; b0 += kGuideBatch) {
        const int b1 = min(b0 + kGuideBatch, s1);
        if (tid == 0) s_kept = 0;
        __syncthreads();
        // keep the segments near the tile, in order: per round of kBlock
        // segments, ballots give each kept one its rank
        for (int r0 = b0; r0 < b1; r0 += kBlock) {
            const int k = r0 + tid;
            bool keep = false;
            if (k < b1) {
                const float *S = A.seg + 6ll * k;
                const double sx0 = fmin((double)S[0], (double)S[2]), sx1 = fmax((double)S[0], (double)S[2]);
                const double sy0 = fmin((double)S[1], (double)S[3]), sy1 = fmax((double)S[1], (double)S[3]);
                keep = sx1 >= bx0 && sx0 <= bx1 && sy1 >= by0 && sy0 <= by1;
            }
            const unsigned long long m = __ballot(keep);
            if (lane == 0) s_wave[wave] = (int)__popcll(m);
            __syncthreads();
            int pos = s_kept;
            for (int w = 0; w < wave; ++w) pos += s_wave[w];
            pos += (int)__popcll(m & ((1ull << lane) - 1ull));
            if (keep) {
                const float *S = A.seg + 6ll * k;
#pragma unroll
                for (int c = 0; c < 6; ++c) s_seg[pos * 6 + c] = S[c];
                s_idx[pos] = k;
            }
            __syncthreads();
            if (tid == 0) {
                int tot = 0;
                for (int w = 0; w < kBlock / 64; ++w) tot += s_wave[w];
                s_kept += tot;
            }
            __syncthreads();
        }
        const int nk = s_kept;
#pragma unroll
        for (int e = 0; e < kGuideSlots; ++e) {
            const int pi = tid + e * kBlock;
            if (pi >= n) continue;
            const int i = s_pix[pi];
            const double px = (double)(x0 + (i & (kGuideTile - 1))), py = (double)(y0 + i / kGuideTile);
            for (int j = 0; j < nk; ++j) {
                const float *S = s_seg + 6 * j;
                const double sx = S[0], sy = S[1];
                const double dx = (double)S[2] - sx, dy = (double)S[3] - sy;
                const double qx = px - sx, qy = py - sy;
                const double len2 = dx * dx + dy * dy;
                double tt = 0.0;
                if (len2 > 0.0) {
                    tt = (qx * dx + qy * dy) / len2;
                    tt = tt < 0.0 ? 0.0 : (tt > 1.0 ? 1.0 : tt);
                }
                const double ex = qx - tt * dx, ey = qy - tt * dy;
                const double d2 = ex * ex + ey * ey;
                if (d2 < best[e]) {
                    best[e] = d2;
                    arg[e] = s_idx[j];
                }
            }
        }
        __syncthreads();  // the next batch overwrites the staged segments
    }
    const double den = 2.0 * A.eta * A.eta;
#pragma unroll
    for (int e = 0; e < kGuideSlots; ++e) {
        const int pi = tid + e * kBlock;
        if (pi >= n) continue;
        const int i = s_pix[pi];
        const long long q = (long long)(y0 + i / kGuideTile) * A.W + x0 + (i & (kGuideTile - 1));
        float2 g = make_float2(0.0f, 0.0f);
        if (arg[e] >= 0 && !(best[e] > cut2)) {
            const double fct = exp(-best[e] / den);
            g.x = (float)((double)A.seg[6ll * arg[e] + 4] * fct);
            g.y = (float)((double)A.seg[6ll * arg[e] + 5] * fct);
        }
        out[q] = g;
    }
}

}  // namespace gfk
