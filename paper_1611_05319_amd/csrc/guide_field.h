// Guide field of Guidefill (arXiv 1611.05319, Sec. 3.2) on the device: for
// every inpaint pixel x, the spline nearest to x and
//     g(x) = g_Gamma exp(-d(x, Gamma)^2 / (2 eta^2)),
// 0 beyond the cutoff distance and on every other pixel.  A spline is a
// polyline of segments, each carrying its spline's direction; the nearest
// spline holds the nearest segment (equal distances keep the first).  The
// distances and the argmin are FP64 with no contraction, so the choice of
// spline and the cutoff test are exact; the result is rounded to binary32.
#pragma once

#include "device_common.h"

namespace gfk {

struct GuideArgs {
    const uint8_t *label;
    const float *seg;       // nseg x (x0, y0, x1, y1, gx, gy)
    const int32_t *seg_off; // B + 1
    float *guide;           // B x H x W x 2
    long long HW, NP;
    int B, H, W;
    double eta, cutoff;
};

constexpr int kGuideChunk = 1024;  // pixels a workgroup scans per step

// Each workgroup scans chunks of kGuideChunk pixels: pixels off the hole get
// 0 at once, the hole pixels are listed in LDS (one atomic per wavefront) and
// then taken densely, one per thread, over their frame's segments.
__global__ __launch_bounds__(kBlock) void guide_kernel(GuideArgs A) {
    __shared__ int s_list[kGuideChunk];
    __shared__ int s_n;
    const int tid = threadIdx.x;
    const double den = 2.0 * A.eta * A.eta;
    const double cut2 = A.cutoff * A.cutoff;
    float2 *out = reinterpret_cast<float2 *>(A.guide);
    const long long nchunk = (A.NP + kGuideChunk - 1) / kGuideChunk;
    for (long long c = blockIdx.x; c < nchunk; c += gridDim.x) {
        const long long p0 = c * kGuideChunk;
        if (tid == 0) s_n = 0;
        __syncthreads();
        for (int i = tid; i < kGuideChunk; i += kBlock) {  // uniform trip count
            const long long p = p0 + i;
            const bool hole = p < A.NP && A.label[p] == 1;
            if (p < A.NP && !hole) out[p] = make_float2(0.0f, 0.0f);
            const int slot = wave_append(hole, &s_n);
            if (hole) s_list[slot] = i;
        }
        __syncthreads();
        const int n = s_n;
        for (int e = tid; e < n; e += kBlock) {
            const long long p = p0 + s_list[e];
            const long long f = p / A.HW;
            const int q = (int)(p - f * A.HW);
            const int j = q / A.W, i = q - j * A.W;
            const int s0 = A.seg_off[f], s1 = A.seg_off[f + 1];
            double best = INFINITY;
            int arg = -1;
            for (int k = s0; k < s1; ++k) {
                const float *S = A.seg + 6ll * k;
                const double x0 = S[0], y0 = S[1];
                const double dx = (double)S[2] - x0, dy = (double)S[3] - y0;
                const double qx = (double)i - x0, qy = (double)j - y0;
                const double len2 = dx * dx + dy * dy;
                double t = 0.0;
                if (len2 > 0.0) {
                    t = (qx * dx + qy * dy) / len2;
                    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                }
                const double ex = qx - t * dx, ey = qy - t * dy;
                const double d2 = ex * ex + ey * ey;
                if (d2 < best) {
                    best = d2;
                    arg = k;
                }
            }
            float2 g = make_float2(0.0f, 0.0f);
            if (arg >= 0 && !(best > cut2)) {
                const double fct = exp(-best / den);
                g.x = (float)((double)A.seg[6ll * arg + 4] * fct);
                g.y = (float)((double)A.seg[6ll * arg + 5] * fct);
            }
            out[p] = g;
        }
        __syncthreads();
    }
}

}  // namespace gfk
