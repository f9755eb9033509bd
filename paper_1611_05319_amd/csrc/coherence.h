// Coherence-transport comparison mode (arXiv 1611.05319, Sec. 3.2,
// eqn:modStructureTensor).  Before each shell, every front pixel x (a pixel to
// fill with a known 8-neighbour) takes as its guide the coherence direction of
// the modified structure tensor of the pixels known at that shell:
//   v(p) = sum_q g_sigma(q - p) 1_K(q) u(q) / sum_q g_sigma(q - p) 1_K(q)
//   T(p) = sum_c grad v_c (x) grad v_c           (p known; central differences,
//                                                  one-sided at the frame edge
//                                                  or next to an undefined v)
//   J(x) = sum_p g_rho(p - x) 1_K(p) T(p) / sum_p g_rho(p - x) 1_K(p)
//   g(x) = tanh((lambda+ - lambda-) / Lambda) v-   (0 where J is undefined)
// with Gaussians of variance s^2 truncated to |dx|, |dy| <= floor(2 s).
//
// One workgroup per 16 x 16 (or 8 x 8) tile: tiles without a front pixel leave
// at once; the others stage colours and known flags of the tile plus a halo of
// floor(2 rho) + 1 + floor(2 sigma) pixels in LDS and compute v, T and J there
// in FP64, so no intermediate leaves the CU.  The Gaussian weight of v is the
// product of its row and column factors, so v is summed in two passes (rows,
// then columns: 2 (2 floor(2 sigma) + 1) terms a pixel instead of its square);
// J keeps the direct sum, over the front pixels only.
#pragma once

#include "device_common.h"

namespace gfk {

struct CtArgs {
    const void *img;       // B x H x W x C storage: the colours at this shell
    const uint8_t *label;  // working labels: 0 known, 1 still to fill, 2 neither
    float *guide;          // B x H x W x 2: written at the front pixels
    long long HW;
    int B, H, W, C;
    int tile, tiles_x, tiles_y;
    int rs, rr;  // window half widths floor(2 sigma), floor(2 rho)
    double sigma, rho, lambda;
};

// LDS regions of one tile: T over the tile plus rr, v one pixel wider, the
// colours another rs wider; the row sums of the smoothing over the colour
// region's rows and v's columns.  Regions whose lifetimes do not overlap
// share memory: the row sums, later T; the colours, later v.
struct CtLds {
    int RU, RV, RT;
    size_t rsum, T, u, v, w1, wr, kn, vok, total;
};

__host__ __device__ inline size_t ct_align16(size_t v) { return (v + 15) & ~(size_t)15; }

__host__ __device__ inline CtLds ct_lds(int tile, int rs, int rr, int C) {
    CtLds L;
    L.RT = tile + 2 * rr;
    L.RV = L.RT + 2;
    L.RU = L.RV + 2 * rs;
    const size_t rsum = (size_t)L.RU * L.RV * (C + 1) * sizeof(double);
    const size_t tens = (size_t)L.RT * L.RT * 3 * sizeof(double);
    const size_t cols = (size_t)L.RU * L.RU * C * sizeof(float);
    const size_t vals = (size_t)L.RV * L.RV * C * sizeof(double);
    size_t off = 0;
    L.rsum = L.T = off; off = ct_align16(off + (rsum > tens ? rsum : tens));
    L.u = L.v = off; off = ct_align16(off + (cols > vals ? cols : vals));
    L.w1 = off; off = ct_align16(off + (size_t)(2 * rs + 1) * sizeof(double));
    L.wr = off; off = ct_align16(off + (size_t)(2 * rr + 1) * (2 * rr + 1) * sizeof(double));
    L.kn = off; off = ct_align16(off + (size_t)L.RU * L.RU);
    L.vok = off; off = ct_align16(off + (size_t)L.RV * L.RV);
    L.total = off;
    return L;
}

// Coherence direction of the tensor (a, b; b, c): with h = (a - c) / 2 and
// r = sqrt(h^2 + b^2), lambda+ - lambda- = 2 r and the eigenvector of the
// smaller eigenvalue lies along (b, -(h + r)) for h >= 0, else (h - r, b).
// Its sign, which the weights do not see, is fixed so that gx > 0 (or gx == 0
// and gy > 0).
__device__ __attribute__((always_inline)) inline float2 coherence_direction(double a, double b,
                                                                            double c,
                                                                            double lambda) {
    const double h = (a - c) / 2.0;
    const double r = sqrt(h * h + b * b);
    if (!(r > 0.0)) return make_float2(0.0f, 0.0f);
    double vx, vy;
    if (h >= 0.0) {
        vx = b;
        vy = -(h + r);
    } else {
        vx = h - r;
        vy = b;
    }
    const double n = sqrt(vx * vx + vy * vy);
    vx /= n;
    vy /= n;
    if (vx < 0.0 || (vx == 0.0 && vy < 0.0)) {
        vx = -vx;
        vy = -vy;
    }
    const double m = tanh(2.0 * r / lambda);
    return make_float2((float)(m * vx), (float)(m * vy));
}

template <typename TS>
__global__ __launch_bounds__(kBlock) void ct_guide_kernel(CtArgs A) {
    extern __shared__ __align__(16) unsigned char ct_smem[];
    const CtLds L = ct_lds(A.tile, A.rs, A.rr, A.C);
    const int tid = threadIdx.x;
    const int per_frame = A.tiles_x * A.tiles_y;
    const int f = (int)blockIdx.x / per_frame;
    const int t = (int)blockIdx.x - f * per_frame;
    const int x0 = (t % A.tiles_x) * A.tile, y0 = (t / A.tiles_x) * A.tile;
    const int W = A.W, H = A.H, C = A.C;
    const uint8_t *lab = A.label + (long long)f * A.HW;

    // the tile's front pixels: to fill, with a known in-frame 8-neighbour
    bool front = false;
    const int px = x0 + tid % A.tile, py = y0 + tid / A.tile;
    if (tid < A.tile * A.tile && px < W && py < H && lab[(long long)py * W + px] == 1) {
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int qx = px + dx, qy = py + dy;
                if ((dx | dy) == 0 || qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                if (lab[(long long)qy * W + qx] == 0) front = true;
            }
    }
    if (!__syncthreads_or(front ? 1 : 0)) return;

    double *v = reinterpret_cast<double *>(ct_smem + L.v);
    double *T = reinterpret_cast<double *>(ct_smem + L.T);
    double *rsum = reinterpret_cast<double *>(ct_smem + L.rsum);
    double *w1 = reinterpret_cast<double *>(ct_smem + L.w1);
    double *wr = reinterpret_cast<double *>(ct_smem + L.wr);
    float *u = reinterpret_cast<float *>(ct_smem + L.u);
    uint8_t *kn = ct_smem + L.kn;
    uint8_t *vok = ct_smem + L.vok;
    const int rs = A.rs, rr = A.rr, WS = 2 * rs + 1, WR = 2 * rr + 1;
    const int RU = L.RU, RV = L.RV, RT = L.RT;

    for (int i = tid; i < WS; i += kBlock) {
        const int d = i - rs;
        w1[i] = exp(-(double)(d * d) / (2.0 * A.sigma * A.sigma));
    }
    for (int i = tid; i < WR * WR; i += kBlock) {
        const int dx = i % WR - rr, dy = i / WR - rr;
        wr[i] = exp(-(double)(dx * dx + dy * dy) / (2.0 * A.rho * A.rho));
    }
    // colours and known flags of the u region (a pixel's label and colours
    // are loaded together, and several pixels' loads are in flight at once)
    const TS *img = static_cast<const TS *>(A.img) + (long long)f * A.HW * C;
    const int ux0 = x0 - rr - 1 - rs, uy0 = y0 - rr - 1 - rs;
#pragma unroll 4
    for (int i = tid; i < RU * RU; i += kBlock) {
        const int gx = ux0 + i % RU, gy = uy0 + i / RU;
        const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
        const long long q = in ? (long long)gy * W + gx : 0;
        float cv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) cv[c] = (float)load_px<TS>(img + q * C + min(c, C - 1));
        const bool k = in && lab[q] == 0;
        kn[i] = k ? 1 : 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < C) u[i * C + c] = k ? cv[c] : 0.0f;
    }
    __syncthreads();

    // row sums of the smoothing: for every row of the colour region and every
    // column of the v region, sum_dx w(dx) 1_K u and sum_dx w(dx) 1_K
    const int RS1 = C + 1;
    for (int i = tid; i < RU * RV; i += kBlock) {
        const int ry = i / RV, lx = i - ry * RV;
        double num[4] = {0.0, 0.0, 0.0, 0.0};
        double den = 0.0;
        for (int dx = -rs; dx <= rs; ++dx) {
            const int ui = ry * RU + lx + rs + dx;
            if (!kn[ui]) continue;
            const double w = w1[dx + rs];
            den += w;
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < C) num[c] += w * (double)u[ui * C + c];
        }
        double *o = rsum + (size_t)i * RS1;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < C) o[c] = num[c];
        o[C] = den;
    }
    __syncthreads();
    // v over the v region: the column sums of the row sums (the v pixel (lx, ly)
    // is centred on colour row ly + rs)
    for (int i = tid; i < RV * RV; i += kBlock) {
        const int ly = i / RV, lx = i - ly * RV;
        double num[4] = {0.0, 0.0, 0.0, 0.0};
        double den = 0.0;
        for (int dy = -rs; dy <= rs; ++dy) {
            const double w = w1[dy + rs];
            const double *r = rsum + ((size_t)(ly + rs + dy) * RV + lx) * RS1;
            den += w * r[C];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c < C) num[c] += w * r[c];
        }
        vok[i] = den > 0.0 ? 1 : 0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c < C) v[i * C + c] = den > 0.0 ? num[c] / den : 0.0;
    }
    __syncthreads();

    // T over the T region, at known pixels (v-index = T-index + 1 each way)
    const int tx0 = x0 - rr, ty0 = y0 - rr;
    for (int i = tid; i < RT * RT; i += kBlock) {
        const int lx = i % RT, ly = i / RT;
        const int gx = tx0 + lx, gy = ty0 + ly;
        const int vi = (ly + 1) * RV + lx + 1;
        const int ui = (ly + 1 + rs) * RU + lx + 1 + rs;
        double a = 0.0, b = 0.0, cc = 0.0;
        if (kn[ui]) {
            const bool l = gx > 0 && vok[vi - 1], r = gx < W - 1 && vok[vi + 1];
            const bool tp = gy > 0 && vok[vi - RV], bt = gy < H - 1 && vok[vi + RV];
            for (int c = 0; c < C; ++c) {
                double gxv = 0.0, gyv = 0.0;
                if (l && r) gxv = (v[(vi + 1) * C + c] - v[(vi - 1) * C + c]) / 2.0;
                else if (r) gxv = v[(vi + 1) * C + c] - v[vi * C + c];
                else if (l) gxv = v[vi * C + c] - v[(vi - 1) * C + c];
                if (tp && bt) gyv = (v[(vi + RV) * C + c] - v[(vi - RV) * C + c]) / 2.0;
                else if (bt) gyv = v[(vi + RV) * C + c] - v[vi * C + c];
                else if (tp) gyv = v[vi * C + c] - v[(vi - RV) * C + c];
                a += gxv * gxv;
                b += gxv * gyv;
                cc += gyv * gyv;
            }
        }
        T[3 * i] = a;
        T[3 * i + 1] = b;
        T[3 * i + 2] = cc;
    }
    __syncthreads();

    // J and the guide at the front pixels: the tile's front pixels are listed
    // (in the v region, which is no longer read), and each is taken by a
    // group of kJLanes lanes, every lane summing a share of the rho window's
    // rows
    constexpr int kJLanes = 8;
    int *flist = reinterpret_cast<int *>(v);
    int *fcount = flist + A.tile * A.tile;
    if (tid == 0) *fcount = 0;
    __syncthreads();
    const int slot = wave_append(front, fcount);
    if (front) flist[slot] = (py - y0) * A.tile + (px - x0);
    __syncthreads();
    const int nf = *fcount;
    const int gj = tid / kJLanes, lj = tid % kJLanes;
    for (int b0 = 0; b0 < nf; b0 += kBlock / kJLanes) {  // uniform trip count
        const int item = b0 + gj;
        double den = 0.0, a = 0.0, b = 0.0, c = 0.0;
        int lx = 0, ly = 0;
        if (item < nf) {
            lx = flist[item] % A.tile;
            ly = flist[item] / A.tile;
            for (int dy = -rr + lj; dy <= rr; dy += kJLanes)
                for (int dx = -rr; dx <= rr; ++dx) {
                    const int ti = (ly + rr + dy) * RT + lx + rr + dx;
                    const int ui = (ly + rr + dy + 1 + rs) * RU + lx + rr + dx + 1 + rs;
                    if (!kn[ui]) continue;
                    const double w = wr[(dy + rr) * WR + dx + rr];
                    den += w;
                    a += w * T[3 * ti];
                    b += w * T[3 * ti + 1];
                    c += w * T[3 * ti + 2];
                }
        }
        den = gsum<kJLanes>(den);  // every lane of the block takes part
        a = gsum<kJLanes>(a);
        b = gsum<kJLanes>(b);
        c = gsum<kJLanes>(c);
        if (item < nf && lj == 0) {
            float2 g = make_float2(0.0f, 0.0f);
            if (den > 0.0) g = coherence_direction(a / den, b / den, c / den, A.lambda);
            reinterpret_cast<float2 *>(A.guide)[(long long)f * A.HW + (long long)(y0 + ly) * W + x0 + lx] = g;
        }
    }
}

// Start of the comparison fill: working labels, shell map (-1 known, -2
// bystander or invalid label, -3 not yet filled), cleared guides; label
// values outside {0, 1, 2} are counted.
__global__ __launch_bounds__(kBlock) void ct_init_kernel(const uint8_t *label_in, uint8_t *label_w,
                                                         int32_t *shell, float *guide_w,
                                                         float *guide_used, int32_t *bad,
                                                         long long NP) {
    int nbad = 0;
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < NP;
         p += (long long)gridDim.x * kBlock) {
        const uint8_t l = label_in[p];
        nbad += l > 2 ? 1 : 0;
        const uint8_t lw = l > 2 ? 2 : l;
        label_w[p] = lw;
        shell[p] = lw == 0 ? S_READABLE : (lw == 1 ? S_UNFILLED : S_BYSTANDER);
        reinterpret_cast<float2 *>(guide_w)[p] = make_float2(0.0f, 0.0f);
        if (guide_used) reinterpret_cast<float2 *>(guide_used)[p] = make_float2(0.0f, 0.0f);
    }
    if (nbad) atomicAdd(bad, nbad);
}

// After shell k: the pixels that shell filled become known, take shell k and
// keep the guide they were filled with.
__global__ __launch_bounds__(kBlock) void ct_commit_kernel(uint8_t *label_w, const int32_t *s_step,
                                                           int32_t *shell, const float *guide_w,
                                                           float *guide_used, long long NP, int k) {
    for (long long p = blockIdx.x * (long long)kBlock + threadIdx.x; p < NP;
         p += (long long)gridDim.x * kBlock) {
        if (label_w[p] != 1 || s_step[p] != 0) continue;
        label_w[p] = 0;
        shell[p] = k;
        if (guide_used)
            reinterpret_cast<float2 *>(guide_used)[p] = reinterpret_cast<const float2 *>(guide_w)[p];
    }
}

}  // namespace gfk
