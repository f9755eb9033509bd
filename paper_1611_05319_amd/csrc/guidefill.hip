// Shell fill of Guidefill (Hocking, MacKenzie, Schoenlieb, arXiv 1611.05319)
// for MI355X (gfx950): kernels and the C ABI declared in include/guidefill.h.
//
// What runs on the device, per call:
//   prep kernel     zeroes the control words and the stats.
//   fill kernel     one cooperative persistent launch:
//     init          one bandwidth pass over the frames: copy the image (out of
//                   place), write the shell-map codes, count the hole, and
//                   (tracked form) emit the shell-0 front, i.e. hole pixels
//                   with a readable in-image 8-neighbour (Notation, active
//                   boundary; Algorithm 1 initialisation).
//     shells        k = 0, 1, ...: every pixel of the front is filled by a
//                   group of G lanes, one lane per ball offset (Sec. 3.1):
//                   FP64 ghost geometry -> readable test against the shell
//                   map -> weights (eqn:weight) -> ready (onion or
//                   eqn:confidence / eqn:ready) -> bilinear gather
//                   (eqn:bilinearDef) -> group reductions -> one store.
//                   Tracked form (Sec. 3.5): filled pixels emit their
//                   unfilled 8-neighbours, deduplicated by a compare-and-swap
//                   on the shell map, not-ready pixels carry over; emits are
//                   staged in LDS and appended with one global atomic per
//                   workgroup.  Untracked form: every pixel gets a lane each
//                   shell and tests its own membership in the active boundary;
//                   active pixels are compacted per wavefront by ballot.
//                   A grid barrier separates the shells.  Pixels filled in
//                   shell k are never read in shell k (the readable test is
//                   0 <= s < k), which is the Jacobi reading of Algorithm 1.
//     finish        leftover hole pixels become shell -3; stats.
//   backward kernel one cooperative persistent launch replaying the shells
//                   from last to first (reverse-mode derivative).
//
// FP64 throughout: the ghost offsets must be bit-identical to the reference
// (points that land on lattice lines change the readable set), so the
// rotation is evaluated as ox = n*s + m*c, oy = m*s - n*c with (c, s) =
// g/|g|, IEEE division and square root, and no contraction into FMA.

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "guidefill.h"

#pragma clang fp contract(off)

namespace {

constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts)
constexpr int kMaxOffsets = 256;   // eps <= 9: 252 offsets
constexpr int kPerLaneMax = 4;     // ball offsets handled by one lane
constexpr int kStageCap = 2048;    // LDS staging entries per workgroup per shell
constexpr int kFrameCap = 64;      // frames with LDS statistics accumulators
constexpr int kCtlWords = 64;      // control block (int32) at the start of the workspace
constexpr int kXcd = 8;            // XCDs of the MI355X; workgroups are dealt round robin

// control words
enum : int {
    CTL_BAR_COUNT = 0,
    CTL_BAR_GEN = 1,
    CTL_LIST = 2,    // [3] front-list lengths, ring indexed by shell % 3
    CTL_FILL = 5,    // [3] pixels filled in the shell
    CTL_ACTIVE = 8,  // [3] active pixels (untracked form)
    CTL_HOLE = 11,   // label-1 pixels
    CTL_LABEL_ERR = 12,
    CTL_ORDER = 13,  // entries written to order_out
};

// shell-map codes during the fill
constexpr int32_t S_READABLE = -1;
constexpr int32_t S_BYSTANDER = -2;
constexpr int32_t S_UNFILLED = -3;
constexpr int32_t S_HOLE = -4;     // in D, not on the front list
constexpr int32_t S_FRONT = -5;    // in D, on the next front list

struct FillArgs {
    const void *in;
    void *out;
    const uint8_t *label;
    const float *guide;
    int32_t *shell;
    int32_t *stats;
    int32_t *order;
    int32_t *shell_off;
    int32_t *front_hist;
    int32_t *listA;
    int32_t *listB;
    int32_t *ctl;
    long long HW;
    long long NP;  // B * H * W
    int B, H, W, C;
    int kcap;
    int tracking;
    int max_shells;
    int inplace;
    double eps;
    double a;      // mu^2 / (2 eps^2)
    double c;      // < 0 onion
    int ghost;
};

struct BwdArgs {
    const float *grad_out;
    const void *img;
    const float *guide;
    const int32_t *shell;
    const int32_t *order;
    const int32_t *shell_off;
    float *grad_img;
    float *grad_guide;
    int32_t *ctl;
    long long HW;
    long long NP;
    int B, H, W, C, K;
    int aliased;
    double eps;
    double a;
    int ghost;
};

// ---------------------------------------------------------------------------
// storage types

template <typename TS> __device__ inline double load_px(const TS *p);
template <> __device__ inline double load_px<float>(const float *p) { return (double)*p; }
template <> __device__ inline double load_px<__half>(const __half *p) {
    return (double)__half2float(*p);
}

// binary16 round to nearest even straight from binary64 (no double rounding
// through binary32): keep 11 significant bits, round on the dropped ones.
__device__ inline unsigned short f64_to_f16_bits(double v) {
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    unsigned short sign = (unsigned short)((b >> 48) & 0x8000u);
    int e = (int)((b >> 52) & 0x7ff);
    unsigned long long man = b & 0xFFFFFFFFFFFFFull;
    if (e == 0x7ff) return (unsigned short)(sign | 0x7c00u | (man ? 0x200u : 0u));
    if (e == 0) return sign;  // binary64 subnormals are far below binary16's range
    int E = e - 1023;
    if (E > 15) return (unsigned short)(sign | 0x7c00u);
    unsigned long long full = man | (1ull << 52);
    int shift;
    unsigned hexp;
    if (E >= -14) {
        shift = 42;
        hexp = (unsigned)(E + 15);
    } else {
        shift = 42 + (-14 - E);
        hexp = 0;
        if (shift > 63) return sign;
    }
    unsigned long long q = full >> shift;
    unsigned long long rem = full & ((1ull << shift) - 1);
    unsigned long long halfway = 1ull << (shift - 1);
    if (rem > halfway || (rem == halfway && (q & 1ull))) ++q;
    unsigned bits = hexp ? ((hexp << 10) + (unsigned)(q - 1024)) : (unsigned)q;
    if (bits >= 0x7c00u) bits = 0x7c00u;
    return (unsigned short)(sign | bits);
}

template <typename TS> __device__ inline void store_px(TS *p, double v);
template <> __device__ inline void store_px<float>(float *p, double v) { *p = (float)v; }
template <> __device__ inline void store_px<__half>(__half *p, double v) {
    *p = __ushort_as_half(f64_to_f16_bits(v));
}

// ---------------------------------------------------------------------------
// group (G lanes) reductions

template <int G> __device__ inline double gsum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}
template <int G> __device__ inline double gmin(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, G));
    return v;
}

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

// readable at shell k: -1 (label 0) or filled in an earlier shell
__device__ inline bool readable(int32_t s, int k) {
    return (unsigned)(s + 1) <= (unsigned)k;
}

// ---------------------------------------------------------------------------
// grid barrier (all workgroups co-resident: cooperative launch)

__device__ void grid_sync(int32_t *ctl, unsigned nblocks) {
    // Waves of a workgroup share the CU's path to L2, so a workgroup-scope
    // release plus one agent-scope release (L2 write-back) by thread 0 makes
    // the whole workgroup's stores visible; thread 0 spins with relaxed loads
    // (an acquire load would invalidate the caches on every iteration) and
    // acquires once when the generation moves.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned *cnt = (unsigned *)&ctl[CTL_BAR_COUNT];
        unsigned *gen = (unsigned *)&ctl[CTL_BAR_GEN];
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // orders the load above, too
        const unsigned prev =
            __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == nblocks - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g)
                __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__device__ inline int ld_ctl(const int32_t *ctl, int i) {
    return __hip_atomic_load(&ctl[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// logical workgroup id: consecutive logical ids share an XCD, so contiguous
// ranges of pixels / front entries stay in one L2
__device__ inline int logical_block() {
    int n = (int)gridDim.x;
    int b = (int)blockIdx.x;
    return (b % kXcd) * (n / kXcd) + b / kXcd;
}

// ball offsets {(n, m): 0 < n^2 + m^2 <= eps^2}, m ascending then n
__device__ void build_offsets(double eps, short2 *off, int *T) {
    if (threadIdx.x == 0) {
        int R = (int)floor(eps);
        int cnt = 0;
        for (int m = -R; m <= R; ++m)
            for (int n = -R; n <= R; ++n) {
                int r2 = n * n + m * m;
                if (r2 == 0 || (double)r2 > eps * eps) continue;
                if (cnt < kMaxOffsets) off[cnt] = make_short2((short)n, (short)m);
                ++cnt;
            }
        *T = cnt < kMaxOffsets ? cnt : kMaxOffsets;
    }
}

// rotated offset R(n, m), R taking (0, 1) to g/|g| (Sec. 3.1)
__device__ inline void rot_offset(bool rot, double cs, double sn, int n, int m, double &ox,
                                  double &oy) {
    if (rot) {
        double a = (double)n * sn;
        double b = (double)m * cs;
        double d = (double)m * sn;
        double e = (double)n * cs;
        ox = a + b;
        oy = d - e;
    } else {
        ox = (double)n;
        oy = (double)m;
    }
}

// bilinear support of a ghost point at offset (ox, oy) from (X, Y)
struct Support {
    int x0, x1, y0, y1;     // x1 == x0 / y1 == y0 on a lattice line
    double wx0, wx1, wy0, wy1;
    bool in_image;
};

__device__ inline Support support_of(int X, int Y, int W, int H, double ox, double oy) {
    Support s;
    double fx = floor(ox), fy = floor(oy);
    bool ex = (ox == fx), ey = (oy == fy);
    s.x0 = X + (int)fx;
    s.y0 = Y + (int)fy;
    s.x1 = s.x0 + (ex ? 0 : 1);
    s.y1 = s.y0 + (ey ? 0 : 1);
    if (ex) { s.wx0 = 1.0; s.wx1 = 0.0; } else { double f = ox - fx; s.wx0 = 1.0 - f; s.wx1 = f; }
    if (ey) { s.wy0 = 1.0; s.wy1 = 0.0; } else { double f = oy - fy; s.wy0 = 1.0 - f; s.wy1 = f; }
    s.in_image = s.x0 >= 0 && s.y0 >= 0 && s.x1 < W && s.y1 < H;
    return s;
}

// ---------------------------------------------------------------------------
// one pixel of the front, G lanes (group-uniform call)

template <typename TS, int G>
__device__ bool fill_pixel(const FillArgs &A, const short2 *off, int T, long long gidx, int k,
                           int l) {
    const long long f = gidx / A.HW;
    const int p = (int)(gidx - f * A.HW);
    const int Y = p / A.W, X = p - Y * A.W;
    const int32_t *S = A.shell + f * A.HW;
    const float2 gv = reinterpret_cast<const float2 *>(A.guide)[gidx];
    const double gx = (double)gv.x, gy = (double)gv.y;
    const bool rot = A.ghost && (gx != 0.0 || gy != 0.0);
    double cs = 0.0, sn = 0.0;
    if (rot) {
        double L = sqrt(gx * gx + gy * gy);
        cs = gx / L;
        sn = gy / L;
    }
    // pass 1: readable set and exponents
    double q[kPerLaneMax];
    unsigned rmask = 0;
    double qmin_r = INFINITY, qmin_all = INFINITY;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        q[r] = INFINITY;
        int t = l + r * G;
        if (t < T) {
            short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            Support s = support_of(X, Y, A.W, A.H, ox, oy);
            bool rd = false;
            if (s.in_image) {
                int32_t a0 = S[s.y0 * A.W + s.x0], a1 = S[s.y0 * A.W + s.x1];
                int32_t a2 = S[s.y1 * A.W + s.x0], a3 = S[s.y1 * A.W + s.x1];
                rd = ((int)readable(a0, k) & (int)readable(a1, k) & (int)readable(a2, k) & (int)readable(a3, k)) != 0;
            }
            double tp = (-gy) * ox + gx * oy;
            q[r] = A.a * tp * tp;
            qmin_all = fmin(qmin_all, q[r]);
            if (rd) {
                rmask |= 1u << r;
                qmin_r = fmin(qmin_r, q[r]);
            }
        }
    }
    qmin_r = gmin<G>(qmin_r);
    if (!(qmin_r < INFINITY)) return false;  // no readable point: wait
    if (A.c >= 0.0) {                        // smart order (eqn:confidence, eqn:ready)
        qmin_all = gmin<G>(qmin_all);
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int r = 0; r < kPerLaneMax; ++r) {
            int t = l + r * G;
            if (t < T) {
                short2 nm = off[t];
                double ox, oy;
                rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
                double w = exp(-(q[r] - qmin_all)) / sqrt(ox * ox + oy * oy);
                den += w;
                if (rmask & (1u << r)) num += w;
            }
        }
        num = gsum<G>(num);
        den = gsum<G>(den);
        if (!(num / den > A.c)) return false;
    }
    // pass 2: weighted average of the readable ghost values
    const TS *U = reinterpret_cast<const TS *>(A.out) + f * A.HW * A.C;
    double Ssum = 0.0, acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    const int C = A.C;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        if (rmask & (1u << r)) {
            int t = l + r * G;
            short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            Support s = support_of(X, Y, A.W, A.H, ox, oy);
            double w = exp(-(q[r] - qmin_r)) / sqrt(ox * ox + oy * oy);
            Ssum += w;
            const TS *u00 = U + (long long)(s.y0 * A.W + s.x0) * C;
            const TS *u10 = U + (long long)(s.y0 * A.W + s.x1) * C;
            const TS *u01 = U + (long long)(s.y1 * A.W + s.x0) * C;
            const TS *u11 = U + (long long)(s.y1 * A.W + s.x1) * C;
            double b00 = s.wx0 * s.wy0, b10 = s.wx1 * s.wy0, b01 = s.wx0 * s.wy1, b11 = s.wx1 * s.wy1;
#define GF_CH(ch, acc)                                                                       \
    if (ch < C) {                                                                            \
        double v = b00 * load_px(u00 + ch) + b10 * load_px(u10 + ch) + b01 * load_px(u01 + ch) + \
                   b11 * load_px(u11 + ch);                                                  \
        acc += w * v;                                                                        \
    }
            GF_CH(0, acc0)
            GF_CH(1, acc1)
            GF_CH(2, acc2)
            GF_CH(3, acc3)
#undef GF_CH
        }
    }
    Ssum = gsum<G>(Ssum);
    acc0 = gsum<G>(acc0);
    if (C > 1) acc1 = gsum<G>(acc1);
    if (C > 2) acc2 = gsum<G>(acc2);
    if (C > 3) acc3 = gsum<G>(acc3);
    if (l == 0) {
        TS *o = reinterpret_cast<TS *>(A.out) + gidx * C;
        store_px(o + 0, acc0 / Ssum);
        if (C > 1) store_px(o + 1, acc1 / Ssum);
        if (C > 2) store_px(o + 2, acc2 / Ssum);
        if (C > 3) store_px(o + 3, acc3 / Ssum);
        A.shell[gidx] = k;
    }
    return true;
}

// ---------------------------------------------------------------------------
// LDS staging of list appends: one global atomic per workgroup per shell

struct Stage {
    int *buf;
    int *n;
};

__device__ inline void stage_push(Stage st, int v, int32_t *glist, int32_t *gcount) {
    int slot = atomicAdd(st.n, 1);
    if (slot < kStageCap) {
        st.buf[slot] = v;
    } else {  // LDS full: append directly
        int pos = atomicAdd(gcount, 1);
        glist[pos] = v;
    }
}

__device__ inline void stage_flush(Stage st, int32_t *glist, int32_t *gcount, int *s_base) {
    __syncthreads();
    int n = *st.n;
    if (n > kStageCap) n = kStageCap;
    if (threadIdx.x == 0) *s_base = n ? atomicAdd(gcount, n) : 0;
    __syncthreads();
    int base = *s_base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) glist[base + i] = st.buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *st.n = 0;
}

// ---------------------------------------------------------------------------
// the fill kernel

template <typename TS, int G>
__global__ __launch_bounds__(kBlock) void fill_kernel(FillArgs A) {
    __shared__ short2 s_off[kMaxOffsets];
    __shared__ int s_T;
    __shared__ int s_list[kStageCap];
    __shared__ int s_list_n;
    __shared__ int s_ord[kStageCap];
    __shared__ int s_ord_n;
    __shared__ int s_fill_n, s_active_n, s_hole_n, s_err_n;
    __shared__ int s_base;
    __shared__ int s_frame_fill[kFrameCap];
    __shared__ int s_frame_k[kFrameCap];
    __shared__ int s_frame_hole[kFrameCap];

    const int tid = threadIdx.x;
    const int nblk = (int)gridDim.x;
    const int lw = logical_block();
    build_offsets(A.eps, s_off, &s_T);
    if (tid == 0) {
        s_list_n = s_ord_n = s_fill_n = s_active_n = s_hole_n = s_err_n = 0;
    }
    for (int i = tid; i < kFrameCap; i += kBlock) {
        s_frame_fill[i] = 0;
        s_frame_k[i] = 0;
        s_frame_hole[i] = 0;
    }
    __syncthreads();
    const int T = s_T;
    int32_t *ctl = A.ctl;
    const int W = A.W, H = A.H;
    const bool track = A.tracking != 0;

    // ---- init: copy, shell codes, hole count, shell-0 front -----------------
    {
        const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
        if (!A.inplace) {
            // bulk copy of this block's pixel range, 16 bytes per lane where aligned
            const size_t esz = sizeof(TS) * (size_t)A.C;
            const char *src = reinterpret_cast<const char *>(A.in);
            char *dst = reinterpret_cast<char *>(A.out);
            size_t b0 = (size_t)lo * esz, b1 = (size_t)hi * esz;
            size_t v0 = (b0 + 15) & ~(size_t)15, v1 = b1 & ~(size_t)15;
            // 16-byte lanes only when both buffers share 16-byte alignment
            if (v0 > v1 || (((uintptr_t)src | (uintptr_t)dst) & 15) != 0) v0 = v1 = b0;
            for (size_t i = b0 + tid; i < v0; i += kBlock) dst[i] = src[i];
            for (size_t i = v0 + (size_t)tid * 16; i < v1; i += (size_t)kBlock * 16)
                *reinterpret_cast<uint4 *>(dst + i) = *reinterpret_cast<const uint4 *>(src + i);
            for (size_t i = (v1 > b0 ? v1 : b0) + tid; i < b1; i += kBlock) dst[i] = src[i];
        }
        Stage st{s_list, &s_list_n};
        for (long long p = lo + tid; p < hi; p += kBlock) {
            const uint8_t lab = A.label[p];
            int32_t code;
            if (lab == 0) {
                code = S_READABLE;
            } else if (lab == 1) {
                code = S_HOLE;
                const long long f = p / A.HW;
                const int q = (int)(p - f * A.HW);
                if (f < kFrameCap) atomicAdd(&s_frame_hole[f], 1);
                else atomicAdd(&A.stats[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f + 2], 1);
                atomicAdd(&s_hole_n, 1);
                if (track) {
                    const int y = q / W, x = q - y * W;
                    const uint8_t *L = A.label + f * A.HW;
                    bool act = false;
#pragma unroll
                    for (int d = 0; d < 9; ++d) {
                        int dx = d % 3 - 1, dy = d / 3 - 1;
                        int xx = x + dx, yy = y + dy;
                        if (d != 4 && xx >= 0 && xx < W && yy >= 0 && yy < H)
                            act |= (L[yy * W + xx] == 0);
                    }
                    if (act) {
                        code = S_FRONT;
                        stage_push(st, (int)p, A.listA, &ctl[CTL_LIST + 0]);
                    }
                }
            } else {
                code = S_BYSTANDER;
                if (lab != 2) atomicAdd(&s_err_n, 1);
            }
            A.shell[p] = code;
        }
        stage_flush(st, A.listA, &ctl[CTL_LIST + 0], &s_base);
        if (tid == 0) {
            if (s_hole_n) atomicAdd(&ctl[CTL_HOLE], s_hole_n);
            if (s_err_n) atomicAdd(&ctl[CTL_LABEL_ERR], s_err_n);
        }
        for (int i = tid; i < kFrameCap && i < A.B; i += kBlock)
            if (s_frame_hole[i])
                atomicAdd(&A.stats[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * i + 2], s_frame_hole[i]);
    }
    grid_sync(ctl, (unsigned)nblk);

    // ---- shells -------------------------------------------------------------
    const int total_hole = ld_ctl(ctl, CTL_HOLE);
    long long total_filled = 0;
    int K = 0, max_front = 0, trunc = 0;
    const int nG = kBlock / G;
    const int gi = tid / G;          // group within the workgroup
    const int l = tid & (G - 1);     // lane within the group
    Stage lst{s_list, &s_list_n};
    Stage ord{s_ord, &s_ord_n};
    const bool want_order = A.order != nullptr;
    int nk = ld_ctl(ctl, CTL_LIST + 0);
    for (int k = 0; total_filled < total_hole; ++k) {
        if (A.max_shells > 0 && k >= A.max_shells) break;
        if (track && nk == 0) break;
        if (lw == 0 && tid == 0) {
            ctl[CTL_LIST + (k + 2) % 3] = 0;
            ctl[CTL_FILL + (k + 1) % 3] = 0;
            ctl[CTL_ACTIVE + (k + 1) % 3] = 0;
        }
        int32_t *nxt_list = (k & 1) ? A.listA : A.listB;
        int32_t *nxt_cnt = &ctl[CTL_LIST + (k + 1) % 3];
        int my_fill = 0;
        if (track) {
            const int32_t *cur = (k & 1) ? A.listB : A.listA;
            const long long lo = (long long)nk * lw / nblk, hi = (long long)nk * (lw + 1) / nblk;
            for (long long base = lo; base < hi; base += nG) {
                const long long item = base + gi;
                if (item < hi) {
                    const long long gidx = cur[item];
                    bool ok = fill_pixel<TS, G>(A, s_off, T, gidx, k, l);
                    const long long f = gidx / A.HW;
                    const int p = (int)(gidx - f * A.HW);
                    if (ok) {
                        if (l < 8) {  // emit the unfilled 8-neighbours (dedup by CAS on the map)
                            const int d = l < 4 ? l : l + 1;
                            const int y = p / W, x = p - y * W;
                            const int xx = x + d % 3 - 1, yy = y + d / 3 - 1;
                            if (xx >= 0 && xx < W && yy >= 0 && yy < H) {
                                int32_t *sp = A.shell + f * A.HW + (long long)yy * W + xx;
                                if (*sp == S_HOLE && atomicCAS(sp, S_HOLE, S_FRONT) == S_HOLE)
                                    stage_push(lst, (int)(f * A.HW + (long long)yy * W + xx),
                                               nxt_list, nxt_cnt);
                            }
                        }
                        if (l == 0) {
                            ++my_fill;
                            if (want_order) stage_push(ord, (int)gidx, A.order, &ctl[CTL_ORDER]);
                            if (f < kFrameCap) {
                                atomicAdd(&s_frame_fill[f], 1);
                                atomicMax(&s_frame_k[f], k + 1);
                            } else {
                                int32_t *fs = A.stats + GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f;
                                atomicAdd(&fs[1], 1);
                                atomicMax(&fs[0], k + 1);
                            }
                        }
                    } else if (l == 0) {
                        stage_push(lst, (int)gidx, nxt_list, nxt_cnt);  // not ready: carry over
                    }
                }
            }
        } else {
            // one lane per pixel: test membership in the active boundary
            const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
            const int wave_base = tid & ~63;
            for (long long base = lo; base < hi; base += kBlock) {
                const long long p = base + tid;
                bool act = false;
                if (p < hi && A.shell[p] == S_HOLE) {
                    const long long f = p / A.HW;
                    const int q = (int)(p - f * A.HW);
                    const int y = q / W, x = q - y * W;
                    const int32_t *S = A.shell + f * A.HW;
#pragma unroll
                    for (int d = 0; d < 9; ++d) {
                        int xx = x + d % 3 - 1, yy = y + d / 3 - 1;
                        if (d != 4 && xx >= 0 && xx < W && yy >= 0 && yy < H)
                            act |= readable(S[yy * W + xx], k);
                    }
                }
                unsigned long long mask = __ballot(act);
                if (lane_id() == 0 && mask) atomicAdd(&s_active_n, __popcll(mask));
                const int gpw = 64 / G;                 // groups per wavefront
                const int gw = (tid & 63) / G;          // this lane's group in the wavefront
                while (mask) {
                    unsigned long long m2 = mask;
                    int mybit = -1;
                    for (int j = 0; j < gpw && m2; ++j) {
                        int b = __ffsll((long long)m2) - 1;
                        m2 &= m2 - 1;
                        if (j == gw) mybit = b;
                    }
                    mask = m2;
                    if (mybit >= 0) {
                        const long long px = base + wave_base + mybit;
                        bool ok = fill_pixel<TS, G>(A, s_off, T, px, k, l);
                        if (ok && l == 0) {
                            ++my_fill;
                            const long long f = px / A.HW;
                            if (want_order) stage_push(ord, (int)px, A.order, &ctl[CTL_ORDER]);
                            if (f < kFrameCap) {
                                atomicAdd(&s_frame_fill[f], 1);
                                atomicMax(&s_frame_k[f], k + 1);
                            } else {
                                int32_t *fs = A.stats + GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f;
                                atomicAdd(&fs[1], 1);
                                atomicMax(&fs[0], k + 1);
                            }
                        }
                    }
                }
            }
        }
        if (my_fill) atomicAdd(&s_fill_n, my_fill);
        if (track) stage_flush(lst, nxt_list, nxt_cnt, &s_base);
        if (want_order) stage_flush(ord, A.order, &ctl[CTL_ORDER], &s_base);
        __syncthreads();
        if (tid == 0) {
            if (s_fill_n) atomicAdd(&ctl[CTL_FILL + k % 3], s_fill_n);
            if (!track && s_active_n) atomicAdd(&ctl[CTL_ACTIVE + k % 3], s_active_n);
            s_fill_n = 0;
            s_active_n = 0;
        }
        grid_sync(ctl, (unsigned)nblk);
        const int filled_k = ld_ctl(ctl, CTL_FILL + k % 3);
        const int front_k = track ? nk : ld_ctl(ctl, CTL_ACTIVE + k % 3);
        if (front_k > max_front) max_front = front_k;
        if (lw == 0 && tid == 0) {
            if (A.front_hist && k < A.kcap) A.front_hist[k] = front_k;
            if (want_order) {
                if (k + 1 < A.kcap) A.shell_off[k + 1] = ld_ctl(ctl, CTL_ORDER);
                else trunc = 1;
            }
        }
        if (filled_k == 0) break;
        total_filled += filled_k;
        K = k + 1;
        nk = ld_ctl(ctl, CTL_LIST + (k + 1) % 3);
    }

    // ---- finish -------------------------------------------------------------
    if (total_filled < total_hole) {  // leftovers never became ready
        const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
        for (long long p = lo + tid; p < hi; p += kBlock) {
            int32_t s = A.shell[p];
            if (s == S_HOLE || s == S_FRONT) A.shell[p] = S_UNFILLED;
        }
    }
    __syncthreads();
    for (int i = tid; i < kFrameCap && i < A.B; i += kBlock) {
        int32_t *fs = A.stats + GF_STAT_FRAME0 + GF_STAT_PER_FRAME * i;
        if (s_frame_fill[i]) atomicAdd(&fs[1], s_frame_fill[i]);
        if (s_frame_k[i]) atomicMax(&fs[0], s_frame_k[i]);
    }
    if (lw == 0 && tid == 0) {
        A.stats[GF_STAT_SHELLS] = K;
        A.stats[GF_STAT_FILLED] = (int32_t)total_filled;
        A.stats[GF_STAT_HOLE] = total_hole;
        A.stats[GF_STAT_MAX_FRONT] = max_front;
        A.stats[GF_STAT_LABEL_ERR] = ld_ctl(ctl, CTL_LABEL_ERR);
        A.stats[GF_STAT_ORDER_TRUNC] = trunc;
    }
}

// ---------------------------------------------------------------------------
// reverse shells

template <typename TS, int G>
__device__ void bwd_pixel(const BwdArgs &A, const short2 *off, int T, long long gidx, int k,
                          int l) {
    const long long f = gidx / A.HW;
    const int p = (int)(gidx - f * A.HW);
    const int Y = p / A.W, X = p - Y * A.W;
    const int W = A.W;
    const int32_t *S = A.shell + f * A.HW;
    const float2 gv = reinterpret_cast<const float2 *>(A.guide)[gidx];
    const double gx = (double)gv.x, gy = (double)gv.y;
    const bool rot = A.ghost && (gx != 0.0 || gy != 0.0);
    double cs = 0.0, sn = 0.0, L = 1.0;
    if (rot) {
        L = sqrt(gx * gx + gy * gy);
        cs = gx / L;
        sn = gy / L;
    }
    const int C = A.C;
    const TS *U = reinterpret_cast<const TS *>(A.img) + f * A.HW * C;
    double q[kPerLaneMax];
    unsigned rmask = 0;
    double qmin = INFINITY;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        q[r] = INFINITY;
        int t = l + r * G;
        if (t < T) {
            short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            Support s = support_of(X, Y, A.W, A.H, ox, oy);
            bool rd = false;
            if (s.in_image) {
                int32_t a0 = S[s.y0 * W + s.x0], a1 = S[s.y0 * W + s.x1];
                int32_t a2 = S[s.y1 * W + s.x0], a3 = S[s.y1 * W + s.x1];
                rd = ((int)readable(a0, k) & (int)readable(a1, k) & (int)readable(a2, k) & (int)readable(a3, k)) != 0;
            }
            double tp = (-gy) * ox + gx * oy;
            q[r] = A.a * tp * tp;
            if (rd) {
                rmask |= 1u << r;
                qmin = fmin(qmin, q[r]);
            }
        }
    }
    qmin = gmin<G>(qmin);
    // weights, values and the value of x
    double w[kPerLaneMax];
    double v[kPerLaneMax][4];
    double Ssum = 0.0, u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        w[r] = 0.0;
        v[r][0] = v[r][1] = v[r][2] = v[r][3] = 0.0;
        if (rmask & (1u << r)) {
            int t = l + r * G;
            short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            Support s = support_of(X, Y, A.W, A.H, ox, oy);
            w[r] = exp(-(q[r] - qmin)) / sqrt(ox * ox + oy * oy);
            Ssum += w[r];
            double b00 = s.wx0 * s.wy0, b10 = s.wx1 * s.wy0, b01 = s.wx0 * s.wy1, b11 = s.wx1 * s.wy1;
            for (int ch = 0; ch < C && ch < 4; ++ch) {
                v[r][ch] = b00 * load_px(U + (long long)(s.y0 * W + s.x0) * C + ch) +
                           b10 * load_px(U + (long long)(s.y0 * W + s.x1) * C + ch) +
                           b01 * load_px(U + (long long)(s.y1 * W + s.x0) * C + ch) +
                           b11 * load_px(U + (long long)(s.y1 * W + s.x1) * C + ch);
                u[ch] += w[r] * v[r][ch];
            }
        }
    }
    Ssum = gsum<G>(Ssum);
    for (int ch = 0; ch < 4; ++ch)
        if (ch < C) u[ch] = gsum<G>(u[ch]) / Ssum;
    double ub[4] = {0.0, 0.0, 0.0, 0.0};
    float *GI = A.grad_img;
    for (int ch = 0; ch < C && ch < 4; ++ch) ub[ch] = (double)GI[gidx * C + ch];
    double dgx = 0.0, dgy = 0.0;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        if (rmask & (1u << r)) {
            int t = l + r * G;
            short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            Support s = support_of(X, Y, A.W, A.H, ox, oy);
            const double lam = w[r] / Ssum;
            double dox_dgx = 0.0, dox_dgy = 0.0, doy_dgx = 0.0, doy_dgy = 0.0;
            if (rot) {
                dox_dgx = sn * oy / L;
                dox_dgy = -cs * oy / L;
                doy_dgx = -sn * ox / L;
                doy_dgy = cs * ox / L;
            }
            const double tp = (-gy) * ox + gx * oy;
            const double dt_dgx = oy + (-gy) * dox_dgx + gx * doy_dgx;
            const double dt_dgy = -ox + (-gy) * dox_dgy + gx * doy_dgy;
            const double r2 = ox * ox + oy * oy;
            const double dlw_dgx = -2.0 * A.a * tp * dt_dgx - (ox * dox_dgx + oy * doy_dgx) / r2;
            const double dlw_dgy = -2.0 * A.a * tp * dt_dgy - (ox * dox_dgy + oy * doy_dgy) / r2;
            const bool ex = s.x1 == s.x0, ey = s.y1 == s.y0;
            const long long i00 = f * A.HW + (long long)s.y0 * W + s.x0;
            const long long i10 = f * A.HW + (long long)s.y0 * W + s.x1;
            const long long i01 = f * A.HW + (long long)s.y1 * W + s.x0;
            const long long i11 = f * A.HW + (long long)s.y1 * W + s.x1;
            for (int ch = 0; ch < C && ch < 4; ++ch) {
                const double u00 = load_px(U + (long long)(s.y0 * W + s.x0) * C + ch);
                const double u10 = load_px(U + (long long)(s.y0 * W + s.x1) * C + ch);
                const double u01 = load_px(U + (long long)(s.y1 * W + s.x0) * C + ch);
                const double u11 = load_px(U + (long long)(s.y1 * W + s.x1) * C + ch);
                const double vpx = ex ? 0.0 : s.wy0 * (u10 - u00) + s.wy1 * (u11 - u01);
                const double vpy = ey ? 0.0 : s.wx0 * (u01 - u00) + s.wx1 * (u11 - u10);
                const double dvx = vpx * dox_dgx + vpy * doy_dgx;
                const double dvy = vpx * dox_dgy + vpy * doy_dgy;
                dgx += ub[ch] * lam * ((v[r][ch] - u[ch]) * dlw_dgx + dvx);
                dgy += ub[ch] * lam * ((v[r][ch] - u[ch]) * dlw_dgy + dvy);
                // pass the adjoint to the bilinear support
                const double g = ub[ch] * lam;
                unsafeAtomicAdd(&GI[i00 * C + ch], (float)(g * s.wx0 * s.wy0));
                if (!ex) unsafeAtomicAdd(&GI[i10 * C + ch], (float)(g * s.wx1 * s.wy0));
                if (!ey) unsafeAtomicAdd(&GI[i01 * C + ch], (float)(g * s.wx0 * s.wy1));
                if (!ex && !ey) unsafeAtomicAdd(&GI[i11 * C + ch], (float)(g * s.wx1 * s.wy1));
            }
        }
    }
    dgx = gsum<G>(dgx);
    dgy = gsum<G>(dgy);
    if (l == 0) {
        A.grad_guide[gidx * 2 + 0] = (float)dgx;
        A.grad_guide[gidx * 2 + 1] = (float)dgy;
        for (int ch = 0; ch < C; ++ch) GI[gidx * C + ch] = 0.0f;  // input of a filled pixel is unused
    }
}

template <typename TS, int G>
__global__ __launch_bounds__(kBlock) void bwd_kernel(BwdArgs A) {
    __shared__ short2 s_off[kMaxOffsets];
    __shared__ int s_T;
    const int tid = threadIdx.x;
    const int nblk = (int)gridDim.x;
    const int lw = logical_block();
    build_offsets(A.eps, s_off, &s_T);
    __syncthreads();
    const int T = s_T;
    {
        // grad_img = grad_out, grad_guide = 0
        const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
        if (!A.aliased)
            for (long long i = lo * A.C + tid; i < hi * A.C; i += kBlock) A.grad_img[i] = A.grad_out[i];
        for (long long i = lo * 2 + tid; i < hi * 2; i += kBlock) A.grad_guide[i] = 0.0f;
    }
    grid_sync(A.ctl, (unsigned)nblk);
    const int nG = kBlock / G;
    const int gi = tid / G, l = tid & (G - 1);
    for (int k = A.K - 1; k >= 0; --k) {
        const long long b0 = A.shell_off[k], b1 = A.shell_off[k + 1];
        const long long n = b1 - b0;
        const long long lo = b0 + n * lw / nblk, hi = b0 + n * (lw + 1) / nblk;
        for (long long base = lo; base < hi; base += nG) {
            const long long item = base + gi;
            if (item < hi) bwd_pixel<TS, G>(A, s_off, T, (long long)A.order[item], k, l);
        }
        grid_sync(A.ctl, (unsigned)nblk);
    }
}

__global__ void prep_kernel(int32_t *ctl, int32_t *stats, int nstats, int32_t *shell_off) {
    for (int i = threadIdx.x; i < kCtlWords; i += blockDim.x) ctl[i] = 0;
    if (stats)
        for (int i = threadIdx.x; i < nstats; i += blockDim.x) stats[i] = 0;
    if (threadIdx.x == 0 && shell_off) shell_off[0] = 0;
}

// ---------------------------------------------------------------------------
// host side

thread_local char g_last_error[512] = "";

void set_err(const char *what, hipError_t e) {
    snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorString(e));
}

int count_offsets(double eps) {
    int R = (int)floor(eps);
    int cnt = 0;
    for (int m = -R; m <= R; ++m)
        for (int n = -R; n <= R; ++n) {
            int r2 = n * n + m * m;
            if (r2 == 0 || (double)r2 > eps * eps) continue;
            ++cnt;
        }
    return cnt;
}

struct DevInfo {
    int cus = 0;
    bool coop = false;
};

DevInfo device_info(int dev) {
    static std::mutex mu;
    static DevInfo cache[64];
    static bool have[64] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= 0 && dev < 64 && have[dev]) return cache[dev];
    DevInfo d;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) d.cus = v;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess) d.coop = v != 0;
    if (dev >= 0 && dev < 64) {
        cache[dev] = d;
        have[dev] = true;
    }
    return d;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

gf_status validate(const gf_params *p, int B, int H, int W, int C, gf_dtype dt) {
    if (!p) return GF_EINVAL;
    if (B < 1 || H < 1 || W < 1 || C < 1 || C > 4) return GF_EINVAL;
    if (dt != GF_F32 && dt != GF_F16) return GF_EINVAL;
    if (!(p->eps >= 1.0) || !(p->eps <= 9.0) || !(p->mu > 0.0) || !isfinite(p->mu)) return GF_EINVAL;
    if (!(p->c == p->c)) return GF_EINVAL;
    if (p->max_shells < 0) return GF_EINVAL;
    if (p->group != 0 && p->group != 32 && p->group != 64) return GF_EINVAL;
    if (p->blocks_per_cu < 0 || p->blocks_per_cu > 8) return GF_EINVAL;
    long long np = (long long)B * H * W;
    if (np * C >= (1ll << 31)) return GF_EUNSUPPORTED;  // int32 pixel indices in the lists
    return GF_OK;
}

int pick_group(const gf_params *p, int T) {
    if (p->group) return p->group;
    return T <= 32 ? 32 : 64;
}

template <typename K>
gf_status launch_coop(K kernel, const void *args_ptr, int blocks_per_cu, long long work_items,
                      hipStream_t stream, int *grid_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_err("hipGetDevice", e); return GF_EDEVICE; }
    DevInfo di = device_info(dev);
    if (!di.coop || di.cus <= 0) {
        snprintf(g_last_error, sizeof g_last_error, "device %d has no cooperative launch", dev);
        return GF_EUNSUPPORTED;
    }
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(kernel),
                                                     kBlock, 0);
    if (e != hipSuccess || occ < 1) { set_err("occupancy", e); return GF_EDEVICE; }
    int per_cu = blocks_per_cu > 0 ? blocks_per_cu : 4;
    if (per_cu > occ) per_cu = occ;
    long long grid = (long long)per_cu * di.cus;
    // no more workgroups than there is work for (at least one per XCD)
    long long need = (work_items + kBlock - 1) / kBlock;
    if (need < kXcd) need = kXcd;
    if (grid > need) grid = need;
    grid = (grid / kXcd) * kXcd;
    if (grid < kXcd) grid = kXcd;
    if (grid_out) *grid_out = (int)grid;
    void *kargs[] = {const_cast<void *>(args_ptr)};
    e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kernel), dim3((unsigned)grid),
                                   dim3(kBlock), kargs, 0, stream);
    if (e != hipSuccess) { set_err("hipLaunchCooperativeKernel", e); return GF_EDEVICE; }
    return GF_OK;
}

template <typename TS>
gf_status run_fill(const FillArgs &A, int G, int blocks_per_cu, hipStream_t stream) {
    long long work = A.NP;
    if (G == 32) return launch_coop(fill_kernel<TS, 32>, &A, blocks_per_cu, work, stream, nullptr);
    return launch_coop(fill_kernel<TS, 64>, &A, blocks_per_cu, work, stream, nullptr);
}

template <typename TS>
gf_status run_bwd(const BwdArgs &A, int G, int blocks_per_cu, hipStream_t stream) {
    long long work = A.NP;
    if (G == 32) return launch_coop(bwd_kernel<TS, 32>, &A, blocks_per_cu, work, stream, nullptr);
    return launch_coop(bwd_kernel<TS, 64>, &A, blocks_per_cu, work, stream, nullptr);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int gf_version(void) { return 1; }

const char *gf_status_string(gf_status s) {
    switch (s) {
    case GF_OK: return "ok";
    case GF_EINVAL: return "invalid argument";
    case GF_EDEVICE: return "HIP device error";
    case GF_EUNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *gf_last_error(void) { return g_last_error; }

size_t gf_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p) {
    (void)C; (void)dt; (void)p;
    if (B < 1 || H < 1 || W < 1) return 0;
    size_t np = (size_t)B * H * W;
    return align256(kCtlWords * sizeof(int32_t)) + 2 * align256(np * sizeof(int32_t));
}

size_t gf_backward_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p) {
    (void)B; (void)H; (void)W; (void)C; (void)dt; (void)p;
    return align256(kCtlWords * sizeof(int32_t));
}

gf_status gf_fill_batched(const void *img_in, void *img_out, int B, int H, int W, int C,
                          gf_dtype dt, const uint8_t *label, const float *guide,
                          const gf_params *p, int32_t *shell_out, int32_t *stats,
                          int32_t *order_out, int32_t *shell_offsets, int32_t *front_hist,
                          int kcap, void *workspace, size_t ws_bytes, void *stream) {
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    if (!img_in || !img_out || !label || !guide || !shell_out || !stats || !workspace)
        return GF_EINVAL;
    if ((order_out == nullptr) != (shell_offsets == nullptr)) return GF_EINVAL;
    if ((order_out || front_hist) && kcap < 1) return GF_EINVAL;
    if (ws_bytes < gf_workspace_size(B, H, W, C, dt, p)) return GF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return GF_EINVAL;
    const int T = count_offsets(p->eps);
    const int G = pick_group(p, T);
    if (T > G * kPerLaneMax || T > kMaxOffsets) return GF_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t np = (size_t)B * H * W;
    char *ws = reinterpret_cast<char *>(workspace);
    FillArgs A;
    A.in = img_in;
    A.out = img_out;
    A.label = label;
    A.guide = guide;
    A.shell = shell_out;
    A.stats = stats;
    A.order = order_out;
    A.shell_off = shell_offsets;
    A.front_hist = front_hist;
    A.ctl = reinterpret_cast<int32_t *>(ws);
    A.listA = reinterpret_cast<int32_t *>(ws + align256(kCtlWords * sizeof(int32_t)));
    A.listB = reinterpret_cast<int32_t *>(ws + align256(kCtlWords * sizeof(int32_t)) +
                                          align256(np * sizeof(int32_t)));
    A.HW = (long long)H * W;
    A.NP = (long long)np;
    A.B = B;
    A.H = H;
    A.W = W;
    A.C = C;
    A.kcap = kcap;
    A.tracking = p->tracking ? 1 : 0;
    A.max_shells = p->max_shells;
    A.inplace = img_in == img_out;
    A.eps = p->eps;
    A.a = p->mu * p->mu / (2.0 * p->eps * p->eps);
    A.c = p->c;
    A.ghost = p->ghost ? 1 : 0;
    hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(256), 0, s, A.ctl, stats,
                       GF_STAT_FRAME0 + GF_STAT_PER_FRAME * B, shell_offsets);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_err("prep launch", e); return GF_EDEVICE; }
    if (dt == GF_F32) return run_fill<float>(A, G, p->blocks_per_cu, s);
    return run_fill<__half>(A, G, p->blocks_per_cu, s);
}

gf_status gf_fill(const void *img_in, void *img_out, int H, int W, int C, gf_dtype dt,
                  const uint8_t *label, const float *guide, const gf_params *p,
                  int32_t *shell_out, int32_t *stats, void *workspace, size_t ws_bytes,
                  void *stream) {
    return gf_fill_batched(img_in, img_out, 1, H, W, C, dt, label, guide, p, shell_out, stats,
                           nullptr, nullptr, nullptr, 0, workspace, ws_bytes, stream);
}

gf_status gf_fill_backward(const float *grad_out, const void *img_out, int B, int H, int W, int C,
                           gf_dtype dt, const uint8_t *label, const float *guide,
                           const int32_t *shell, const int32_t *order,
                           const int32_t *shell_offsets, int K, const gf_params *p,
                           float *grad_img, float *grad_guide, void *workspace,
                           size_t ws_bytes, void *stream) {
    (void)label;
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    if (!grad_out || !img_out || !guide || !shell || !order || !shell_offsets || !grad_img ||
        !grad_guide || !workspace || K < 0)
        return GF_EINVAL;
    if (ws_bytes < gf_backward_workspace_size(B, H, W, C, dt, p)) return GF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return GF_EINVAL;
    const int T = count_offsets(p->eps);
    const int G = pick_group(p, T);
    if (T > G * kPerLaneMax || T > kMaxOffsets) return GF_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    BwdArgs A;
    A.grad_out = grad_out;
    A.img = img_out;
    A.guide = guide;
    A.shell = shell;
    A.order = order;
    A.shell_off = shell_offsets;
    A.grad_img = grad_img;
    A.grad_guide = grad_guide;
    A.ctl = reinterpret_cast<int32_t *>(workspace);
    A.HW = (long long)H * W;
    A.NP = (long long)B * H * W;
    A.B = B;
    A.H = H;
    A.W = W;
    A.C = C;
    A.K = K;
    A.aliased = grad_out == grad_img;
    A.eps = p->eps;
    A.a = p->mu * p->mu / (2.0 * p->eps * p->eps);
    A.ghost = p->ghost ? 1 : 0;
    hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(256), 0, s, A.ctl, (int32_t *)nullptr, 0,
                       (int32_t *)nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) { set_err("prep launch", e); return GF_EDEVICE; }
    if (dt == GF_F32) return run_bwd<float>(A, G, p->blocks_per_cu, s);
    return run_bwd<__half>(A, G, p->blocks_per_cu, s);
}

}  // extern "C"
