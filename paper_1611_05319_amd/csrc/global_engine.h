// Global-front engine: one persistent launch, a grid barrier
// between shells, the front kept as a global list (tracked form) or found by
// one lane per pixel per shell (untracked form); Guidefill, arXiv 1611.05319,
// Algorithm 1 and Sec. 3.5.  Also the reverse-shell adjoint over a recorded
// fill order.
#pragma once

#include "fill_core.h"

namespace gfk {

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
    double a;  // mu^2 / (2 eps^2)
    double c;  // < 0 onion
    double c2; // < 0: no data term; else eqn:ready2's |g| > c2 until it leaves nothing ready
    int ghost;
    LaunchSync sync;  // launch start-up (join words and epoch)
};

// The data term of eqn:ready2: D(x) = |g(x)| > c2 (FP64, as the shell order
// depends on it)
__device__ inline bool data_term_ok(float2 g, double c2) {
    const double gx = (double)g.x, gy = (double)g.y;
    return sqrt(gx * gx + gy * gy) > c2;
}

constexpr int kItemCap = 512;  // front-list entries a workgroup stages per chunk

// LDS staging of list appends: one global atomic per workgroup per flush
struct Stage {
    int *buf;
    int *n;
    int cap;  // entries of buf
};

__device__ inline void stage_push(Stage st, int v, int32_t *glist, int32_t *gcount) {
    int slot = atomicAdd(st.n, 1);
    if (slot < st.cap) {
        st.buf[slot] = v;
    } else {  // LDS full: append directly
        int pos = atomicAdd(gcount, 1);
        glist[pos] = v;
    }
}

__device__ inline void stage_flush(Stage st, int32_t *glist, int32_t *gcount, int *s_base) {
    __syncthreads();
    int n = *st.n;
    if (n > st.cap) n = st.cap;
    if (threadIdx.x == 0) *s_base = n ? atomicAdd(gcount, n) : 0;
    __syncthreads();
    const int base = *s_base;
    for (int i = threadIdx.x; i < n; i += blockDim.x) glist[base + i] = st.buf[i];
    __syncthreads();
    if (threadIdx.x == 0) *st.n = 0;
}

// bulk copy of bytes [b0, b1) with 16-byte lanes where both buffers allow,
// four lanes in flight per thread
__device__ inline void copy_range(const char *src, char *dst, size_t b0, size_t b1) {
    const int tid = threadIdx.x, nt = blockDim.x;
    size_t v0 = (b0 + 15) & ~(size_t)15, v1 = b1 & ~(size_t)15;
    if (v0 > v1 || (((uintptr_t)src | (uintptr_t)dst) & 15) != 0) v0 = v1 = b0;
    for (size_t i = b0 + tid; i < v0; i += nt) dst[i] = src[i];
    const size_t step = (size_t)nt * 16;
    size_t i = v0 + (size_t)tid * 16;
    for (; i + 3 * step < v1; i += 4 * step) {
        const uint4 a = *reinterpret_cast<const uint4 *>(src + i);
        const uint4 b = *reinterpret_cast<const uint4 *>(src + i + step);
        const uint4 c = *reinterpret_cast<const uint4 *>(src + i + 2 * step);
        const uint4 d = *reinterpret_cast<const uint4 *>(src + i + 3 * step);
        *reinterpret_cast<uint4 *>(dst + i) = a;
        *reinterpret_cast<uint4 *>(dst + i + step) = b;
        *reinterpret_cast<uint4 *>(dst + i + 2 * step) = c;
        *reinterpret_cast<uint4 *>(dst + i + 3 * step) = d;
    }
    for (; i < v1; i += step)
        *reinterpret_cast<uint4 *>(dst + i) = *reinterpret_cast<const uint4 *>(src + i);
    for (size_t j = (v1 > b0 ? v1 : b0) + tid; j < b1; j += nt) dst[j] = src[j];
}

// Per-group neighbourhood window in LDS: the (2D + 1)^2 pixels around a front
// pixel, D = ceil(eps) (every bilinear support of its ball lies within D
// pixels in each direction), with their states and colours (4 slots per
// pixel).  The group's lanes stage it with loads along the window rows, so
// the fill's many support reads become LDS reads instead of scattered global
// gathers.  Pixels outside the frame are staged as bystanders (never
// readable), as an out-of-frame support is unreadable.
template <typename TS> __host__ __device__ inline int window_bytes(int D) {
    const int WN = (2 * D + 1) * (2 * D + 1);
    return ((WN * 4 + 15) & ~15) + ((WN * 4 * (int)sizeof(TS) + 15) & ~15);
}

template <typename TS>
__device__ inline void store_colours(TS *dst, const float c[4]);
template <> __device__ inline void store_colours<float>(float *dst, const float c[4]) {
    *reinterpret_cast<float4 *>(__builtin_assume_aligned(dst, 16)) = make_float4(c[0], c[1], c[2], c[3]);
}
template <> __device__ inline void store_colours<__half>(__half *dst, const float c[4]) {
    uint2 v;
    v.x = (unsigned)__half_as_ushort(__float2half_rn(c[0])) | ((unsigned)__half_as_ushort(__float2half_rn(c[1])) << 16);
    v.y = (unsigned)__half_as_ushort(__float2half_rn(c[2])) | ((unsigned)__half_as_ushort(__float2half_rn(c[3])) << 16);
    *reinterpret_cast<uint2 *>(__builtin_assume_aligned(dst, 8)) = v;
}

// Stage the window of pixel (X, Y) of frame f; lane l of the group takes the
// window pixels l, l + G, ...  The states are the shell map as it stands:
// another group's concurrent writes in this shell (s = k for a pixel it fills,
// the next-front mark) are unreadable at shell k whenever they are seen, so
// the readable sets do not depend on the timing.
// NU > 1: each lane's first NU window pixels are loaded with every load in
// flight at once (more registers), the rest one after another.
// Window pixels a lane of the fill loads before it stores any to LDS: more
// loads in flight per round trip against more registers held.  Measured on
// the 1080p, 4K, 64-frame and 16-frame workloads: 7 where registers allow,
// 2 for the binary16 kernel with 8 lanes, which is at its register limit.
template <typename TS, int G> __host__ __device__ constexpr int stage_unroll() {
    return sizeof(TS) == 2 && G == 8 ? 2 : 7;
}

template <typename TS, int G, int NU = 1>
__device__ inline void stage_window(const int32_t *S, const TS *U, int W, int H, int C, int X, int Y,
                                    int D, int32_t *st, TS *col, int l) {
    const int WW = 2 * D + 1, WN = WW * WW;
    int wy = 0, wx = l;
    while (wx >= WW) { wx -= WW; ++wy; }
    // window pixel (wx, wy): state and colours (channels past C repeat channel
    // C - 1, never used, so no load is conditional on C)
    auto fetch = [&](int wxx, int wyy, int32_t &s, float c[4]) {
        const int x = X - D + wxx, y = Y - D + wyy;
        s = S_BYSTANDER;
        c[0] = c[1] = c[2] = c[3] = 0.0f;
        if (x >= 0 && x < W && y >= 0 && y < H) {
            const long long q = (long long)y * W + x;
            s = S[q];
            const TS *p = U + q * C;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) c[ch] = px_f32(p[min(ch, C - 1)]);
        }
    };
    int i = l;
    if constexpr (NU > 1) {
        int32_t sv[NU];
        float cv[NU][4];
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            sv[j] = S_BYSTANDER;
            if (i + j * G < WN) fetch(wx, wy, sv[j], cv[j]);
            wx += G;
            while (wx >= WW) { wx -= WW; ++wy; }
        }
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            if (i + j * G < WN) {
                st[i + j * G] = sv[j];
                store_colours<TS>(col + (i + j * G) * 4, cv[j]);
            }
        }
        i += NU * G;
    }
    for (; i < WN; i += G) {
        int32_t sv;
        float cv[4];
        fetch(wx, wy, sv, cv);
        st[i] = sv;
        store_colours<TS>(col + i * 4, cv);
        wx += G;
        while (wx >= WW) { wx -= WW; ++wy; }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // the group's lanes read each other's stores
}

// Fill front pixel gidx at shell k from its staged window; lane 0 stores the
// colour and the shell.  Returns ready.
template <typename TS, int G>
__device__ __attribute__((always_inline)) bool global_fill_pixel(const FillArgs &A, const short2 *off, const double *rinv, int T,
                                  long long gidx, float2 gv, int k, int l, int D, const int32_t *st,
                                  const TS *col) {
    const int WW = 2 * D + 1;
    LdsView<TS> v{st, col, WW, WW, A.C, 4};
    double val[4];
    if (!fill_core<TS, G>(v, D, D, (double)gv.x, (double)gv.y, A.ghost != 0, off, rinv, T,
                          (int)floor(A.eps), k, l, A.a, A.c, val))
        return false;
    if (l == 0) {
        TS *o = reinterpret_cast<TS *>(A.out) + gidx * A.C;
        for (int ch = 0; ch < A.C; ++ch) o[ch] = to_storage<TS>(val[ch]);
        A.shell[gidx] = k;
    }
    return true;
}

// three workgroups of 256 per CU (12 wavefronts): the register budget that
// keeps the fill free of spills while holding more front pixels in flight;
// two for 16-lane groups, whose 5 offsets per lane need more registers
template <typename TS, int G>
__global__ __launch_bounds__(kBlock, G == 16 ? 2 : 3) void fill_kernel(FillArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];  // one neighbourhood window per group
    __shared__ short2 s_off[kMaxOffsets];
    __shared__ double s_rinv[kMaxOffsets];
    __shared__ int s_T;
    __shared__ int s_list[kStageCap];
    __shared__ int s_list_n;
    __shared__ int s_ord[kStageCap];
    __shared__ int s_ord_n;
    __shared__ int s_fill_n, s_active_n, s_hole_n, s_err_n;
    __shared__ int s_base;
    __shared__ int s_item[kItemCap];    // this shell's list entries of the workgroup
    __shared__ float2 s_gd[kItemCap];   // and their guides
    __shared__ int s_frame_fill[kFrameCap];
    __shared__ int s_frame_k[kFrameCap];
    __shared__ int s_frame_hole[kFrameCap];

    const int tid = threadIdx.x;
    GridInfo grid;
    if (!launch_start(A.ctl, A.sync, grid, A.stats, 8 + 4 * A.B, A.front_hist, A.front_hist ? A.kcap : 0,
                      A.shell_off, A.shell_off ? 1 : 0))
        return;  // joined after the poll closed
    const int nblk = grid.n, lw = grid.lw, xcd = grid.x;
    build_offsets(A.eps, s_off, s_rinv, &s_T);
    if (tid == 0) s_list_n = s_ord_n = s_fill_n = s_active_n = s_hole_n = s_err_n = 0;
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
    GF_T0();
    GF_RT_DECL(rt_stage);
    GF_RT_DECL(rt_fill);
    GF_RT_DECL(rt_emit);

    // ---- init: copy, shell codes, hole count, shell-0 front ----------------
    {
        const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
        if (!A.inplace) {
            const size_t esz = sizeof(TS) * (size_t)A.C;
            copy_range(reinterpret_cast<const char *>(A.in), reinterpret_cast<char *>(A.out),
                       (size_t)lo * esz, (size_t)hi * esz);
        }
        Stage st{s_list, &s_list_n, kStageCap};
        const uint8_t *__restrict__ Lab = A.label;
        int32_t *__restrict__ Sh = A.shell;
        auto code_of = [&](long long p, uint8_t lab) -> int32_t {
            if (lab == 0) return S_READABLE;
            if (lab != 1) {
                if (lab != 2) atomicAdd(&s_err_n, 1);
                return S_BYSTANDER;
            }
            const long long f = p / A.HW;
            const int q = (int)(p - f * A.HW);
            if (f < kFrameCap) atomicAdd(&s_frame_hole[f], 1);
            else atomicAdd(&A.stats[8 + 4 * f + 2], 1);
            atomicAdd(&s_hole_n, 1);
            if (!track) return S_HOLE;
            const int y = q / W, x = q - y * W;
            const uint8_t *L = Lab + f * A.HW;
            bool act = false;
#pragma unroll
            for (int d = 0; d < 9; ++d) {
                const int xx = x + d % 3 - 1, yy = y + d / 3 - 1;
                if (d != 4 && xx >= 0 && xx < W && yy >= 0 && yy < H) act |= (L[yy * W + xx] == 0);
            }
            if (!act) return S_HOLE;
            stage_push(st, (int)p, A.listA, &ctl[G_LIST + 0]);
            return S_FRONT;
        };
        // 16 pixels per thread and step where the label and shell buffers allow
        // vector accesses and rows hold whole groups (W a multiple of 16): one
        // label load covers a group; a group with hole pixels finds its shell-0
        // front from bit masks of the readable pixels in its row segment and the
        // segments above and below (x - 1 .. x + 16), with no per-pixel loads
        long long v0 = hi, v1 = hi;
        if ((((uintptr_t)Lab | (uintptr_t)Sh) & 15) == 0 && (W & 15) == 0) {
            v0 = (lo + 15) & ~15ll;
            v1 = hi & ~15ll;
            if (v0 > v1) v0 = v1 = hi;
        }
        for (long long p = lo + tid; p < v0; p += kBlock) Sh[p] = code_of(p, Lab[p]);
        // readable pixels (label 0) of the 18 pixels x0 - 1 .. x0 + 16 of a row
        // segment, bit k for pixel x0 - 1 + k
        auto readable18 = [&](const uint8_t *row, int x0) -> uint32_t {
            const uint4 v = *reinterpret_cast<const uint4 *>(row);
            const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
            uint32_t m = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) m |= (((wd[j >> 2] >> (8 * (j & 3))) & 0xffu) == 0u ? 2u : 0u) << j;
            if (x0 > 0 && row[-1] == 0) m |= 1u;
            if (x0 + 16 < W && row[16] == 0) m |= 1u << 17;
            return m;
        };
#pragma unroll 2
        for (long long g = v0 + 16ll * tid; g < v1; g += 16ll * kBlock) {
            const uint4 lv = *reinterpret_cast<const uint4 *>(Lab + g);
            int4 *dst = reinterpret_cast<int4 *>(Sh + g);
            if ((lv.x | lv.y | lv.z | lv.w) == 0u) {
                const int4 r = make_int4(S_READABLE, S_READABLE, S_READABLE, S_READABLE);
                dst[0] = r;
                dst[1] = r;
                dst[2] = r;
                dst[3] = r;
                continue;
            }
            const uint32_t wd[4] = {lv.x, lv.y, lv.z, lv.w};
            uint32_t hole = 0, err = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t b = (wd[j >> 2] >> (8 * (j & 3))) & 0xffu;
                hole |= (b == 1u ? 1u : 0u) << j;
                err |= (b > 2u ? 1u : 0u) << j;
            }
            uint32_t front = 0;
            if (hole) {
                const long long f = g / A.HW;
                const int q = (int)(g - f * A.HW);
                const int y = q / W, x0 = q - y * W;
                const int nh = __popc(hole);
                if (f < kFrameCap) atomicAdd(&s_frame_hole[f], nh);
                else atomicAdd(&A.stats[8 + 4 * f + 2], nh);
                atomicAdd(&s_hole_n, nh);
                if (track) {
                    const uint32_t c = readable18(Lab + g, x0);
                    const uint32_t u = y > 0 ? readable18(Lab + g - W, x0) : 0u;
                    const uint32_t d = y + 1 < H ? readable18(Lab + g + W, x0) : 0u;
                    const uint32_t vert = u | d;  // pixel j: bits j, j + 1, j + 2 above and below
                    const uint32_t act = vert | (vert >> 1) | (vert >> 2) | c | (c >> 2);
                    front = hole & act & 0xffffu;
                    const int nf = __popc(front);
                    if (nf) {  // one reservation for the group's front pixels
                        const int slot = atomicAdd(st.n, nf);
                        const int inl = max(0, min(nf, st.cap - slot));
                        const int gpos = inl < nf ? atomicAdd(&ctl[G_LIST + 0], nf - inl) : 0;
                        int j = 0;
                        for (uint32_t m = front; m; m &= m - 1u, ++j) {
                            const int px = (int)(g + __ffs(m) - 1);
                            if (j < inl) st.buf[slot + j] = px;
                            else A.listA[gpos + (j - inl)] = px;
                        }
                    }
                }
            }
            if (err) atomicAdd(&s_err_n, __popc(err));
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                int32_t c4[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int jj = 4 * q4 + j;
                    const uint32_t b = (wd[q4] >> (8 * j)) & 0xffu;
                    c4[j] = b == 0u ? S_READABLE
                            : b == 1u ? (((front >> jj) & 1u) ? S_FRONT : S_HOLE)
                                      : S_BYSTANDER;
                }
                dst[q4] = make_int4(c4[0], c4[1], c4[2], c4[3]);
            }
        }
        for (long long p = v1 + tid; p < hi; p += kBlock) Sh[p] = code_of(p, Lab[p]);
        stage_flush(st, A.listA, &ctl[G_LIST + 0], &s_base);
        if (tid == 0) {
            if (s_hole_n) atomicAdd(&ctl[xw(xcd, XF_HOLE)], s_hole_n);
            if (s_err_n) atomicAdd(&ctl[xw(xcd, XF_ERR)], s_err_n);
        }
        for (int i = tid; i < kFrameCap && i < A.B; i += kBlock)
            if (s_frame_hole[i]) atomicAdd(&A.stats[8 + 4 * i + 2], s_frame_hole[i]);
    }
    GF_TACC(0);
    grid_sync(ctl, grid);
    GF_TACC(3);

    // ---- shells -------------------------------------------------------------
    const int total_hole = sum_x(ctl, XF_HOLE);
    long long total_filled = 0;
    int K = 0, max_front = 0, trunc = 0;
    const int nG = kBlock / G;
    const int gi = tid / G;       // group within the workgroup
    const int l = tid & (G - 1);  // lane within the group
    const int D = (int)ceil(A.eps);
    const int WW = 2 * D + 1, WN = WW * WW;
    int32_t *w_st = reinterpret_cast<int32_t *>(smem + gi * window_bytes<TS>(D));
    TS *w_col = reinterpret_cast<TS *>(reinterpret_cast<unsigned char *>(w_st) + ((WN * 4 + 15) & ~15));
    Stage lst{s_list, &s_list_n, kStageCap};
    Stage ord{s_ord, &s_ord_n, kStageCap};
    const bool want_order = A.order != nullptr;
    int nk = (int)min((long long)ld_ctl(ctl, G_LIST + 0), A.NP);
    // eqn:ready2: the data term holds pixels back until a shell fills nothing;
    // that shell is then taken again without it (k stays, the iteration it
    // moves on: the lists and counter rings follow it)
    bool phase1 = A.c2 >= 0.0;
    for (int it = 0, k = 0; track || total_filled < total_hole; ++it) {
        if (A.max_shells > 0 && k >= A.max_shells) break;
        if (track && nk == 0) break;
        if (lw == 0 && tid == 0) {
            ctl[G_LIST + (it + 2) % 3] = 0;
            ctl[G_ACTIVE + (it + 1) % 3] = 0;
        }
        int32_t *nxt_list = (it & 1) ? A.listA : A.listB;
        int32_t *nxt_cnt = &ctl[G_LIST + (it + 1) % 3];
        int my_fill = 0;
        auto on_filled = [&](long long gidx) {
            ++my_fill;
            const long long f = gidx / A.HW;
            if (want_order) stage_push(ord, (int)gidx, A.order, &ctl[G_ORDER]);
            if (f < kFrameCap) {
                atomicAdd(&s_frame_fill[f], 1);
                atomicMax(&s_frame_k[f], k + 1);
            } else {
                int32_t *fs = A.stats + 8 + 4 * f;
                atomicAdd(&fs[1], 1);
                atomicMax(&fs[0], k + 1);
            }
        };
        if (track) {
            const int32_t *cur = (it & 1) ? A.listB : A.listA;
            const long long lo = (long long)nk * lw / nblk, hi = (long long)nk * (lw + 1) / nblk;
            // this workgroup's items and their guides are staged in LDS first, so
            // the rounds of groups start from LDS instead of two dependent loads
            for (long long c0 = lo; c0 < hi; c0 += kItemCap) {
                const int cn = (int)min((long long)kItemCap, hi - c0);
                __syncthreads();  // the previous chunk's readers are done
                for (int i = tid; i < cn; i += kBlock) {
                    const int gidx = cur[c0 + i];
                    s_item[i] = gidx;
                    s_gd[i] = reinterpret_cast<const float2 *>(A.guide)[gidx];
                }
                __syncthreads();
                for (int base = 0; base < cn; base += nG) {
                    const int item = base + gi;
                    GF_TCNT(8, 1);
                    if (item < cn && phase1 && !data_term_ok(s_gd[item], A.c2)) {
                        if (l == 0) stage_push(lst, s_item[item], nxt_list, nxt_cnt);  // waits
                    } else if (item < cn) {
                        const long long gidx = s_item[item];
                        const long long f = gidx / A.HW;
                        const int p = (int)(gidx - f * A.HW);
                        const int y = p / W, x = p - y * W;
                        GF_RT_BEGIN(rt_stage);
                        stage_window<TS, G, stage_unroll<TS, G>()>(A.shell + f * A.HW, reinterpret_cast<const TS *>(A.out) + f * A.HW * A.C,
                                            W, H, A.C, x, y, D, w_st, w_col, l);
                        GF_RT_END(rt_stage);
                        GF_RT_BEGIN(rt_fill);
                        const bool ok = global_fill_pixel<TS, G>(A, s_off, s_rinv, T, gidx, s_gd[item],
                                                                 k, l, D, w_st, w_col);
                        GF_RT_END(rt_fill);
                        GF_RT_BEGIN(rt_emit);
                        if (ok) {
                            if (l < 8) {  // emit the unfilled 8-neighbours (dedup by CAS on the map)
                                const int d = l < 4 ? l : l + 1;
                                const int dxn = d % 3 - 1, dyn = d / 3 - 1;
                                const int xx = x + dxn, yy = y + dyn;
                                // the window's state filters: a state only leaves S_HOLE in a shell
                                if (xx >= 0 && xx < W && yy >= 0 && yy < H &&
                                    w_st[(D + dyn) * WW + D + dxn] == S_HOLE) {
                                    int32_t *sp = A.shell + f * A.HW + (long long)yy * W + xx;
                                    if (atomicCAS(sp, S_HOLE, S_FRONT) == S_HOLE)
                                        stage_push(lst, (int)(f * A.HW + (long long)yy * W + xx),
                                                   nxt_list, nxt_cnt);
                                }
                            }
                            if (l == 0) on_filled(gidx);
                        } else if (l == 0) {
                            stage_push(lst, (int)gidx, nxt_list, nxt_cnt);  // not ready: carry over
                        }
                        GF_RT_END(rt_emit);
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
                        const int xx = x + d % 3 - 1, yy = y + d / 3 - 1;
                        if (d != 4 && xx >= 0 && xx < W && yy >= 0 && yy < H)
                            act |= readable(S[yy * W + xx], k);
                    }
                }
                unsigned long long mask = __ballot(act);
                if (lane_id() == 0 && mask) atomicAdd(&s_active_n, __popcll(mask));
                const int gpw = 64 / G;         // groups per wavefront
                const int gw = (tid & 63) / G;  // this lane's group in the wavefront
                while (mask) {
                    unsigned long long m2 = mask;
                    int mybit = -1;
                    for (int j = 0; j < gpw && m2; ++j) {
                        const int b = __ffsll((long long)m2) - 1;
                        m2 &= m2 - 1;
                        if (j == gw) mybit = b;
                    }
                    mask = m2;
                    if (mybit >= 0) {
                        const long long px = base + wave_base + mybit;
                        const float2 gv = reinterpret_cast<const float2 *>(A.guide)[px];
                        if (phase1 && !data_term_ok(gv, A.c2)) continue;  // waits (group-uniform)
                        const long long f = px / A.HW;
                        const int q = (int)(px - f * A.HW);
                        const int y = q / W, x = q - y * W;
                        stage_window<TS, G, stage_unroll<TS, G>()>(A.shell + f * A.HW, reinterpret_cast<const TS *>(A.out) + f * A.HW * A.C,
                                            W, H, A.C, x, y, D, w_st, w_col, l);
                        const bool ok = global_fill_pixel<TS, G>(A, s_off, s_rinv, T, px, gv, k, l, D,
                                                                 w_st, w_col);
                        if (ok && l == 0) on_filled(px);
                    }
                }
            }
        }
        GF_TACC(1);
        if (my_fill) atomicAdd(&s_fill_n, my_fill);
        __syncthreads();
        const int appended = s_list_n;  // every push of this shell, staged or spilled
        if (track) stage_flush(lst, nxt_list, nxt_cnt, &s_base);
        if (want_order) stage_flush(ord, A.order, &ctl[G_ORDER], &s_base);
        __syncthreads();
        const int wg_fill = s_fill_n, wg_active = s_active_n;
        __syncthreads();
        if (tid == 0) {
            if (wg_fill) atomicAdd(&ctl[G_FILLED], wg_fill);
            if (!track && wg_active) atomicAdd(&ctl[G_ACTIVE + it % 3], wg_active);
            s_fill_n = 0;
            s_active_n = 0;
        }
        GF_TACC(2);
        // the barrier carries what every workgroup needs next: the length of the
        // next front (tracked) or this shell's fills (untracked), and whether any
        // workgroup filled a pixel
        const SyncSum ss = grid_sync_sum(ctl, grid, (unsigned)(track ? appended : wg_fill),
                                         wg_fill != 0);
        GF_TACC(3);
        GF_TCNT(7, 1);
        if (lw == 0 && tid == 0) {  // statistics: one workgroup loads what only it needs
            const int front_k = track ? nk : ld_ctl(ctl, G_ACTIVE + it % 3);
            max_front = max(max_front, front_k);
            if (A.front_hist && k < A.kcap) A.front_hist[k] = front_k;
            if (want_order) {
                if (k + 1 < A.kcap) A.shell_off[k + 1] = ld_ctl(ctl, G_ORDER);
                else trunc = 1;
            }
        }
        if (ss.flags == 0) {  // nothing filled: done or stalled, or the data term's end
            if (!phase1) break;
            phase1 = false;
            if (track) nk = (int)min((long long)ss.a, A.NP);  // every pixel was carried over
            continue;
        }
        K = k + 1;
        ++k;
        if (track) nk = (int)min((long long)ss.a, A.NP);
        else total_filled += ss.a;
        GF_TACC(4);
    }

    // ---- finish -------------------------------------------------------------
    GF_RT_FLUSH(11, rt_stage);
    GF_RT_FLUSH(12, rt_fill);
    GF_RT_FLUSH(13, rt_emit);
    if (track) total_filled = ld_ctl(ctl, G_FILLED);
    if (total_filled < total_hole) {  // leftovers never became ready
        const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
        for (long long p = lo + tid; p < hi; p += kBlock) {
            const int32_t s = A.shell[p];
            if (s == S_HOLE || s == S_FRONT) A.shell[p] = S_UNFILLED;
        }
    }
    __syncthreads();
    for (int i = tid; i < kFrameCap && i < A.B; i += kBlock) {
        int32_t *fs = A.stats + 8 + 4 * i;
        if (s_frame_fill[i]) atomicAdd(&fs[1], s_frame_fill[i]);
        if (s_frame_k[i]) atomicMax(&fs[0], s_frame_k[i]);
    }
    if (lw == 0 && tid == 0) {
        A.stats[0] = K;
        A.stats[1] = (int32_t)total_filled;
        A.stats[2] = total_hole;
        A.stats[3] = max_front;
        A.stats[4] = sum_x(ctl, XF_ERR);
        A.stats[5] = trunc;
        A.stats[6] = ld_ctl(ctl, G_TIMEOUT);
        A.stats[7] = nblk;
    }
}

// ---------------------------------------------------------------------------
// reverse shells, grouped from the shell map

constexpr int kBwdBins = 2048;  // shells counted per round of the counting sort (LDS bins)

struct BwdArgs {
    const float *grad_out;
    const void *img;
    const float *guide;
    const int32_t *shell;
    float *grad_img;
    float *grad_guide;
    int32_t *ctl;
    int32_t *gcount;  // [2][kBwdBins]: pixels per shell of a sorting round (two buffers)
    int32_t *offs;    // start of shell k in order; entry K its end
    int32_t *order;   // [NP] filled pixels grouped by shell
    long long HW;
    long long NP;
    int B, H, W, C, K;  // K < 0: replay every shell of the map (max s + 1)
    int aliased;
    double eps;
    double a;
    int ghost;
    LaunchSync sync;  // launch start-up (join words and epoch)
};

// exclusive prefix sum of v over the workgroup (kBlock threads); *total gets the sum
__device__ inline int block_exclusive_scan(int v, int *s_wave, int *total) {
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wv] = x;
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int t = s_wave[w];
        before += w < wv ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

// Adjoint of one filled pixel x (shell k), one pass over its ball:
//   u = (1/S) sum_j w_j v_j,  S = sum_j w_j,  log w_j = -a t_j^2 - log|o_j|,
//   t_j = g_perp . o_j (g unnormalised, as in the weight), o_j = R(theta) n_j
//   du/dg = (1/S) sum_j w_j ((v_j - u) dlog w_j/dg + dv_j/dg)
//         = (1/S) [sum_j w_j v_j dlw_j - u sum_j w_j dlw_j + sum_j w_j dv_j]
// and the guide gradient is ubar(x) . du/dg.  ubar(x) is known before the
// pass, so each ghost value enters only as its projection e_j = ubar . v_j
// (bilinear in the corners' projections, as v_j is in their colours).  |o_j|
// does not depend on g (the rotation preserves length).  With c = cos theta,
// s = sin theta, L = |g| and p_j = c o_x + s o_y (the offset along g), the
// rotation's derivative d o / d theta = (-o_y, o_x), d theta/dg = (-s, c) / L
// give
//   dt_j/dgx = o_y - s p_j,   dt_j/dgy = c p_j - o_x,
//   de_j/dg  = (s, -c) / L * (de_j/do_x o_y - de_j/do_y o_x),
// so seven scalar sums over the ball (S, sum w e, sum w e dlw and sum w dlw
// for each component of g, and sum w (e_x o_y - e_y o_x)) carry every channel.  Pass 1 is
// the forward's geometry (exact, uncontracted: it decides the readable set);
// the sums and the scatter may contract.  A second pass scatters
// ubar(x) w_j / S times the bilinear basis values into the support pixels, in
// binary32 (the precision of the gradient buffer).
// agg: this group's LDS patch of (2D + 1)^2 floats; it lies over the group's
// window, which pass 3 no longer reads.
template <typename TS, int G>
__device__ __attribute__((always_inline)) void bwd_pixel(const BwdArgs &A, const short2 *off,
                                                         const double *rinv, int T, long long gidx,
                                                         float2 gv, int k, int l, float *agg, int D,
                                                         const int32_t *wst, const TS *wcol,
                                                         const float ubf[4]) {
    const long long f = gidx / A.HW;
    const int p = (int)(gidx - f * A.HW);
    const int Y = p / A.W, X = p - Y * A.W;
    const int W = A.W;
    const int C = A.C;
    const int WW = 2 * D + 1;  // the staged window: x at (D, D)
    float *GI = A.grad_img;
    const double gx = (double)gv.x, gy = (double)gv.y;
    const bool rot = A.ghost && (gx != 0.0 || gy != 0.0);
    double cs = 0.0, sn = 0.0, L = 1.0;
    if (rot) {
        L = sqrt(gx * gx + gy * gy);
        cs = gx / L;
        sn = gy / L;
    }
    // pass 1: geometry and readable set; the rotated offsets and the supports
    // (as window indices: every support lies inside the window; pixels outside
    // the frame are staged as bystanders, hence unreadable) are kept
    double oxs[kPerLaneMax], oys[kPerLaneMax];
    int base[kPerLaneMax];
    unsigned rmask = 0, exmask = 0, eymask = 0;
    double qmin = INFINITY;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        oxs[r] = oys[r] = 0.0;
        base[r] = 0;
        const int t = l + r * G;
        if (t < T) {
            const short2 nm = off[t];
            double ox, oy;
            rot_offset(rot, cs, sn, nm.x, nm.y, ox, oy);
            oxs[r] = ox;
            oys[r] = oy;
            const double fx0 = floor(ox), fy0 = floor(oy);
            const bool ex = (ox == fx0), ey = (oy == fy0);
            exmask |= ex ? (1u << r) : 0u;
            eymask |= ey ? (1u << r) : 0u;
            const int b = (D + (int)fy0) * WW + (D + (int)fx0);
            base[r] = b;
            const int dx = ex ? 0 : 1, dy = ey ? 0 : WW;
            const bool rd = ((int)readable(wst[b], k) & (int)readable(wst[b + dx], k) &
                             (int)readable(wst[b + dy], k) & (int)readable(wst[b + dy + dx], k)) != 0;
            if (rd) {
                const double tp = (-gy) * ox + gx * oy;
                rmask |= 1u << r;
                qmin = fmin(qmin, A.a * tp * tp);
            }
        }
    }
    qmin = gmin<G>(qmin);
    // pass 2: weights, projected values and their derivatives, all sums
    double w[kPerLaneMax];
    double Ssum = 0.0, Bx = 0.0, By = 0.0, P = 0.0, Ax = 0.0, Ay = 0.0, E = 0.0;
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        w[r] = 0.0;
        if (rmask & (1u << r)) {
#pragma clang fp contract(fast)
            const int t = l + r * G;
            const double ox = oxs[r], oy = oys[r];
            const double tp = (-gy) * ox + gx * oy;
            const double wr = exp(qmin - A.a * tp * tp) * rinv[t];
            w[r] = wr;
            Ssum += wr;
            const double pr = cs * ox + sn * oy;  // 0 without rotation
            const double m2a = -2.0 * A.a * tp;
            const double dlx = m2a * (oy - sn * pr), dly = m2a * (cs * pr - ox);
            Bx += wr * dlx;
            By += wr * dly;
            const bool ex = (exmask >> r) & 1u, ey = (eymask >> r) & 1u;
            const double wx1 = ox - floor(ox), wy1 = oy - floor(oy), wx0 = 1.0 - wx1, wy0 = 1.0 - wy1;
            const int i00 = base[r], i10 = i00 + (ex ? 0 : 1), i01 = i00 + (ey ? 0 : WW),
                      i11 = i01 + (ex ? 0 : 1);
            float c00[4], c10[4], c01[4], c11[4];
            lds_colours<TS>(wcol + i00 * 4, c00);
            lds_colours<TS>(wcol + i10 * 4, c10);
            lds_colours<TS>(wcol + i01 * 4, c01);
            lds_colours<TS>(wcol + i11 * 4, c11);
            double e00 = 0.0, e10 = 0.0, e01 = 0.0, e11 = 0.0;  // ubar . corner colour
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) {
                if (ch < C) {
                    const double u = (double)ubf[ch];
                    e00 += u * (double)c00[ch];
                    e10 += u * (double)c10[ch];
                    e01 += u * (double)c01[ch];
                    e11 += u * (double)c11[ch];
                }
            }
            const double v = wy0 * (wx0 * e00 + wx1 * e10) + wy1 * (wx0 * e01 + wx1 * e11);
            const double vpx = ex ? 0.0 : wy0 * (e10 - e00) + wy1 * (e11 - e01);
            const double vpy = ey ? 0.0 : wx0 * (e01 - e00) + wx1 * (e11 - e10);
            P += wr * v;
            Ax += wr * v * dlx;
            Ay += wr * v * dly;
            E += wr * (vpx * oy - vpy * ox);
        }
    }
    Ssum = gsum<G>(Ssum);
    const double inv = 1.0 / Ssum;
    const double u = gsum<G>(P) * inv;  // ubar(x) . u(x)
    const double Eg = rot ? gsum<G>(E) / L : 0.0;
    const double dgx = (gsum<G>(Ax) - u * gsum<G>(Bx) + sn * Eg) * inv;
    const double dgy = (gsum<G>(Ay) - u * gsum<G>(By) - cs * Eg) * inv;
    // pass 3: pass the adjoint to the bilinear supports.  Support pixel y
    // receives ubar(x) times the scalar sum over the ghost points of
    // (w_j / S) times y's bilinear basis value.  Those scalars are first
    // summed in the group's LDS patch of (2D + 1)^2 pixels around x (laid out
    // as the window), so each touched pixel takes one global atomic per
    // channel instead of one per ghost point that reads it.
    const long long fo = f * A.HW;
    // the group's lanes share a wavefront, so its window reads above are done
    // before the patch, laid over the window, is cleared
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int i = l; i < WW * WW; i += G) agg[i] = 0.0f;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int r = 0; r < kPerLaneMax; ++r) {
        if (rmask & (1u << r)) {
            const bool ex = (exmask >> r) & 1u, ey = (eymask >> r) & 1u;
            const float lam = (float)(w[r] * inv);
            const float wx1 = (float)(oxs[r] - floor(oxs[r])), wy1 = (float)(oys[r] - floor(oys[r]));
            const float wx0 = 1.0f - wx1, wy0 = 1.0f - wy1;
            const int j00 = base[r];
            const int j10 = j00 + (ex ? 0 : 1), j01 = j00 + (ey ? 0 : WW), j11 = j01 + (ex ? 0 : 1);
            atomicAdd(&agg[j00], lam * wx0 * wy0);
            if (!ex) atomicAdd(&agg[j10], lam * wx1 * wy0);
            if (!ey) atomicAdd(&agg[j01], lam * wx0 * wy1);
            if (!ex && !ey) atomicAdd(&agg[j11], lam * wx1 * wy1);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    for (int i = l; i < WW * WW; i += G) {
        const float v = agg[i];
        if (v != 0.0f) {  // a nonzero sum only lands on a support pixel, inside the frame
            const int yy = Y - D + i / WW, xx = X - D + i % WW;
            float *gp = GI + (fo + (long long)yy * W + xx) * C;
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                if (ch < C) unsafeAtomicAdd(gp + ch, ubf[ch] * v);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");  // before the next window
    if (l == 0) {
        A.grad_guide[gidx * 2 + 0] = (float)dgx;
        A.grad_guide[gidx * 2 + 1] = (float)dgy;
        for (int ch = 0; ch < C; ++ch) GI[gidx * C + ch] = 0.0f;  // input of a filled pixel is unused
    }
}

// Bytes of dynamic LDS per group of the adjoint's reverse shells: the
// neighbourhood window; the support patch (one float per window pixel) lies
// over its states once pass 2 has read the window
template <typename TS> __host__ __device__ inline int bwd_group_bytes(int D, int C) {
    (void)C;
    return window_bytes<TS>(D);
}

// Bytes of dynamic LDS the adjoint launch takes: the sorting bins, later the
// groups' windows and support patches
template <typename TS> __host__ __device__ inline size_t bwd_dyn_lds(int G, int D, int C) {
    const size_t bins = 2 * (size_t)kBwdBins * sizeof(int);
    const size_t groups = (size_t)(kBlock / G) * bwd_group_bytes<TS>(D, C);
    return bins > groups ? bins : groups;
}

// One persistent launch: (1) group the filled pixels by shell with a counting
// sort over the shell map (per-workgroup LDS histograms, one global atomic per
// workgroup and shell, prefix sums), in the same sweep that passes grad_out
// through to grad_img and clears grad_guide; (2) replay the shells from the
// last to the first, one grid barrier apart.
template <typename TS, int G>
__global__ __launch_bounds__(kBlock, 3) void bwd_kernel(BwdArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ short2 s_off[kMaxOffsets];
    __shared__ double s_rinv[kMaxOffsets];
    __shared__ int s_T;
    __shared__ int s_item[kItemCap];
    __shared__ float2 s_gd[kItemCap];
    __shared__ int s_wave[kBlock / 64];
    __shared__ int s_kend;  // max s + 1 over this workgroup's pixels
    const int tid = threadIdx.x;
    GridInfo grid;
    if (!launch_start(A.ctl, A.sync, grid, A.gcount, 2 * kBwdBins, nullptr, 0, nullptr, 0)) return;
    const int nblk = grid.n, lw = grid.lw;
    build_offsets(A.eps, s_off, s_rinv, &s_T);
    const int C = A.C;
    int *s_bin = reinterpret_cast<int *>(smem);  // per shell: count, then this workgroup's next slot
    int *s_boff = s_bin + kBwdBins;              // per shell: start in order
    GF_T0();
    // ---- counting sort of the filled pixels by shell -------------------------
    const long long lo = A.NP * lw / nblk, hi = A.NP * (lw + 1) / nblk;
    int K = A.K;
    int first = 0;  // order position of the round's first shell
    for (int c = 0;; ++c) {
        const int cb = c * kBwdBins;
        int32_t *gcnt = A.gcount + (c & 1) * kBwdBins;
        for (int i = tid; i < kBwdBins; i += kBlock) s_bin[i] = 0;
        if (tid == 0) s_kend = 0;
        __syncthreads();
        int kend = 0;
        for (long long p = lo + tid; p < hi; p += kBlock) {
            const int s = A.shell[p];
            if (c == 0) {  // gradient of the output passes through; guide gradient 0
                if (!A.aliased)
                    for (int ch = 0; ch < C; ++ch) A.grad_img[p * C + ch] = A.grad_out[p * C + ch];
                A.grad_guide[2 * p] = 0.0f;
                A.grad_guide[2 * p + 1] = 0.0f;
                kend = max(kend, s + 1);
            }
            const int kk = s - cb;
            if (s >= 0 && (K < 0 || s < K) && kk < kBwdBins && kk >= 0) atomicAdd(&s_bin[kk], 1);
        }
        if (c == 0) wave_max(kend, &s_kend);
        __syncthreads();
        for (int i = tid; i < kBwdBins; i += kBlock) {  // reserve this workgroup's slots per shell
            const int n = s_bin[i];
            s_bin[i] = n ? atomicAdd(&gcnt[i], n) : 0;
        }
        if (c == 0 && tid == 0 && s_kend > 0) atomicMax(&A.ctl[G_KEND], s_kend);
        GF_TACC(0);
        grid_sync(A.ctl, grid);
        GF_TACC(1);
        if (c == 0 && K < 0) K = ld_ctl(A.ctl, G_KEND);
        const int nb = min(kBwdBins, K - cb);  // shells of this round
        int run = first;
        for (int b0 = 0; b0 < nb; b0 += kBlock) {
            const int i = b0 + tid;
            const int v = i < nb ? ld_ctl(gcnt, i) : 0;
            int tot = 0;
            const int ex = block_exclusive_scan(v, s_wave, &tot);
            if (i < nb) {
                s_boff[i] = run + ex;
                if (lw == 0) A.offs[cb + i] = run + ex;
            }
            run += tot;
        }
        if (lw == 0 && tid == 0 && cb + kBwdBins >= K) A.offs[K > 0 ? K : 0] = run;
        __syncthreads();
        for (long long p = lo + tid; p < hi; p += kBlock) {
            const int s = A.shell[p];
            const int kk = s - cb;
            if (s >= 0 && s < K && kk >= 0 && kk < nb) {
                const int slot = atomicAdd(&s_bin[kk], 1);
                A.order[s_boff[kk] + slot] = (int)p;
            }
        }
        // the other count buffer was last read before the previous barrier
        if (lw == 0)
            for (int i = tid; i < kBwdBins; i += kBlock) A.gcount[((c + 1) & 1) * kBwdBins + i] = 0;
        first = run;
        GF_TACC(2);
        grid_sync(A.ctl, grid);
        GF_TACC(3);
        if (cb + kBwdBins >= K) break;
    }
    // ---- reverse shells ---------------------------------------------------------
    // The shell map and the forward's colours do not change here, so a shell's
    // list entries, guides and each group's first window are fetched before
    // the barrier that opens the shell; only the arriving adjoint ubar(x)
    // waits for it.
    const int T = s_T;
    const int nG = kBlock / G;
    const int gi = tid / G, l = tid & (G - 1);
    const int D = (int)ceil(A.eps);
    const int WN = (2 * D + 1) * (2 * D + 1);
    unsigned char *gbase = smem + gi * bwd_group_bytes<TS>(D, C);
    int32_t *w_st = reinterpret_cast<int32_t *>(gbase);
    TS *w_col = reinterpret_cast<TS *>(gbase + ((WN * 4 + 15) & ~15));
    float *agg = reinterpret_cast<float *>(gbase);
    // this workgroup's share [lo, hi) of shell k's entries in order
    auto share = [&](int k, long long &lo, long long &hi) {
        const long long b0 = ld_ctl(A.offs, k), n = ld_ctl(A.offs, k + 1) - b0;
        lo = b0 + n * lw / nblk;
        hi = b0 + n * (lw + 1) / nblk;
    };
    // entries [c0, c0 + cn) and their guides into LDS (between two workgroup barriers)
    auto fetch_items = [&](long long c0, int cn) {
        __syncthreads();
        for (int i = tid; i < cn; i += kBlock) {
            const int gidx = A.order[c0 + i];
            s_item[i] = gidx;
            s_gd[i] = reinterpret_cast<const float2 *>(A.guide)[gidx];
        }
        __syncthreads();
    };
    auto fetch_window = [&](long long gidx) {
        const long long f = gidx / A.HW;
        const int p = (int)(gidx - f * A.HW);
        const int y = p / A.W, x = p - y * A.W;
        stage_window<TS, G, 8>(A.shell + f * A.HW, reinterpret_cast<const TS *>(A.img) + f * A.HW * C,
                               A.W, A.H, C, x, y, D, w_st, w_col, l);
    };
    long long lo2 = 0, hi2 = 0;
    if (K > 0) {
        share(K - 1, lo2, hi2);
        const int cn = (int)min((long long)kItemCap, hi2 - lo2);
        fetch_items(lo2, cn);
        if (gi < cn) fetch_window(s_item[gi]);
    }
    for (int k = K - 1; k >= 0; --k) {
        for (long long c0 = lo2; c0 < hi2; c0 += kItemCap) {  // items and guides via LDS
            const int cn = (int)min((long long)kItemCap, hi2 - c0);
            if (c0 != lo2) fetch_items(c0, cn);
            for (int base = 0; base < cn; base += nG) {
                const int item = base + gi;
                if (item < cn) {
                    const long long gidx = s_item[item];
                    // the adjoint arriving at x is complete (every shell after k
                    // is done); its load is in flight with the window's
                    float ubf[4];
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) ubf[ch] = A.grad_img[gidx * C + min(ch, C - 1)];
                    if (c0 != lo2 || base != 0) fetch_window(gidx);
                    bwd_pixel<TS, G>(A, s_off, s_rinv, T, gidx, s_gd[item], k, l, agg, D, w_st,
                                     w_col, ubf);
                }
                GF_TCNT(6, 1);
            }
        }
        if (k > 0) {  // the next shell's first entries and windows
            share(k - 1, lo2, hi2);
            const int cn = (int)min((long long)kItemCap, hi2 - lo2);
            fetch_items(lo2, cn);
            if (gi < cn) fetch_window(s_item[gi]);
        }
        GF_TACC(4);
        grid_sync(A.ctl, grid);
        GF_TACC(5);
    }
}

}  // namespace gfk
