// Tiled engine: the shells of Algorithm 1 (Guidefill, arXiv 1611.05319) run
// S at a time inside LDS-resident tile windows, with one grid barrier per S
// shells instead of one per shell.
//
// A workgroup owns a tile of TW x TH pixels and stages a window that extends
// Hh = S * ceil(eps) pixels beyond it (states and colours in LDS).  Every
// dependency of a pixel in one shell lies within ceil(eps) pixels (the bilinear
// support of the ball and the 8-neighbourhood), so after j local shells the
// window is exact at distance >= j * ceil(eps) from its edge: the tile interior
// is exact through S shells.  Only interior results are written back; pixels
// filled in the current pass by neighbouring tiles are recomputed locally, so
// no workgroup waits for another inside a pass.
//
// Tracking (Sec. 3.5) works at two levels: inside a window a local front list
// gives lanes only to the active boundary (CAS dedup on the LDS state, carry
// over of waiting pixels); across the frame only tiles whose 3 x 3 tile
// neighbourhood filled something in the previous pass are visited (the halo
// never reaches beyond the neighbouring tiles, Hh <= min(TW, TH), and a window
// whose content did not change fills nothing again).  The untracked form
// visits every tile in every pass and gives every window pixel a lane in every
// shell.
#pragma once

#include "global_engine.h"

namespace gfk {

struct TileArgs {
    const void *in;
    void *out;
    const uint8_t *label;
    const float *guide;
    int32_t *shell;
    int32_t *stats;
    int32_t *front_hist;
    int32_t *ctl;
    int32_t *t_hole, *t_rem, *t_kmax, *t_fill, *t_mark;
    int32_t *act0, *act1;  // 8 segments of ntiles entries each
    long long HW, NP;
    int B, H, W, C, kcap;
    int TW, TH, S, Hh, WW, WH, WN;
    int tiles_x, tiles_y, ntiles;
    int max_shells, inplace, ghost, tile_track, local_track;
    double eps, a, c;
    double c2;        // < 0: no data term; else eqn:ready2's |g| > c2 until it leaves nothing ready
    LaunchSync sync;  // launch start-up (join words and epoch)
};


constexpr int kWinPerThread = 4;     // window pixels staged per thread per round trip
constexpr int kStagePerThread = 2;   // the same in the one-round staging (fewer threads)
constexpr int kMaxWindow = 8192;     // window pixels (uint16 local lists)
constexpr int kTileStageCap = 512;   // LDS staging of next-pass tiles per workgroup
constexpr int kTileStaticLds = 8192; // bytes of static LDS the tile kernel may use
constexpr int32_t kKnown = 1;        // window staging: readable from the start (not stored)

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// LDS of one window: states (int32), colours (storage type), guide (float2),
// two local front lists (uint16)
template <typename TS> __host__ __device__ inline size_t tile_lds_bytes(int WN, int C) {
    return align16((size_t)WN * 4) + align16((size_t)WN * padded_channels(C) * sizeof(TS)) +
           align16((size_t)WN * 8) + (size_t)WN * 4;
}

// NT threads per workgroup: 1024 (one large window per CU) or 256 (several
// small windows share a CU)
// Out-of-place copy of the pixels that are not in the hole (label != 1), by
// this workgroup's share [share, share + 1) of `shares`.  Pixels go in chunks
// of whole 16-byte lanes (4 binary32 RGB pixels: three lanes): a chunk with no
// hole pixel is copied lane by lane, the others pixel by pixel.  No pixel it
// writes is read back by the kernel: windows take the colours of pixels known
// from the start from the input, so the copy runs beside the first pass's
// fills.  Falls back to pixel by pixel where the buffers are not aligned.
template <typename TS>
__device__ __attribute__((always_inline)) void copy_known(const TS *__restrict__ in, TS *__restrict__ out, const uint8_t *__restrict__ label,
                           int C, long long NP, int share, int shares) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int bpp = C * (int)sizeof(TS);                   // 2 .. 16 bytes per pixel
    const int g = (bpp & 15) == 0 ? 16 : (bpp & 7) == 0 ? 8 : (bpp & 3) == 0 ? 4 : 2;  // gcd(bpp, 16)
    const int ppc = 16 / g, lanes = bpp / g;                // pixels and 16-byte lanes per chunk
    const bool vec = ((((uintptr_t)in | (uintptr_t)out) & 15) == 0) && (((uintptr_t)label & (ppc - 1)) == 0);
    const long long nch = vec ? NP / ppc : 0;
    const long long c0 = nch * share / shares, c1 = nch * (share + 1) / shares;
    for (long long c = c0 + tid; c < c1; c += nt) {
        const long long p0 = c * ppc;
        uint32_t lo = 0, hi = 0;  // the chunk's labels, one byte each
        if (ppc == 8) {
            const uint2 v = *reinterpret_cast<const uint2 *>(label + p0);
            lo = v.x;
            hi = v.y;
        } else if (ppc == 4) {
            lo = *reinterpret_cast<const uint32_t *>(label + p0);
        } else if (ppc == 2) {
            lo = *reinterpret_cast<const uint16_t *>(label + p0);
        } else {
            lo = label[p0];
        }
        // a byte equal to 1 marks a hole pixel; bytes past ppc are 0
        const uint32_t xl = lo ^ 0x01010101u, xh = hi ^ 0x01010101u;
        const uint32_t ml = ppc >= 4 ? 0xffffffffu : (ppc == 2 ? 0xffffu : 0xffu);
        const uint32_t zl = ((xl - 0x01010101u) & ~xl & 0x80808080u) & (ml & 0x80808080u);
        const uint32_t zh = ppc == 8 ? ((xh - 0x01010101u) & ~xh & 0x80808080u) : 0u;
        const uint4 *src = reinterpret_cast<const uint4 *>(in) + c * lanes;
        uint4 *dst = reinterpret_cast<uint4 *>(out) + c * lanes;
        if ((zl | zh) == 0u) {
            for (int u = 0; u < lanes; ++u) dst[u] = src[u];
        } else {
            for (int j = 0; j < ppc; ++j) {
                const uint32_t b = ((j < 4 ? lo >> (8 * j) : hi >> (8 * (j - 4)))) & 0xffu;
                if (b == 1u) continue;
                for (int ch = 0; ch < C; ++ch) out[(p0 + j) * C + ch] = in[(p0 + j) * C + ch];
            }
        }
    }
    // the pixels past the whole chunks (all of them without alignment)
    const long long rest0 = nch * ppc, nrest = NP - rest0;
    const long long r0 = rest0 + nrest * share / shares, r1 = rest0 + nrest * (share + 1) / shares;
    for (long long p = r0 + tid; p < r1; p += nt)
        if (label[p] != 1)
            for (int ch = 0; ch < C; ++ch) out[p * C + ch] = in[p * C + ch];
}

template <typename TS, int G, int NT>
__global__ __launch_bounds__(NT) void tile_kernel(TileArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ short2 s_off[kMaxOffsets];
    __shared__ double s_rinv[kMaxOffsets];
    __shared__ int s_T;
    __shared__ int s_stage[kTileStageCap];
    __shared__ int s_stage_n;
    __shared__ int s_base;
    __shared__ int s_fn[2];       // local front lengths
    __shared__ int s_filled_j;    // pixels filled in the window in the current local shell
    __shared__ int s_r[4];        // tile reductions: filled, remaining, kmax
    __shared__ int s_pass_fill, s_pass_kmax, s_hole_n, s_err_n;
    __shared__ int s_front_in[32];  // interior active pixels per local shell
    __shared__ int s_tcnt[16];      // phase A: hole pixels per tile of a batch
    __shared__ int s_seg[kXcd];     // this pass's active-tile list length per XCD
    __shared__ int s_pf[kXcd];      // the pass's fills per XCD
    __shared__ int s_km[kXcd];      // largest shell + 1 filled so far, per XCD
    __shared__ int s_nbhole[9];     // hole counts of the tile's 3 x 3 neighbourhood

    const int tid = threadIdx.x;
    const int WN = A.WN, WW = A.WW, C = A.C, W = A.W, H = A.H;
    const int CP = padded_channels(C);  // channels per window pixel
    const float rWW = 1.0f / (float)WW;  // window rows by div_small
    int32_t *st = reinterpret_cast<int32_t *>(smem);
    TS *col = reinterpret_cast<TS *>(smem + align16((size_t)WN * 4));
    float2 *gd = reinterpret_cast<float2 *>(smem + align16((size_t)WN * 4) +
                                            align16((size_t)WN * CP * sizeof(TS)));
    uint16_t *fl = reinterpret_cast<uint16_t *>(smem + align16((size_t)WN * 4) +
                                                align16((size_t)WN * CP * sizeof(TS)) +
                                                align16((size_t)WN * 8));
    int32_t *ctl = A.ctl;
    GridInfo grid;
    if (!launch_start(ctl, A.sync, grid, A.stats, 8 + 4 * A.B, A.front_hist, A.front_hist ? A.kcap : 0,
                 nullptr, 0))
        return;  // joined after the poll closed
    const int nblk = grid.n, lw = grid.lw, xcd = grid.x;
    build_offsets(A.eps, s_off, s_rinv, &s_T);
    if (tid == 0) {
        s_stage_n = 0;
        s_hole_n = 0;
        s_err_n = 0;
        s_r[0] = s_r[1] = s_r[2] = s_r[3] = 0;
    }
    __syncthreads();
    const int T = s_T;
    const int Rb = (int)floor(A.eps);
    const int tpf = A.tiles_x * A.tiles_y;  // tiles per frame
    Stage stage{s_stage, &s_stage_n, kTileStageCap};
    GF_T0();
    GF_RT_DECL(rt_fill);
    GF_RT_DECL(rt_sync);

    // ---- phase A: shell codes, per-tile hole counts, pass-0 tiles ----------
    // (the out-of-place copy of known pixels waits for the first pass)
    bool copied = A.inplace != 0;
    {
        // 16-pixel row segments per thread where tiles and rows hold whole
        // segments and the buffers allow vector accesses (one label load, four
        // stores), else single pixels, kWinPerThread per thread
        const bool vec = (A.TW & 15) == 0 && (W & 15) == 0 &&
                         ((((uintptr_t)A.label | (uintptr_t)A.shell) & 15) == 0);
        const int segs = A.TW / 16;
        const int tpx = vec ? segs * A.TH : A.TW * A.TH;  // work items per tile
        int nb = vec ? NT / tpx : (kWinPerThread * NT) / tpx;  // tiles per batch
        nb = nb < 1 ? 1 : (nb > 16 ? 16 : nb);
        for (int b0 = 0; lw + b0 * nblk < A.ntiles; b0 += nb) {
            if (tid < 16) s_tcnt[tid] = 0;
            __syncthreads();
            if (vec) {
                int ne = 0;
                for (int sb = 0; sb < nb * tpx; sb += NT) {
                    const int slot = sb + tid;
                    const int j = slot / tpx, i = slot - j * tpx;
                    const int t = lw + (b0 + j) * nblk;
                    if (j >= nb || t >= A.ntiles) continue;
                    const int f = t / tpf, rr = t - f * tpf, ty = rr / A.tiles_x, tx = rr - ty * A.tiles_x;
                    const int row = i / segs, sg = i - row * segs;
                    const int y = ty * A.TH + row, x = tx * A.TW + sg * 16;
                    if (x >= W || y >= H) continue;
                    const long long q = (long long)f * A.HW + (long long)y * W + x;
                    const uint4 lv = *reinterpret_cast<const uint4 *>(A.label + q);
                    int4 *dst = reinterpret_cast<int4 *>(A.shell + q);
                    if ((lv.x | lv.y | lv.z | lv.w) == 0u) {
                        const int4 rdb = make_int4(S_READABLE, S_READABLE, S_READABLE, S_READABLE);
                        dst[0] = rdb;
                        dst[1] = rdb;
                        dst[2] = rdb;
                        dst[3] = rdb;
                        continue;
                    }
                    const uint32_t wd[4] = {lv.x, lv.y, lv.z, lv.w};
                    int nh = 0;
#pragma unroll
                    for (int q4 = 0; q4 < 4; ++q4) {
                        int32_t c4[4];
#pragma unroll
                        for (int jj = 0; jj < 4; ++jj) {
                            const uint32_t b = (wd[q4] >> (8 * jj)) & 0xffu;
                            nh += b == 1u ? 1 : 0;
                            ne += b > 2u ? 1 : 0;
                            c4[jj] = b == 0u ? S_READABLE : b == 1u ? S_HOLE : S_BYSTANDER;
                        }
                        dst[q4] = make_int4(c4[0], c4[1], c4[2], c4[3]);
                    }
                    if (nh) atomicAdd(&s_tcnt[j], nh);
                }
                if (ne) atomicAdd(&s_err_n, ne);
            } else
            for (int sb = 0; sb < nb * tpx; sb += kWinPerThread * NT) {
            uint8_t lab[kWinPerThread];
            long long pix[kWinPerThread];
            int tj[kWinPerThread];
#pragma unroll
            for (int r = 0; r < kWinPerThread; ++r) {
                const int slot = sb + tid + r * NT;
                tj[r] = -1;
                pix[r] = 0;
                lab[r] = 0;
                const int j = slot / tpx, i = slot - j * tpx;
                const int t = lw + (b0 + j) * nblk;
                if (j < nb && t < A.ntiles) {
                    const int f = t / tpf, rr = t - f * tpf, ty = rr / A.tiles_x, tx = rr - ty * A.tiles_x;
                    const int y = ty * A.TH + i / A.TW, x = tx * A.TW + i % A.TW;
                    if (x < W && y < H) {
                        tj[r] = j;
                        pix[r] = (long long)f * A.HW + (long long)y * W + x;
                        lab[r] = A.label[pix[r]];
                    }
                }
            }
            int ne = 0;
#pragma unroll
            for (int r = 0; r < kWinPerThread; ++r) {
                if (tj[r] < 0) continue;
                int32_t code = S_BYSTANDER;
                if (lab[r] == 0) code = S_READABLE;
                else if (lab[r] == 1) { code = S_HOLE; atomicAdd(&s_tcnt[tj[r]], 1); }
                else if (lab[r] != 2) ++ne;
                A.shell[pix[r]] = code;
            }
            if (ne) atomicAdd(&s_err_n, ne);
            }
            __syncthreads();
            if (tid < nb) {
                const int t = lw + (b0 + tid) * nblk;
                if (t < A.ntiles) {
                    const int h = s_tcnt[tid];
                    A.t_hole[t] = h;
                    A.t_rem[t] = h;
                    A.t_fill[t] = 0;
                    A.t_kmax[t] = 0;
                    A.t_mark[t] = 0;
                    if (h && A.tile_track)
                        stage_push(stage, t, A.act0 + (long long)xcd * A.ntiles,
                                   &ctl[xw(xcd, XF_ACT + 0)]);
                    if (h) atomicAdd(&s_hole_n, h);
                }
            }
            __syncthreads();
        }
    }
    stage_flush(stage, A.act0 + (long long)xcd * A.ntiles, &ctl[xw(xcd, XF_ACT + 0)], &s_base);
    if (tid == 0) {
        if (s_hole_n) atomicAdd(&ctl[xw(xcd, XF_HOLE)], s_hole_n);
        if (s_err_n) atomicAdd(&ctl[xw(xcd, XF_ERR)], s_err_n);
    }
    GF_TACC(0);
    grid_sync(ctl, grid);
    GF_TACC(5);

    // ---- passes of S shells -------------------------------------------------
    // hole total and the first pass's list lengths, in one round trip
    if (tid < kXcd) {
        s_pf[tid] = ld_ctl(ctl, xw(tid, XF_HOLE));
        if (A.tile_track) s_seg[tid] = ld_ctl(ctl, xw(tid, XF_ACT + 0));
    }
    __syncthreads();
    int total_hole = 0;
#pragma unroll
    for (int x = 0; x < kXcd; ++x) total_hole += s_pf[x];
    long long total_filled = 0;
    int max_front = 0;  // kept by thread 0 of logical workgroup 0
    const int nG = NT / G;
    const int l = tid & (G - 1);
    const int wave_base = tid & ~63;
    // eqn:ready2: the data term holds pixels back until a shell fills nothing;
    // from that shell on (the next pass starts there) it is dropped, and that
    // pass visits every tile with holes left, whose windows may now change
    // although nothing near them was filled
    bool phase1 = A.c2 >= 0.0, force_all = false;
    int k0 = 0;  // first shell of the pass
    for (int p = 0; total_filled < total_hole; ++p) {
        if (A.max_shells > 0 && k0 >= A.max_shells) break;
        const int Sp = A.max_shells > 0 ? min(A.S, A.max_shells - k0) : A.S;
        if (lw == 0 && tid < kXcd) {
            ctl[xw(tid, XF_ACT + (p + 2) % 3)] = 0;
            ctl[xw(tid, XF_PFILL + (p + 1) % 3)] = 0;
        }
        if (tid == 0) {
            s_pass_fill = 0;
            s_pass_kmax = 0;
        }
        int32_t *cur_act = (p & 1) ? A.act1 : A.act0;
        int32_t *nxt_act = ((p & 1) ? A.act0 : A.act1) + (long long)xcd * A.ntiles;
        int32_t *nxt_cnt = &ctl[xw(xcd, XF_ACT + (p + 1) % 3)];
        __syncthreads();  // s_seg holds this pass's list lengths
        const bool listed = A.tile_track && !force_all;  // the pass visits the listed tiles
        int n_tiles_pass = A.ntiles;
        if (listed) {
            n_tiles_pass = 0;
#pragma unroll
            for (int x = 0; x < kXcd; ++x) n_tiles_pass += s_seg[x];
        }
        for (int v = lw; v < n_tiles_pass; v += nblk) {
            int t = v;
            if (force_all && A.tile_track && A.t_rem[t] == 0) continue;  // no hole left in the tile
            if (listed) {
                int i = v, x = 0;
                while (x < kXcd - 1 && i >= s_seg[x]) i -= s_seg[x++];
                // a listed tile whose holes are all filled finds nothing to do; its
                // remaining count is not checked first (one load fewer on the way in)
                t = cur_act[(long long)x * A.ntiles + i];
            }
            const int f = t / tpf, rr = t - f * tpf, ty = rr / A.tiles_x, tx = rr - ty * A.tiles_x;
            const int ox0 = tx * A.TW - A.Hh, oy0 = ty * A.TH - A.Hh;
            const int32_t *S = A.shell + (long long)f * A.HW;
            const TS *U = reinterpret_cast<const TS *>(A.out) + (long long)f * A.HW * C;
            const TS *Ui = reinterpret_cast<const TS *>(A.in) + (long long)f * A.HW * C;
            // hole counts of the 3 x 3 tile neighbourhood, needed by the bookkeeping
            // at the end of the tile: loaded now, beside the window
            int nbh = 0;
            if (A.tile_track && tid < 9) {
                const int nx = tx + tid % 3 - 1, ny = ty + tid / 3 - 1;
                if (nx >= 0 && nx < A.tiles_x && ny >= 0 && ny < A.tiles_y)
                    nbh = A.t_hole[f * tpf + ny * A.tiles_x + nx];
            }
            const float2 *Gd = reinterpret_cast<const float2 *>(A.guide) + (long long)f * A.HW;
            // 1. stage the window.  With 1024 threads (128 registers a lane): in
            //    two round trips, the states (readable before the pass / bystander /
            //    hole; pixels filled by neighbours during this pass count as hole),
            //    then colours of readable pixels (from the input for pixels known
            //    from the start, else from the output) and guides of hole pixels.
            //    With fewer threads there are registers for one round trip: state,
            //    guide, input colour and (after the first pass) output colour of
            //    a pixel are loaded together and the state then picks.
            if constexpr (NT >= 1024) {
                for (int base = 0; base < WN; base += kWinPerThread * NT) {
                    int32_t code[kWinPerThread];
#pragma unroll
                    for (int r = 0; r < kWinPerThread; ++r) {
                        const int i = base + tid + r * NT;
                        code[r] = S_BYSTANDER;
                        if (i < WN) {
                            const int wy = div_small(i, WW, rWW), wx = i - wy * WW;
                            const int x = ox0 + wx, y = oy0 + wy;
                            if (x >= 0 && x < W && y >= 0 && y < H) {
                                const int32_t s = S[y * W + x];
                                code[r] = s == -1                    ? kKnown
                                          : (s >= 0 && s < k0)         ? S_READABLE
                                          : (s == S_BYSTANDER || s == S_UNFILLED) ? S_BYSTANDER : S_HOLE;
                            }
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kWinPerThread; ++r) {
                        const int i = base + tid + r * NT;
                        if (i < WN) {
                            const bool known = code[r] == kKnown;
                            st[i] = known ? S_READABLE : code[r];
                            const int wy = div_small(i, WW, rWW), wx = i - wy * WW;
                            const long long q = (long long)(oy0 + wy) * W + (ox0 + wx);
                            if (known || code[r] == S_READABLE) {
                                const TS *src = known ? Ui : U;
#pragma unroll
                                for (int ch = 0; ch < 4; ++ch) col[i * CP + ch] = ch < C ? src[q * C + ch] : TS(0.0f);
                            } else if (code[r] == S_HOLE) {
                                gd[i] = Gd[q];
                            }
                        }
                    }
                }
            } else {
                for (int base = 0; base < WN; base += kStagePerThread * NT) {
                    int32_t sv[kStagePerThread];
                    TS ci[kStagePerThread][4], co[kStagePerThread][4];
                    float2 gv[kStagePerThread];
#pragma unroll
                    for (int r = 0; r < kStagePerThread; ++r) {
                        const int i = base + tid + r * NT;
                        sv[r] = S_BYSTANDER;
                        if (i < WN) {
                            const int wy = div_small(i, WW, rWW), wx = i - wy * WW;
                            const int x = ox0 + wx, y = oy0 + wy;
                            if (x >= 0 && x < W && y >= 0 && y < H) {
                                const long long q = (long long)y * W + x;
                                sv[r] = S[q];
                                gv[r] = Gd[q];
#pragma unroll
                                for (int ch = 0; ch < 4; ++ch) {
                                    ci[r][ch] = ch < C ? Ui[q * C + ch] : TS(0.0f);
                                    co[r][ch] = ch < C && k0 > 0 ? U[q * C + ch] : TS(0.0f);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int r = 0; r < kStagePerThread; ++r) {
                        const int i = base + tid + r * NT;
                        if (i < WN) {
                            const int32_t sp = sv[r];
                            const bool known = sp == -1, earlier = sp >= 0 && sp < k0;
                            const bool bys = sp == S_BYSTANDER || sp == S_UNFILLED;
                            st[i] = known || earlier ? S_READABLE : (bys ? S_BYSTANDER : S_HOLE);
                            if (known || earlier) {
#pragma unroll
                                for (int ch = 0; ch < 4; ++ch) col[i * CP + ch] = known ? ci[r][ch] : co[r][ch];
                            } else if (!bys) {
                                gd[i] = gv[r];
                            }
                        }
                    }
                }
            }
            if (tid < 9) s_nbhole[tid] = nbh;
            if (tid == 0) {
                s_fn[0] = s_fn[1] = 0;
                s_filled_j = 0;
            }
            if (tid < 32) s_front_in[tid] = 0;
            __syncthreads();
            GF_TACC(1);
            GF_TCNT(6, 1);
            LdsView<TS> view{st, col, WW, A.WH, C, CP};
            // Chebyshev distance of a window pixel from the tile interior.  A
            // result at distance d in local shell j reaches the interior no
            // earlier than shell j + d / rd, so local shell j only computes
            // pixels with d <= (S - 1 - j) rd: the band shrinks by rd a shell
            // and errors left outside it never reach the interior.
            const int rd = A.Hh / A.S;
            auto halo_dist = [&](int x, int y) {
                const int dx = max(max(A.Hh - x, x - (A.Hh + A.TW - 1)), 0);
                const int dy = max(max(A.Hh - y, y - (A.Hh + A.TH - 1)), 0);
                return max(dx, dy);
            };
            // 2. local shells; the first local front: hole pixels with a readable
            //    8-neighbour inside the band that can still reach the interior,
            //    marked and listed in one sweep
            if (A.local_track) {
                for (int base = 0; base < WN; base += NT) {  // uniform trip count
                    const int i = base + tid;
                    bool act = false;
                    if (i < WN && st[i] == S_HOLE) {
                        const int wy = div_small(i, WW, rWW), wx = i - wy * WW;
                        if (halo_dist(wx, wy) <= (Sp - 1) * rd) {
#pragma unroll
                            for (int d = 0; d < 9; ++d) {
                                const int xx = wx + d % 3 - 1, yy = wy + d / 3 - 1;
                                if (d != 4 && xx >= 0 && xx < WW && yy >= 0 && yy < A.WH)
                                    act |= (st[yy * WW + xx] == S_READABLE);
                            }
                        }
                    }
                    if (act) st[i] = S_FRONT;  // other lanes only test for S_READABLE
                    const int slot = wave_append(act, &s_fn[0]);
                    if (act) fl[slot] = (uint16_t)i;
                }
                __syncthreads();
            }
            GF_TACC(2);
            int cur = 0;
            for (int j = 0; j < Sp; ++j) {
                // fill one window pixel with a group; returns ready, sets the counters
                auto fill_one = [&](int wi, bool &filled_here, bool &interior) -> bool {
                    const int Y = div_small(wi, WW, rWW), X = wi - Y * WW;
                    const float2 gv = gd[wi];
                    double val[4];
                    // the data term of eqn:ready2 holds the pixel back (group-uniform)
                    const bool ok = !(phase1 && !data_term_ok(gv, A.c2)) &&
                                    fill_core<TS, G>(view, X, Y, (double)gv.x, (double)gv.y,
                                                     A.ghost != 0, s_off, s_rinv, T, Rb, j, l,
                                                     A.a, A.c, val);
                    if (l == 0) {
                        interior = X >= A.Hh && X < A.Hh + A.TW && Y >= A.Hh && Y < A.Hh + A.TH;
                        if (ok) {
#pragma unroll
                            for (int ch = 0; ch < 4; ++ch)
                                col[wi * CP + ch] = ch < C ? to_storage<TS>(val[ch]) : TS(0.0f);
                            st[wi] = j;
                            filled_here = true;
                        }
                    }
                    return ok;
                };
                if (A.local_track) {
                    const int n = s_fn[cur];
                    GF_TCNT(7, n);
                    GF_TCNT(8, 1);
                    const uint16_t *list = fl + cur * WN;
                    uint16_t *nlist = fl + (cur ^ 1) * WN;
                    const int band = (Sp - 1 - j) * rd;
                    constexpr int kEmit = G < 8 ? 8 / G : 1;  // neighbours per lane
                    for (int base = 0; base < n; base += nG) {
                        int lt = tid;
                        asm volatile("" : "+v"(lt));  // recompute lane values here, not hoisted
                        const int gi = lt / G, l = lt & (G - 1);
                        const int item = base + gi;
                        int push[kEmit];
#pragma unroll
                        for (int e = 0; e < kEmit; ++e) push[e] = -1;
                        bool filled_here = false, interior = false;
                        if (item < n) {
                            const int wi = list[item];
                            const int Y = div_small(wi, WW, rWW), X = wi - Y * WW;
                            if (halo_dist(X, Y) <= band) {  // else it cannot reach the interior
                                GF_RT_BEGIN(rt_fill);
                                const bool ok = fill_one(wi, filled_here, interior);
                                GF_RT_END(rt_fill);
                                if (ok) {
#pragma unroll
                                    for (int e = 0; e < kEmit; ++e) {
                                        const int dl = l + e * G;  // emit unfilled 8-neighbours, CAS dedup
                                        if (dl < 8) {
                                            const int d = dl < 4 ? dl : dl + 1;
                                            const int xx = X + d % 3 - 1, yy = Y + d / 3 - 1;
                                            if (xx >= 0 && xx < WW && yy >= 0 && yy < A.WH &&
                                                halo_dist(xx, yy) <= band - rd) {
                                                const int nw = yy * WW + xx;
                                                if (st[nw] == S_HOLE &&
                                                    atomicCAS(&st[nw], S_HOLE, S_FRONT) == S_HOLE)
                                                    push[e] = nw;
                                            }
                                        }
                                    }
                                } else if (l == 0) {
                                    push[0] = wi;  // not ready: carry over
                                }
                            }
                        }
#pragma unroll
                        for (int e = 0; e < kEmit; ++e) {
                            const int slot = wave_append(push[e] >= 0, &s_fn[cur ^ 1]);
                            if (push[e] >= 0) nlist[slot] = (uint16_t)push[e];
                        }
                        wave_count(filled_here, &s_filled_j);
                        wave_count(interior, &s_front_in[j & 31]);
                    }
                } else {
                    for (int base = 0; base < WN; base += NT) {
                        const int i = base + tid;
                        bool act = false;
                        if (i < WN && st[i] == S_HOLE) {
                            const int wy = div_small(i, WW, rWW), wx = i - wy * WW;
                            if (halo_dist(wx, wy) <= (Sp - 1 - j) * rd) {
#pragma unroll
                                for (int d = 0; d < 9; ++d) {
                                    const int xx = wx + d % 3 - 1, yy = wy + d / 3 - 1;
                                    if (d != 4 && xx >= 0 && xx < WW && yy >= 0 && yy < A.WH)
                                        act |= readable(st[yy * WW + xx], j);
                                }
                            }
                        }
                        unsigned long long mask = __ballot(act);
                        const int gpw = 64 / G, gw = (tid & 63) / G;
                        while (mask) {
                            unsigned long long m2 = mask;
                            int mybit = -1;
                            for (int q = 0; q < gpw && m2; ++q) {
                                const int b = __ffsll((long long)m2) - 1;
                                m2 &= m2 - 1;
                                if (q == gw) mybit = b;
                            }
                            mask = m2;
                            bool filled_here = false, interior = false;
                            if (mybit >= 0) fill_one(base + wave_base + mybit, filled_here, interior);
                            wave_count(filled_here, &s_filled_j);
                            wave_count(interior, &s_front_in[j & 31]);
                        }
                    }
                }
                GF_RT_BEGIN(rt_sync);
                __syncthreads();
                const int filled = s_filled_j;
                __syncthreads();
                if (tid == 0) {
                    s_filled_j = 0;
                    s_fn[cur] = 0;
                }
                cur ^= 1;
                __syncthreads();
                GF_RT_END(rt_sync);
                if (filled == 0) break;  // the window can no longer change in this pass
            }
            GF_TACC(3);
            // 3. write back the interior; tile bookkeeping
            {
                int nf = 0, nr = 0, km = 0;
                const int tw = min(A.TW, W - tx * A.TW), th = min(A.TH, H - ty * A.TH);
                TS *O = reinterpret_cast<TS *>(A.out) + (long long)f * A.HW * C;
                int32_t *Sw = A.shell + (long long)f * A.HW;
                for (int i = tid; i < tw * th; i += NT) {
                    const int ly = div_small(i, tw, 1.0f / (float)tw), lx = i - ly * tw;
                    const int wi = (ly + A.Hh) * WW + (lx + A.Hh);
                    const int v = st[wi];
                    const int y = ty * A.TH + ly, x = tx * A.TW + lx;
                    if (v >= 0) {
                        Sw[y * W + x] = k0 + v;
                        for (int ch = 0; ch < C; ++ch) O[(long long)(y * W + x) * C + ch] = col[wi * CP + ch];
                        ++nf;
                        km = max(km, k0 + v + 1);
                    } else if (v == S_HOLE || v == S_FRONT) {
                        ++nr;
                    }
                }
                wave_add(nf, &s_r[0]);
                wave_add(nr, &s_r[1]);
                wave_max(km, &s_r[2]);
                __syncthreads();
                const int tf = s_r[0];
                if (tid == 0) {
                    A.t_rem[t] = s_r[1];
                    if (tf) {  // no value returned: nothing waits for these
                        atomicAdd(&A.t_fill[t], tf);
                        atomicMax(&A.t_kmax[t], s_r[2]);
                        s_pass_fill += tf;
                        s_pass_kmax = max(s_pass_kmax, s_r[2]);
                    }
                    for (int j = 0; j < Sp && j < 32; ++j) {
                        if (!s_front_in[j]) continue;
                        atomicAdd(&ctl[G_FRONT + (p & 1) * 32 + j], s_front_in[j]);
                    }
                }
                if (tf && A.tile_track && tid < 9) {  // the 3 x 3 tile neighbourhood may change next pass
                    const int nx = tx + tid % 3 - 1, ny = ty + tid / 3 - 1;
                    if (nx >= 0 && nx < A.tiles_x && ny >= 0 && ny < A.tiles_y) {
                        const int n = f * tpf + ny * A.tiles_x + nx;
                        if (s_nbhole[tid] > 0 && atomicMax(&A.t_mark[n], p + 1) < p + 1)
                            stage_push(stage, n, nxt_act, nxt_cnt);
                    }
                }
                __syncthreads();
                if (tid == 0) s_r[0] = s_r[1] = s_r[2] = 0;
                __syncthreads();
            }
            GF_TACC(4);
        }
        if (!copied) {  // first pass: copy the known pixels, by the workgroups
            const int idle = nblk - n_tiles_pass;  // without a tile if there are enough
            if (idle > 0 && idle >= nblk / 4) {
                if (lw >= n_tiles_pass)
                    copy_known<TS>(reinterpret_cast<const TS *>(A.in), reinterpret_cast<TS *>(A.out), A.label, C,
                                   A.NP, lw - n_tiles_pass, idle);
            } else {
                copy_known<TS>(reinterpret_cast<const TS *>(A.in), reinterpret_cast<TS *>(A.out), A.label, C, A.NP,
                               lw, nblk);
            }
            copied = true;
        }
        stage_flush(stage, nxt_act, nxt_cnt, &s_base);
        if (tid == 0 && s_pass_fill) {
            atomicAdd(&ctl[xw(xcd, XF_PFILL + p % 3)], s_pass_fill);
            atomicMax(&ctl[xw(xcd, XF_KMAX)], s_pass_kmax);
        }
        GF_TACC(9);
        grid_sync(ctl, grid);
        GF_TACC(5);
        GF_TCNT(10, 1);
        // this pass's fills, the shells filled so far and the next pass's list
        // lengths, in one round trip
        if (tid < kXcd) {
            s_pf[tid] = ld_ctl(ctl, xw(tid, XF_PFILL + p % 3));
            if (A.tile_track) s_seg[tid] = ld_ctl(ctl, xw(tid, XF_ACT + (p + 1) % 3));
            if (phase1) s_km[tid] = ld_ctl(ctl, xw(tid, XF_KMAX));
        }
        __syncthreads();
        int fills = 0, km = 0;
#pragma unroll
        for (int x = 0; x < kXcd; ++x) {
            fills += s_pf[x];
            if (phase1) km = max(km, s_km[x]);
        }
        if (lw == 0 && tid == 0) {  // front sizes of the pass; the half is reused two passes on
            for (int j = 0; j < Sp && j < 32; ++j) {
                int32_t *cw = &ctl[G_FRONT + (p & 1) * 32 + j];
                const int nf = ld_ctl(ctl, G_FRONT + (p & 1) * 32 + j);
                max_front = max(max_front, nf);
                if (A.front_hist && k0 + j < A.kcap) A.front_hist[k0 + j] = nf;  // a later pass may rewrite it
                __hip_atomic_store(cw, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        force_all = false;
        if (phase1 && km < k0 + Sp) {
            // shell km filled nothing under the data term: it is taken again
            // without it (nothing after it in this pass changed either)
            phase1 = false;
            force_all = true;
            total_filled += fills;
            k0 = km;
            continue;
        }
        if (fills == 0) break;
        total_filled += fills;
        k0 += Sp;
    }

    // ---- finish ---------------------------------------------------------------
    GF_RT_FLUSH(11, rt_fill);
    GF_RT_FLUSH(13, rt_sync);
    if (!copied)  // no pass ran (no hole pixel)
        copy_known<TS>(reinterpret_cast<const TS *>(A.in), reinterpret_cast<TS *>(A.out), A.label, C, A.NP, lw,
                       nblk);
    if (total_filled < total_hole) {  // leftovers never became ready: shell -3, input colour
        for (int t = lw; t < A.ntiles; t += nblk) {
            if (A.t_rem[t] == 0) continue;
            const int f = t / tpf, rr = t - f * tpf, ty = rr / A.tiles_x, tx = rr - ty * A.tiles_x;
            const int tw = min(A.TW, W - tx * A.TW), th = min(A.TH, H - ty * A.TH);
            int32_t *Sw = A.shell + (long long)f * A.HW;
            for (int i = tid; i < tw * th; i += NT) {
                const int y = ty * A.TH + i / tw, x = tx * A.TW + i % tw;
                if (Sw[y * W + x] == S_HOLE) {
                    Sw[y * W + x] = S_UNFILLED;
                    if (!A.inplace) {
                        const long long q = ((long long)f * A.HW + (long long)y * W + x) * C;
                        for (int ch = 0; ch < C; ++ch)
                            reinterpret_cast<TS *>(A.out)[q + ch] = reinterpret_cast<const TS *>(A.in)[q + ch];
                    }
                }
            }
        }
    }
    for (int f = lw; f < A.B; f += nblk) {  // per-frame statistics, one workgroup per frame
        int kf = 0, ff = 0, hf = 0;
        for (int i = tid; i < tpf; i += NT) {
            const int t = f * tpf + i;
            kf = max(kf, A.t_kmax[t]);
            ff += A.t_fill[t];
            hf += A.t_hole[t];
        }
        if (kf) atomicMax(&s_r[2], kf);
        if (ff) atomicAdd(&s_r[0], ff);
        if (hf) atomicAdd(&s_r[1], hf);
        __syncthreads();
        if (tid == 0) {
            A.stats[8 + 4 * f + 0] = s_r[2];
            A.stats[8 + 4 * f + 1] = s_r[0];
            A.stats[8 + 4 * f + 2] = s_r[1];
            s_r[0] = s_r[1] = s_r[2] = 0;
        }
        __syncthreads();
    }
    if (lw == 0 && tid == 0) {
        A.stats[0] = max_x(ctl, XF_KMAX);
        A.stats[1] = (int32_t)total_filled;
        A.stats[2] = total_hole;
        A.stats[3] = max_front;
        A.stats[4] = sum_x(ctl, XF_ERR);
        A.stats[5] = 0;
        A.stats[6] = ld_ctl(ctl, G_TIMEOUT);
        A.stats[7] = nblk;
    }
}

}  // namespace gfk
