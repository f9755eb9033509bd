// Shell fill of Guidefill (Hocking, MacKenzie, Schoenlieb, arXiv 1611.05319)
// for MI355X (gfx950): host side of the C ABI declared in include/guidefill.h.
//
// Engines (gf_params.engine):
//   GF_ENGINE_TILED   tile windows staged in LDS run S shells between grid
//                     barriers (tile_engine.h); default.
//   GF_ENGINE_FRONT   one grid barrier per shell, the front as a global list
//                     (global_engine.h); also records the fill order the
//                     adjoint replays.
// Both run as one persistent launch (an ordinary grid sized to what the
// device holds); at start-up the resident workgroups join, one of them zeroes
// the control words and the stats while the others wait for it.
//
// Every decision of the fill is FP64: the ghost offsets must be bit-identical
// to the reference (points that land on lattice lines change the readable
// set), so the rotation is evaluated as ox = n*s + m*c, oy = m*s - n*c with
// (c, s) = g/|g|, IEEE division and square root, and no contraction into FMA.
// The weights and weighted sums are FP64 too; each ghost value is
// interpolated in FP32 from the stored colours.

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <mutex>
#include <vector>
#include <unordered_map>

#include "coherence.h"
#include "guide_field.h"
#include "guidefill.h"
#include "tile_engine.h"

using namespace gfk;

namespace {

// Launch start-up per workspace: an epoch the workspace's control block has
// not held (the kernels' start-up handshake waits for it) and the join-word
// set of the ring (each launch clears the next set; a zeroed workspace has
// all of them clear).  The first epoch of a workspace is drawn from the clock
// and the address, so stale or arbitrary content is unlikely to match it; it
// is never 0 (a zeroed workspace).  The state advances only once a launch is
// enqueued (a call that fails before its launch must not skip a set: the
// set after it would not have been cleared).
LaunchSync peek_launch(const void *ws);
void commit_launch(const void *ws, const LaunchSync &ls);

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
    int clock_khz = 100000;    // constant clock (wall_clock64) rate
    size_t lds_block = 65536;  // bytes of LDS one workgroup may use
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
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, dev) == hipSuccess && v > 0)
        d.clock_khz = v;
    v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        d.lds_block = (size_t)v;
    if (dev >= 0 && dev < 64) {
        cache[dev] = d;
        have[dev] = true;
    }
    return d;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct LaunchState {
    unsigned epoch;
    int slot;
};
std::mutex g_launch_mu;
std::unordered_map<const void *, LaunchState> g_launch_states;

LaunchSync peek_launch(const void *ws) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const int khz = device_info(dev).clock_khz;
    std::lock_guard<std::mutex> lk(g_launch_mu);
    auto it = g_launch_states.find(ws);
    if (it == g_launch_states.end()) {
        const unsigned long long t =
            (unsigned long long)std::chrono::steady_clock::now().time_since_epoch().count();
        const unsigned long long p = (unsigned long long)(uintptr_t)ws;
        const unsigned e = (unsigned)((t ^ (t >> 32) ^ (p >> 8) ^ (p >> 40)) * 2654435761u);
        it = g_launch_states.emplace(ws, LaunchState{e, kLaunchSlots - 1}).first;
    }
    LaunchSync ls;
    ls.epoch = it->second.epoch + 1u;
    if (ls.epoch == 0u) ls.epoch = 1u;
    ls.slot = (it->second.slot + 1) % kLaunchSlots;
    // the launched workgroups normally all join within a few microseconds;
    // 50 us bounds the wait when some of them cannot be resident
    ls.join_ticks = (int)std::min<long long>((long long)khz * 50 / 1000, 1 << 30);
    return ls;
}

void commit_launch(const void *ws, const LaunchSync &ls) {
    std::lock_guard<std::mutex> lk(g_launch_mu);
    g_launch_states[ws] = LaunchState{ls.epoch, ls.slot};
}

// The raw value of an enum argument: C callers may pass any int, and loading
// an out-of-range value through the C++ enum type would be undefined, so the
// bits are copied into an int and compared as such.
template <typename E> int raw_enum(const E *v) {
    static_assert(sizeof(E) == sizeof(int), "enum arguments are int-sized");
    int r;
    memcpy(&r, v, sizeof r);
    return r;
}

gf_status validate(const gf_params *p, int B, int H, int W, int C, int dt) {
    if (!p) return GF_EINVAL;
    if (B < 1 || H < 1 || W < 1 || C < 1 || C > 4) return GF_EINVAL;
    if (dt != GF_F32 && dt != GF_F16) return GF_EINVAL;
    if (!(p->eps >= 1.0) || !(p->eps <= 9.0) || !(p->mu > 0.0) || !isfinite(p->mu)) return GF_EINVAL;
    if (!(p->c == p->c) || !(p->c2 == p->c2)) return GF_EINVAL;
    if (p->max_shells < 0) return GF_EINVAL;
    if (p->engine != GF_ENGINE_TILED && p->engine != GF_ENGINE_FRONT) return GF_EINVAL;
    if (p->group != 0 && p->group != 4 && p->group != 8 && p->group != 16 && p->group != 32 &&
        p->group != 64)
        return GF_EINVAL;
    if (p->group == 4 && p->engine != GF_ENGINE_TILED) return GF_EINVAL;
    if (p->blocks_per_cu < 0 || p->blocks_per_cu > 8) return GF_EINVAL;
    if (p->tile_w < 0 || p->tile_h < 0 || p->tile_w > 256 || p->tile_h > 256) return GF_EINVAL;
    if (p->pass_shells < 0 || p->pass_shells > 32) return GF_EINVAL;
    if (p->tile_threads != 0 && p->tile_threads != 256 && p->tile_threads != 512 &&
        p->tile_threads != 768 && p->tile_threads != 1024)
        return GF_EINVAL;
    if (p->tile_threads != 0 && p->engine != GF_ENGINE_TILED) return GF_EINVAL;
    long long np = (long long)B * H * W;
    if (np * C >= (1ll << 31)) return GF_EUNSUPPORTED;  // int32 pixel indices in the lists
    // the data term's switch is a per-frame event; one launch switches once
    if (p->c2 >= 0.0 && B > 1) return GF_EUNSUPPORTED;
    return GF_OK;
}

// lanes per pixel: the smallest group with at most 4 offsets per lane
int pick_group(const gf_params *p, int T) {
    if (p->group) return p->group;
    return T <= 32 ? 8 : (T <= 64 ? 16 : (T <= 128 ? 32 : 64));
}

// tile geometry of the tiled engine
struct TileGeom {
    int TW, TH, S, Hh, WW, WH, WN;
    size_t lds;
};

int rdep_of(double eps) { return (int)ceil(eps); }

template <typename TS>
bool tile_geometry(const gf_params *p, int C, size_t lds_limit, TileGeom &g) {
    const int rd = rdep_of(p->eps);
    const size_t static_lds = kTileStaticLds;  // staging buffer, offsets, counters
    // measured at eps = 3 (1080p): 4 shells per pass beat 6 (180.9 vs 184.7 us)
    int S = p->pass_shells ? p->pass_shells : (rd <= 2 ? 6 : (rd == 3 ? 4 : (rd <= 6 ? 3 : 2)));
    for (;;) {
        const int Hh = S * rd;
        int TW = p->tile_w ? p->tile_w : (Hh > 32 ? Hh : 32);
        int TH = p->tile_h ? p->tile_h : TW;
        if (Hh > TW || Hh > TH) {
            if (p->tile_w || p->tile_h) return false;  // the halo must stay inside the neighbours
        }
        // shrink the tile until the window fits the LDS (not below the halo)
        for (;;) {
            const int WW = TW + 2 * Hh, WH = TH + 2 * Hh, WN = WW * WH;
            const size_t lds = tile_lds_bytes<TS>(WN, C);
            if (WN <= kMaxWindow && lds + static_lds <= lds_limit) {
                g = {TW, TH, S, Hh, WW, WH, WN, lds};
                return true;
            }
            if (p->tile_w || p->tile_h) return false;
            if (TW - 4 < Hh || TW <= 8) break;
            TW -= 4;
            TH = TW;
        }
        if (p->pass_shells || S == 1) return false;
        --S;
    }
}

// Per (device, kernel, block, dynamic LDS): the dynamic-LDS attribute is set
// and the occupancy queried once, so a repeated call costs one launch.
struct LaunchKey {
    int dev;
    const void *fn;
    int block;
    size_t lds;
};

int cached_occupancy(int dev, const void *fn, int block, size_t dyn_lds, hipError_t *err) {
    static std::mutex mu;
    static LaunchKey keys[256];
    static int occs[256];
    static int n = 0;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < n; ++i)
        if (keys[i].dev == dev && keys[i].fn == fn && keys[i].block == block && keys[i].lds == dyn_lds)
            return occs[i];
    *err = hipSuccess;
    if (dyn_lds > 0) {
        *err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_lds);
        if (*err != hipSuccess) return 0;
    }
    int occ = 0;
    *err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, dyn_lds);
    if (*err != hipSuccess) return 0;
    if (occ >= 1 && n < 256) {
        keys[n] = {dev, fn, block, dyn_lds};
        occs[n] = occ;
        ++n;
    }
    return occ;
}

// One persistent launch: an ordinary grid of per_cu workgroups per compute
// unit (at most what the occupancy allows, a multiple of the XCD count); the
// kernels' start-up finds which of them are resident.
template <typename K>
gf_status launch_persistent(K kernel, const void *args_ptr, int blocks_per_cu, long long max_blocks,
                            size_t dyn_lds, hipStream_t stream, int block = kBlock) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_err("hipGetDevice", e); return GF_EDEVICE; }
    DevInfo di = device_info(dev);
    if (di.cus <= 0) {
        snprintf(g_last_error, sizeof g_last_error, "device %d reports no compute units", dev);
        return GF_EDEVICE;
    }
    e = hipSuccess;
    const int occ = cached_occupancy(dev, reinterpret_cast<const void *>(kernel), block, dyn_lds, &e);
    if (e != hipSuccess || occ < 1) {
        if (e == hipSuccess) snprintf(g_last_error, sizeof g_last_error, "kernel does not fit a CU");
        else set_err("launch set-up", e);
        return GF_EDEVICE;
    }
    int per_cu = blocks_per_cu > 0 ? blocks_per_cu : (block > kBlock ? 1 : 2);
    if (per_cu > occ) per_cu = occ;
    long long grid = (long long)per_cu * di.cus;
    if (max_blocks < kXcd) max_blocks = kXcd;
    if (grid > max_blocks) grid = max_blocks;
    grid = (grid / kXcd) * kXcd;
    if (grid < kXcd) grid = kXcd;
    void *kargs[] = {const_cast<void *>(args_ptr)};
    e = hipLaunchKernel(reinterpret_cast<const void *>(kernel), dim3((unsigned)grid), dim3(block), kargs,
                        dyn_lds, stream);
    if (e != hipSuccess) { set_err("hipLaunchKernel", e); return GF_EDEVICE; }
    return GF_OK;
}

template <typename TS>
gf_status run_front(const FillArgs &A, int G, int bpc, hipStream_t s) {
    const long long mb = (A.NP + kBlock - 1) / kBlock;
    if (bpc == 0) bpc = 8;  // as many workgroups per CU as the registers and LDS allow
    // one neighbourhood window per group of G lanes
    const size_t lds = (size_t)(kBlock / G) * window_bytes<TS>((int)ceil(A.eps));
    if (G == 8) return launch_persistent(fill_kernel<TS, 8>, &A, bpc, mb, lds, s);
    if (G == 16) return launch_persistent(fill_kernel<TS, 16>, &A, bpc, mb, lds, s);
    if (G == 32) return launch_persistent(fill_kernel<TS, 32>, &A, bpc, mb, lds, s);
    return launch_persistent(fill_kernel<TS, 64>, &A, bpc, mb, lds, s);
}

// threads per tile workgroup
// (768 by default: 168 registers a lane against 128 at 1024, enough for the
// one-round window staging; 172 vs 183 us on the full-HD frame)
int tile_threads_of(const gf_params *p) { return p->tile_threads ? p->tile_threads : 768; }

template <typename TS, int NT>
gf_status run_tiled_nt(const TileArgs &A, int G, int bpc, size_t lds, hipStream_t s) {
    const long long mb = 1ll << 30;
    if (bpc == 0) bpc = 8;  // as many workgroups per CU as the LDS and registers allow
    if (G == 4) return launch_persistent(tile_kernel<TS, 4, NT>, &A, bpc, mb, lds, s, NT);
    if (G == 8) return launch_persistent(tile_kernel<TS, 8, NT>, &A, bpc, mb, lds, s, NT);
    if (G == 16) return launch_persistent(tile_kernel<TS, 16, NT>, &A, bpc, mb, lds, s, NT);
    if (G == 32) return launch_persistent(tile_kernel<TS, 32, NT>, &A, bpc, mb, lds, s, NT);
    return launch_persistent(tile_kernel<TS, 64, NT>, &A, bpc, mb, lds, s, NT);
}

template <typename TS>
gf_status run_tiled(const TileArgs &A, int G, int NT, int bpc, size_t lds, hipStream_t s) {
    if (NT == 256) return run_tiled_nt<TS, 256>(A, G, bpc, lds, s);
    if (NT == 512) return run_tiled_nt<TS, 512>(A, G, bpc, lds, s);
    if (NT == 768) return run_tiled_nt<TS, 768>(A, G, bpc, lds, s);
    return run_tiled_nt<TS, 1024>(A, G, bpc, lds, s);
}

template <typename TS>
gf_status run_bwd(const BwdArgs &A, int G, int bpc, hipStream_t s) {
    const long long mb = (A.NP + kBlock - 1) / kBlock;
    if (bpc == 0) bpc = 8;  // as many workgroups per CU as the registers and LDS allow
    const size_t lds = bwd_dyn_lds<TS>(G, (int)ceil(A.eps), A.C);
    if (G == 8) return launch_persistent(bwd_kernel<TS, 8>, &A, bpc, mb, lds, s);
    if (G == 16) return launch_persistent(bwd_kernel<TS, 16>, &A, bpc, mb, lds, s);
    if (G == 32) return launch_persistent(bwd_kernel<TS, 32>, &A, bpc, mb, lds, s);
    return launch_persistent(bwd_kernel<TS, 64>, &A, bpc, mb, lds, s);
}

// adjoint workspace: control block, two rounds of shell counts, shell offsets
// (a frame has at most H * W shells), the filled pixels grouped by shell
struct BwdLayout {
    size_t ctl, gcount, offs, order, total;
};

BwdLayout bwd_layout(int B, int H, int W) {
    BwdLayout L;
    size_t off = 0;
    L.ctl = off; off += align256(kCtlWords * sizeof(int32_t));
    L.gcount = off; off += align256(2 * (size_t)kBwdBins * sizeof(int32_t));
    L.offs = off; off += align256(((size_t)H * W + 2) * sizeof(int32_t));
    L.order = off; off += align256((size_t)B * H * W * sizeof(int32_t));
    L.total = off;
    return L;
}

struct WsLayout {
    size_t ctl, listA, listB;                              // front engine
    size_t t_hole, t_rem, t_kmax, t_fill, t_mark, act0, act1;  // tiled engine
    size_t total;
};

bool layout_for(int B, int H, int W, int C, int dt, const gf_params *p, WsLayout &L,
                TileGeom *geom_out, int *tiles_x, int *tiles_y) {
    memset(&L, 0, sizeof L);
    size_t off = align256(kCtlWords * sizeof(int32_t));
    L.ctl = 0;
    const size_t np = (size_t)B * H * W;
    if (p->engine == GF_ENGINE_FRONT) {
        L.listA = off;
        off += align256(np * 4);
        L.listB = off;
        off += align256(np * 4);
        L.total = off;
        return true;
    }
    int dev = 0;
    size_t lds_limit = 65536;
    if (hipGetDevice(&dev) == hipSuccess) lds_limit = device_info(dev).lds_block;
    TileGeom g;
    const bool ok = dt == GF_F16 ? tile_geometry<__half>(p, C, lds_limit, g)
                                 : tile_geometry<float>(p, C, lds_limit, g);
    if (!ok) return false;
    const int tx = (W + g.TW - 1) / g.TW, ty = (H + g.TH - 1) / g.TH;
    const size_t nt = (size_t)B * tx * ty;
    L.t_hole = off; off += align256(nt * 4);
    L.t_rem = off; off += align256(nt * 4);
    L.t_kmax = off; off += align256(nt * 4);
    L.t_fill = off; off += align256(nt * 4);
    L.t_mark = off; off += align256(nt * 4);
    L.act0 = off; off += align256(nt * 4 * kXcd);
    L.act1 = off; off += align256(nt * 4 * kXcd);
    L.total = off;
    if (geom_out) *geom_out = g;
    if (tiles_x) *tiles_x = tx;
    if (tiles_y) *tiles_y = ty;
    return true;
}

// Library-owned scratch for gf_fill_batched_noalloc: a workspace that lives
// in the code object, so callers that cannot allocate device memory (code
// under graph capture, serving loops) still get one.  Each device that loads
// the library holds its own zero-initialised copy until the process ends.  In
// host code `scratch` names a host-side stand-in, never a device address: the
// device address is looked up once per device (scratch_on_device) and only
// that pointer is handed to kernels.
constexpr size_t kScratchBytes = GF_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's scratch; the first call on a device looks
// it up (with that device current) and keeps it.  nullptr on failure (the
// HIP error is recorded for gf_last_error).
void *scratch_on_device(int dev) {
    static std::mutex mu;
    static void *ptrs[64] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (dev < 0 || dev >= 64) {
        snprintf(g_last_error, sizeof g_last_error, "device index %d outside 0..63", dev);
        return nullptr;
    }
    if (ptrs[dev]) return ptrs[dev];
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        set_err("hipGetSymbolAddress(scratch)", e);
        return nullptr;
    }
    ptrs[dev] = ptr;
    return ptr;
}

size_t workspace_bytes(int B, int H, int W, int C, int dt, const gf_params *p) {
    if (!p || B < 1 || H < 1 || W < 1 || C < 1 || (dt != GF_F32 && dt != GF_F16)) return 0;
    WsLayout L;
    if (!layout_for(B, H, W, C, dt, p, L, nullptr, nullptr, nullptr)) return 0;
    return L.total;
}

gf_status fill_batched(const void *img_in, void *img_out, int B, int H, int W, int C, int dt,
                       const uint8_t *label, const float *guide, const gf_params *p,
                       int32_t *shell_out, int32_t *stats, int32_t *order_out,
                       int32_t *shell_offsets, int32_t *front_hist, int kcap, void *workspace,
                       size_t ws_bytes, void *stream);

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

int gf_version(void) { return 2; }

gf_status gf_guide_field(int B, int H, int W, const uint8_t *label, const float *seg,
                         const int32_t *seg_off, double eta, double cutoff, float *guide,
                         void *stream) {
    if (B < 1 || H < 1 || W < 1 || !label || !seg_off || !guide) return GF_EINVAL;
    if (!(eta > 0.0) || !(cutoff >= 0.0) || !isfinite(eta) || !isfinite(cutoff)) return GF_EINVAL;
    GuideArgs A;
    A.label = label;
    A.seg = seg;
    A.seg_off = seg_off;
    A.guide = guide;
    A.HW = (long long)H * W;
    A.B = B;
    A.H = H;
    A.W = W;
    A.tiles_x = (W + kGuideTile - 1) / kGuideTile;
    A.tiles_y = (H + kGuideTile - 1) / kGuideTile;
    A.eta = eta;
    A.cutoff = cutoff;
    const long long grid = (long long)B * A.tiles_x * A.tiles_y;
    if (grid >= (1ll << 31)) return GF_EUNSUPPORTED;
    void *kargs[] = {&A};
    const hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(guide_kernel),
                                         dim3((unsigned)grid), dim3(kBlock), kargs, 0,
                                         reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) { set_err("hipLaunchKernel", e); return GF_EDEVICE; }
    return GF_OK;
}

const char *gf_status_string(gf_status s_arg) {
    switch (raw_enum(&s_arg)) {
    case GF_OK: return "ok";
    case GF_EINVAL: return "invalid argument";
    case GF_EDEVICE: return "HIP device error";
    case GF_EUNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

const char *gf_last_error(void) { return g_last_error; }

size_t gf_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p) {
    return workspace_bytes(B, H, W, C, raw_enum(&dt), p);
}

size_t gf_backward_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p) {
    (void)C; (void)dt; (void)p;
    if (B < 1 || H < 1 || W < 1) return 0;
    return bwd_layout(B, H, W).total;
}

gf_status gf_fill_batched(const void *img_in, void *img_out, int B, int H, int W, int C,
                          gf_dtype dt, const uint8_t *label, const float *guide,
                          const gf_params *p, int32_t *shell_out, int32_t *stats,
                          int32_t *order_out, int32_t *shell_offsets, int32_t *front_hist,
                          int kcap, void *workspace, size_t ws_bytes, void *stream) {
    return fill_batched(img_in, img_out, B, H, W, C, raw_enum(&dt), label, guide, p, shell_out,
                        stats, order_out, shell_offsets, front_hist, kcap, workspace, ws_bytes,
                        stream);
}

}  // extern "C"

namespace {

gf_status fill_batched(const void *img_in, void *img_out, int B, int H, int W, int C, int dt,
                       const uint8_t *label, const float *guide, const gf_params *p,
                       int32_t *shell_out, int32_t *stats, int32_t *order_out,
                       int32_t *shell_offsets, int32_t *front_hist, int kcap, void *workspace,
                       size_t ws_bytes, void *stream) {
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    if (!img_in || !img_out || !label || !guide || !shell_out || !stats || !workspace)
        return GF_EINVAL;
    if ((order_out == nullptr) != (shell_offsets == nullptr)) return GF_EINVAL;
    if ((order_out || front_hist) && kcap < 1) return GF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return GF_EINVAL;
    if (order_out && p->engine != GF_ENGINE_FRONT) return GF_EUNSUPPORTED;
    const int T = count_offsets(p->eps);
    const int G = pick_group(p, T);
    if (T > G * per_lane_of(G) || T > kMaxOffsets || (int)floor(p->eps) >= G)
        return GF_EUNSUPPORTED;
    WsLayout L;
    TileGeom geom;
    int tiles_x = 0, tiles_y = 0;
    if (!layout_for(B, H, W, C, dt, p, L, &geom, &tiles_x, &tiles_y)) return GF_EINVAL;
    if (ws_bytes < L.total) return GF_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    int32_t *ctl = reinterpret_cast<int32_t *>(ws + L.ctl);
    const double a = p->mu * p->mu / (2.0 * p->eps * p->eps);
    const LaunchSync ls = peek_launch(workspace);
    if (p->engine == GF_ENGINE_FRONT) {
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
        A.ctl = ctl;
        A.listA = reinterpret_cast<int32_t *>(ws + L.listA);
        A.listB = reinterpret_cast<int32_t *>(ws + L.listB);
        A.HW = (long long)H * W;
        A.NP = (long long)B * H * W;
        A.B = B;
        A.H = H;
        A.W = W;
        A.C = C;
        A.kcap = kcap;
        A.tracking = p->tracking ? 1 : 0;
        A.max_shells = p->max_shells;
        A.inplace = img_in == img_out;
        A.eps = p->eps;
        A.a = a;
        A.c = p->c;
        A.c2 = p->c2;
        A.ghost = p->ghost ? 1 : 0;
        A.sync = ls;
        const gf_status rc = dt == GF_F32 ? run_front<float>(A, G, p->blocks_per_cu, s)
                                          : run_front<__half>(A, G, p->blocks_per_cu, s);
        if (rc == GF_OK) commit_launch(workspace, ls);
        return rc;
    }
    TileArgs A;
    A.in = img_in;
    A.out = img_out;
    A.label = label;
    A.guide = guide;
    A.shell = shell_out;
    A.stats = stats;
    A.front_hist = front_hist;
    A.ctl = ctl;
    A.t_hole = reinterpret_cast<int32_t *>(ws + L.t_hole);
    A.t_rem = reinterpret_cast<int32_t *>(ws + L.t_rem);
    A.t_kmax = reinterpret_cast<int32_t *>(ws + L.t_kmax);
    A.t_fill = reinterpret_cast<int32_t *>(ws + L.t_fill);
    A.t_mark = reinterpret_cast<int32_t *>(ws + L.t_mark);
    A.act0 = reinterpret_cast<int32_t *>(ws + L.act0);
    A.act1 = reinterpret_cast<int32_t *>(ws + L.act1);
    A.HW = (long long)H * W;
    A.NP = (long long)B * H * W;
    A.B = B;
    A.H = H;
    A.W = W;
    A.C = C;
    A.kcap = kcap;
    A.TW = geom.TW;
    A.TH = geom.TH;
    A.S = geom.S;
    A.Hh = geom.Hh;
    A.WW = geom.WW;
    A.WH = geom.WH;
    A.WN = geom.WN;
    A.tiles_x = tiles_x;
    A.tiles_y = tiles_y;
    A.ntiles = B * tiles_x * tiles_y;
    A.max_shells = p->max_shells;
    A.inplace = img_in == img_out;
    A.ghost = p->ghost ? 1 : 0;
    A.tile_track = p->tracking ? 1 : 0;
    A.local_track = p->tracking ? 1 : 0;
    A.eps = p->eps;
    A.a = a;
    A.c = p->c;
    A.c2 = p->c2;
    A.sync = ls;
    const int NT = tile_threads_of(p);
    const gf_status rc = dt == GF_F32 ? run_tiled<float>(A, G, NT, p->blocks_per_cu, geom.lds, s)
                                      : run_tiled<__half>(A, G, NT, p->blocks_per_cu, geom.lds, s);
    if (rc == GF_OK) commit_launch(workspace, ls);
    return rc;
}

// Workspace of the comparison fill: the per-shell fill's workspace first
// (it keeps its launch handshake state across calls), then working labels,
// guides, the per-shell shell map and stats.
struct CtLayout {
    size_t fill, label, guide, step, stats, bad, total;
};

// Shells the comparison mode enqueues between two host reads of their
// statistics.  A shell enqueued after the fill is over changes nothing (with
// the state unchanged, the tensor field and the shell's fill are those of the
// shell before, which filled nothing), so a batch only ends early in time.
constexpr int kCtBatch = 4;

// the comparison mode's one-shell fills: one shell per launch, and on the
// tiled engine (unless the caller sets it) one shell per pass, so the tile
// windows carry a halo of ceil(eps) only (2.15 -> 2.09 ms at 1080p)
gf_params ct_fill_params(const gf_params *p) {
    gf_params p1 = *p;
    p1.max_shells = 1;
    if (p1.pass_shells == 0) p1.pass_shells = 1;
    return p1;
}

bool ct_layout(int B, int H, int W, int C, int dt, const gf_params *p, CtLayout &L) {
    const gf_params p1 = ct_fill_params(p);
    const size_t fw = workspace_bytes(B, H, W, C, dt, &p1);
    if (fw == 0) return false;
    const size_t np = (size_t)B * H * W;
    size_t off = 0;
    L.fill = off; off += align256(fw);
    L.label = off; off += align256(np);
    L.guide = off; off += align256(np * 2 * sizeof(float));
    L.step = off; off += align256(np * sizeof(int32_t));
    L.stats = off;
    off += align256((size_t)kCtBatch * (GF_STAT_FRAME0 + GF_STAT_PER_FRAME * B) * sizeof(int32_t));
    L.bad = off; off += 256;
    L.total = off;
    return true;
}

// Tile edge of the tensor kernel: 16 when its LDS fits, else 8 (0: neither)
int ct_tile(int rs, int rr, int C, size_t lds_limit) {
    if (ct_lds(16, rs, rr, C).total <= lds_limit) return 16;
    if (ct_lds(8, rs, rr, C).total <= lds_limit) return 8;
    return 0;
}

gf_status ct_validate(const gf_params *p, int B, int H, int W, int C, int dt, double sigma,
                      double rho, double lambda) {
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    if (!(sigma > 0.0) || !(rho > 0.0) || !(lambda > 0.0) || !isfinite(lambda)) return GF_EINVAL;
    if (!(sigma <= 8.0) || !(rho <= 16.0)) return GF_EUNSUPPORTED;
    // the guide changes every shell, so the data term's phase switch has no fixed region
    if (p->c2 >= 0.0) return GF_EUNSUPPORTED;
    return GF_OK;
}

}  // namespace

extern "C" {

size_t gf_coherence_workspace_size(int B, int H, int W, int C, gf_dtype dt_arg, const gf_params *p) {
    const int dt = raw_enum(&dt_arg);
    if (!p || validate(p, B, H, W, C, dt) != GF_OK) return 0;
    CtLayout L;
    if (!ct_layout(B, H, W, C, dt, p, L)) return 0;
    return L.total;
}

gf_status gf_fill_coherence(const void *img_in, void *img_out, int B, int H, int W, int C,
                            gf_dtype dt_arg, const uint8_t *label, const gf_params *p,
                            double sigma, double rho, double lambda, int32_t *shell_out,
                            int32_t *stats, float *guide_used, void *workspace, size_t ws_bytes,
                            void *stream) {
    const int dt = raw_enum(&dt_arg);
    gf_status st = ct_validate(p, B, H, W, C, dt, sigma, rho, lambda);
    if (st != GF_OK) return st;
    if (!img_in || !img_out || !label || !shell_out || !stats || !workspace) return GF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return GF_EINVAL;
    CtLayout L;
    if (!ct_layout(B, H, W, C, dt, p, L)) return GF_EINVAL;
    if (ws_bytes < L.total) return GF_EINVAL;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_err("hipGetDevice", e); return GF_EDEVICE; }
    const DevInfo di = device_info(dev);
    const int rs = (int)floor(2.0 * sigma), rr = (int)floor(2.0 * rho);
    const int tile = ct_tile(rs, rr, C, di.lds_block);
    if (tile == 0) return GF_EUNSUPPORTED;
    const size_t lds = ct_lds(tile, rs, rr, C).total;
    const void *kfn = dt == GF_F32 ? reinterpret_cast<const void *>(ct_guide_kernel<float>)
                                   : reinterpret_cast<const void *>(ct_guide_kernel<__half>);
    cached_occupancy(dev, kfn, kBlock, lds, &e);
    if (e != hipSuccess) { set_err("tensor kernel set-up", e); return GF_EDEVICE; }

    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    char *ws = reinterpret_cast<char *>(workspace);
    uint8_t *label_w = reinterpret_cast<uint8_t *>(ws + L.label);
    float *guide_w = reinterpret_cast<float *>(ws + L.guide);
    int32_t *step = reinterpret_cast<int32_t *>(ws + L.step);
    int32_t *stats_step = reinterpret_cast<int32_t *>(ws + L.stats);
    int32_t *bad = reinterpret_cast<int32_t *>(ws + L.bad);
    const long long NP = (long long)B * H * W;
    const size_t esz = dt == GF_F32 ? 4 : 2;
    const int nstat = GF_STAT_FRAME0 + GF_STAT_PER_FRAME * B;
    const int egrid = (int)std::min<long long>((NP + kBlock - 1) / kBlock, 8192);

    if (img_out != img_in) {
        e = hipMemcpyAsync(img_out, img_in, (size_t)NP * C * esz, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) { set_err("hipMemcpyAsync", e); return GF_EDEVICE; }
    }
    e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
    if (e != hipSuccess) { set_err("hipMemsetAsync", e); return GF_EDEVICE; }
    hipLaunchKernelGGL(ct_init_kernel, dim3(egrid), dim3(kBlock), 0, s, label, label_w, shell_out,
                       guide_w, guide_used, bad, NP);
    e = hipGetLastError();
    if (e != hipSuccess) { set_err("hipLaunchKernel", e); return GF_EDEVICE; }

    CtArgs A;
    A.img = img_out;
    A.label = label_w;
    A.guide = guide_w;
    A.HW = (long long)H * W;
    A.B = B;
    A.H = H;
    A.W = W;
    A.C = C;
    A.tile = tile;
    A.tiles_x = (W + tile - 1) / tile;
    A.tiles_y = (H + tile - 1) / tile;
    A.rs = rs;
    A.rr = rr;
    A.sigma = sigma;
    A.rho = rho;
    A.lambda = lambda;
    const long long ngrid = (long long)B * A.tiles_x * A.tiles_y;
    if (ngrid >= (1ll << 31)) return GF_EUNSUPPORTED;

    const gf_params p1 = ct_fill_params(p);
    std::vector<int32_t> step_stats((size_t)kCtBatch * nstat), total(nstat, 0);
    int k = 0;
    for (bool more = true; more;) {
        int n = kCtBatch;
        if (p->max_shells > 0) n = std::min(n, p->max_shells - k);
        if (n <= 0) break;
        for (int j = 0; j < n; ++j) {  // shells k .. k + n - 1: guide, one-shell fill, commit
            void *kargs[] = {&A};
            e = hipLaunchKernel(kfn, dim3((unsigned)ngrid), dim3(kBlock), kargs, lds, s);
            if (e != hipSuccess) { set_err("hipLaunchKernel", e); return GF_EDEVICE; }
            st = fill_batched(img_out, img_out, B, H, W, C, dt, label_w, guide_w, &p1, step,
                              stats_step + (size_t)j * nstat, nullptr, nullptr, nullptr, 0,
                              ws + L.fill, L.label - L.fill, stream);
            if (st != GF_OK) return st;
            hipLaunchKernelGGL(ct_commit_kernel, dim3(egrid), dim3(kBlock), 0, s, label_w, step,
                               shell_out, guide_w, guide_used, NP, k + j);
            e = hipGetLastError();
            if (e != hipSuccess) { set_err("hipLaunchKernel", e); return GF_EDEVICE; }
        }
        e = hipMemcpyAsync(step_stats.data(), stats_step, (size_t)n * nstat * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) { set_err("shell statistics", e); return GF_EDEVICE; }
        for (int j = 0; j < n && more; ++j) {
            const int32_t *ss = step_stats.data() + (size_t)j * nstat;
            if (k == 0) {
                total[GF_STAT_HOLE] = ss[GF_STAT_HOLE];
                total[GF_STAT_WORKGROUPS] = ss[GF_STAT_WORKGROUPS];
                for (int f = 0; f < B; ++f)
                    total[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f + 2] =
                        ss[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f + 2];
            }
            total[GF_STAT_SYNC_TIMEOUT] |= ss[GF_STAT_SYNC_TIMEOUT];
            total[GF_STAT_MAX_FRONT] = std::max(total[GF_STAT_MAX_FRONT], ss[GF_STAT_MAX_FRONT]);
            const int filled = ss[GF_STAT_FILLED];
            if (filled == 0) {  // a stall, or nothing left: the shells after it changed nothing
                more = false;
                break;
            }
            total[GF_STAT_FILLED] += filled;
            total[GF_STAT_SHELLS] = k + 1;
            for (int f = 0; f < B; ++f) {
                const int ff = ss[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f + 1];
                total[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f] += ff > 0 ? 1 : 0;
                total[GF_STAT_FRAME0 + GF_STAT_PER_FRAME * f + 1] += ff;
            }
            ++k;
            if (total[GF_STAT_FILLED] >= total[GF_STAT_HOLE]) more = false;
        }
    }
    int32_t nbad = 0;
    e = hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_err("label check", e); return GF_EDEVICE; }
    total[GF_STAT_LABEL_ERR] = nbad;
    e = hipMemcpyAsync(stats, total.data(), nstat * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_err("statistics", e); return GF_EDEVICE; }
    return GF_OK;
}

gf_status gf_fill_batched_noalloc(const void *img_in, void *img_out, int B, int H, int W, int C,
                                  gf_dtype dt_arg, const uint8_t *label, const float *guide,
                                  const gf_params *p, int32_t *shell_out, int32_t *stats,
                                  int32_t *order_out, int32_t *shell_offsets, int32_t *front_hist,
                                  int kcap, void *stream) {
    const int dt = raw_enum(&dt_arg);
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    const size_t need = workspace_bytes(B, H, W, C, dt, p);
    if (need == 0) return GF_EINVAL;
    if (need > kScratchBytes) {
        snprintf(g_last_error, sizeof g_last_error,
                 "the request needs %zu bytes of workspace; the library's scratch holds %zu",
                 need, kScratchBytes);
        return GF_EINVAL;
    }
    int dev = 0;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_err("hipGetDevice", e); return GF_EDEVICE; }
    void *ws = scratch_on_device(dev);
    if (!ws) return GF_EDEVICE;
    return fill_batched(img_in, img_out, B, H, W, C, dt, label, guide, p, shell_out, stats,
                        order_out, shell_offsets, front_hist, kcap, ws, kScratchBytes, stream);
}

gf_status gf_fill(const void *img_in, void *img_out, int H, int W, int C, gf_dtype dt,
                  const uint8_t *label, const float *guide, const gf_params *p,
                  int32_t *shell_out, int32_t *stats, void *workspace, size_t ws_bytes,
                  void *stream) {
    return fill_batched(img_in, img_out, 1, H, W, C, raw_enum(&dt), label, guide, p, shell_out,
                        stats, nullptr, nullptr, nullptr, 0, workspace, ws_bytes, stream);
}

gf_status gf_tile_geometry(int H, int W, int C, gf_dtype dt_arg, const gf_params *p, int32_t *out6) {
    const int dt = raw_enum(&dt_arg);
    if (!p || !out6 || H < 1 || W < 1 || C < 1 || C > 4 || (dt != GF_F32 && dt != GF_F16))
        return GF_EINVAL;
    int dev = 0;
    size_t lds_limit = 65536;
    if (hipGetDevice(&dev) == hipSuccess) lds_limit = device_info(dev).lds_block;
    TileGeom g;
    const bool ok = dt == GF_F16 ? tile_geometry<__half>(p, C, lds_limit, g)
                                 : tile_geometry<float>(p, C, lds_limit, g);
    if (!ok) return GF_EINVAL;
    out6[0] = g.TW;
    out6[1] = g.TH;
    out6[2] = g.S;
    out6[3] = g.Hh;
    out6[4] = (int32_t)g.lds;
    out6[5] = pick_group(p, count_offsets(p->eps));
    return GF_OK;
}

gf_status gf_fill_backward(const float *grad_out, const void *img_out, int B, int H, int W, int C,
                           gf_dtype dt_arg, const uint8_t *label, const float *guide,
                           const int32_t *shell, int K, const gf_params *p, float *grad_img,
                           float *grad_guide, void *workspace, size_t ws_bytes, void *stream) {
    (void)label;  // the shell map carries every role the adjoint needs
    const int dt = raw_enum(&dt_arg);
    gf_status st = validate(p, B, H, W, C, dt);
    if (st != GF_OK) return st;
    if (!grad_out || !img_out || !guide || !shell || !grad_img || !grad_guide || !workspace)
        return GF_EINVAL;
    if (K < -1 || (long long)K > (long long)H * W) return GF_EINVAL;
    if (ws_bytes < bwd_layout(B, H, W).total) return GF_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return GF_EINVAL;
    // the launch shape is the adjoint's own (the forward's launch fields are
    // tuned for the forward): the narrowest group that holds the ball, two
    // workgroups per CU (a third fits, but measured slower when the adjoint
    // follows its forward: 445 against 437 us at 16 x 512^2)
    gf_params q = *p;
    q.engine = GF_ENGINE_FRONT;
    q.group = 0;
    q.blocks_per_cu = 2;
    const int T = count_offsets(p->eps);
    const int G = pick_group(&q, T);
    if (T > G * kPerLaneMax || T > kMaxOffsets) return GF_EUNSUPPORTED;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const BwdLayout L = bwd_layout(B, H, W);
    char *ws = reinterpret_cast<char *>(workspace);
    BwdArgs A;
    A.grad_out = grad_out;
    A.img = img_out;
    A.guide = guide;
    A.shell = shell;
    A.grad_img = grad_img;
    A.grad_guide = grad_guide;
    A.ctl = reinterpret_cast<int32_t *>(ws + L.ctl);
    A.gcount = reinterpret_cast<int32_t *>(ws + L.gcount);
    A.offs = reinterpret_cast<int32_t *>(ws + L.offs);
    A.order = reinterpret_cast<int32_t *>(ws + L.order);
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
    A.sync = peek_launch(workspace);
    const gf_status rc = dt == GF_F32 ? run_bwd<float>(A, G, q.blocks_per_cu, s)
                                      : run_bwd<__half>(A, G, q.blocks_per_cu, s);
    if (rc == GF_OK) commit_launch(workspace, A.sync);
    return rc;
}

#ifdef GF_TRACE
// Profiling builds only: copy the per-workgroup timing accumulators out and
// clear them.
int gf_trace_read(long long *host, int n) {
    if (n > 4096 * kTraceSlots) n = 4096 * kTraceSlots;
    if (hipMemcpyFromSymbol(host, HIP_SYMBOL(gf_trace), (size_t)n * sizeof(long long)) != hipSuccess)
        return -1;
    static long long zeros[4096 * kTraceSlots];
    if (hipMemcpyToSymbol(HIP_SYMBOL(gf_trace), zeros, sizeof zeros) != hipSuccess) return -1;
    return n;
}
#endif

}  // extern "C"
