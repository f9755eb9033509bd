// Device helpers shared by the kernels of guidefill.hip: constants, control
// words, storage conversions, group reductions, the grid barrier, the ball
// offsets and the ghost-point geometry (Guidefill, arXiv 1611.05319, Sec. 3.1
// and 3.3).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace gfk {

constexpr int kBlock = 256;       // threads per workgroup (4 wavefronts)
constexpr int kMaxOffsets = 256;  // eps <= 9: 252 offsets
constexpr int kPadOffset = 16384; // (n, m) of the padding entries of the offset table
constexpr int kPerLaneMax = 4;    // ball offsets handled by one lane (8 with 4-lane groups)
// offsets per lane for a group of G lanes: 4-lane groups take a whole
// eps <= 3 ball (28 offsets) in 7 steps, 16-lane groups an eps = 5 ball (80
// offsets) in 5, other widths at most 4 per lane
template <int G> __host__ __device__ constexpr int per_lane() {
    return G <= 4 ? 8 : (G == 16 ? 5 : kPerLaneMax);
}
__host__ __device__ inline int per_lane_of(int G) { return G <= 4 ? 8 : (G == 16 ? 5 : kPerLaneMax); }
constexpr int kStageCap = 1024;   // LDS staging entries per workgroup
constexpr int kFrameCap = 64;     // frames with LDS statistics accumulators (global engine)
constexpr int kXcd = 8;           // XCDs of the MI355X; workgroups are dealt round robin
constexpr int kCtlWords = 1024;   // control block (int32) at the start of the workspace

// Control words.  Counters updated by many workgroups are split per XCD and
// kept on separate 128-byte lines: same-address device atomics serialise.
constexpr int kXStride = 32;
enum : int {
    XF_BAR = 0,     // barrier arrivals of this XCD's workgroups
    XF_ACT = 1,     // [3] active-tile list lengths (tiled engine), ring by pass
    XF_PFILL = 4,   // [3] pixels filled in the pass, ring by pass
    XF_KMAX = 7,    // largest shell + 1 filled so far
    XF_HOLE = 8,    // label-1 pixels
    XF_ERR = 9,     // label errors
    XF_TICKET = 12, // [3] start-up join tickets of this XCD's workgroups, ring by launch slot
};
enum : int {
    G_GEN = 256,    // barrier generation
    G_TOP = 288,    // barrier arrivals of XCD groups
    G_LIST = 320,   // [3] front-list lengths (global engine), ring by shell
    G_ACTIVE = 384, // [3] active pixels (global engine, untracked)
    G_HOLE = 416,
    G_ERR = 448,
    G_ORDER = 480,  // entries written to order_out
    G_FRONT = 512,  // [2][32] front sizes per local shell, ring by pass (tiled engine)
    G_FILLED = 608, // pixels filled so far (global engine)
    G_TOP2 = 640,   // 64-bit: counting barrier, arrivals of XCD groups and their sums
    G_GEN2 = 672,   // 64-bit: counting barrier, generation and the published sums
    G_TIMEOUT = 704,// set when a barrier wait exceeded its spin limit
    G_READY = 736,  // epoch of the launch whose start-up is complete (never zeroed)
    G_LEAD = 768,   // [3] start-up leader election, ring by launch slot
    G_NX = 800,     // [kXcd] workgroups taking part per XCD group, this launch
    G_KEND = 832,   // adjoint: largest shell + 1 in the shell map
};
constexpr int kLaunchSlots = 3;         // join-word sets in the ring (see launch_start)
constexpr unsigned kClosed = 1u << 30;  // join word: the poll is closed
constexpr int XF_SUM = 10;  // 64-bit per-XCD word of the counting barrier (even index)
constexpr unsigned kSpinLimit = 1u << 26;  // barrier polls (s_sleep 1 each) before giving up
__device__ inline int xw(int x, int field) { return x * kXStride + field; }

// Optional timing hooks (compiled in only with -DGF_TRACE, for profiling
// builds): per-workgroup accumulators of wall-clock ticks and counts.
#ifdef GF_TRACE
constexpr int kTraceSlots = 16;
__device__ long long gf_trace[4096 * kTraceSlots];
#define GF_T0() long long gf_t_last = wall_clock64()
#define GF_TACC(slot)                                                                   \
    do {                                                                                \
        if (threadIdx.x == 0) {                                                         \
            const long long gf_t_now = wall_clock64();                                  \
            gf_trace[blockIdx.x * kTraceSlots + (slot)] += gf_t_now - gf_t_last;        \
            gf_t_last = gf_t_now;                                                       \
        }                                                                               \
    } while (0)
#define GF_TCNT(slot, v)                                                                \
    do {                                                                                \
        if (threadIdx.x == 0) gf_trace[blockIdx.x * kTraceSlots + (slot)] += (v);       \
    } while (0)
// register accumulators (no memory traffic inside loops), flushed once
#define GF_RT_DECL(name) long long name = 0, name##_t0 = 0
#define GF_RT_BEGIN(name) name##_t0 = wall_clock64()
#define GF_RT_END(name) name += wall_clock64() - name##_t0
#define GF_RT_FLUSH(slot, name)                                                         \
    do {                                                                                \
        if (threadIdx.x == 0) gf_trace[blockIdx.x * kTraceSlots + (slot)] += name;      \
    } while (0)
#else
#define GF_T0()
#define GF_TACC(slot)
#define GF_TCNT(slot, v)
#define GF_RT_DECL(name)
#define GF_RT_BEGIN(name)
#define GF_RT_END(name)
#define GF_RT_FLUSH(slot, name)
#endif

// shell-map and window codes
constexpr int32_t S_READABLE = -1;
constexpr int32_t S_BYSTANDER = -2;
constexpr int32_t S_UNFILLED = -3;
constexpr int32_t S_HOLE = -4;   // in D, not on a front list
constexpr int32_t S_FRONT = -5;  // in D, on the next front list

// ---------------------------------------------------------------------------
// storage types: arithmetic is FP64, storage binary32 or binary16

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

template <typename TS> __device__ inline TS to_storage(double v);
template <> __device__ inline float to_storage<float>(double v) { return (float)v; }
template <> __device__ inline __half to_storage<__half>(double v) {
    return __ushort_as_half(f64_to_f16_bits(v));
}

// ---------------------------------------------------------------------------
// group (G lanes) reductions

// Groups reduce with DPP lane moves inside a row of 16 lanes (swap
// neighbours, swap pairs within a quad, mirror the two quads of 8, mirror the
// row): VALU operand modifiers instead of round trips through the LDS
// crossbar; the steps across rows (groups of 32 and 64) use shuffles.  Every
// step pairs lanes symmetrically, so all lanes of the group end with the same
// value.
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror: lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // row_mirror: lane i <-> 15 - i within 16

template <int CTRL> __device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ inline double dpp_d(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

struct OpSum {
    __device__ static double d(double a, double b) { return a + b; }
};
struct OpMin {
    __device__ static double d(double a, double b) { return fmin(a, b); }
    __device__ static int i(int a, int b) { return min(a, b); }
};

template <int G, typename Op> __device__ inline double greduce(double v) {
    static_assert(G == 4 || G == 8 || G == 16 || G == 32 || G == 64, "group width");
    v = Op::d(v, dpp_d<kDppXor1>(v));
    v = Op::d(v, dpp_d<kDppXor2>(v));
    if constexpr (G >= 8) v = Op::d(v, dpp_d<kDppHalfMirror>(v));
    if constexpr (G >= 16) v = Op::d(v, dpp_d<kDppMirror>(v));
    if constexpr (G >= 32) v = Op::d(v, __shfl_xor(v, 16, G));
    if constexpr (G >= 64) v = Op::d(v, __shfl_xor(v, 32, G));
    return v;
}

template <int G> __device__ inline double gsum(double v) { return greduce<G, OpSum>(v); }
template <int G> __device__ inline double gmin(double v) { return greduce<G, OpMin>(v); }
template <int G> __device__ inline int gmin_i(int v) {
    v = min(v, dpp_i<kDppXor1>(v));
    v = min(v, dpp_i<kDppXor2>(v));
    if constexpr (G >= 8) v = min(v, dpp_i<kDppHalfMirror>(v));
    if constexpr (G >= 16) v = min(v, dpp_i<kDppMirror>(v));
    if constexpr (G >= 32) v = min(v, __shfl_xor(v, 16, G));
    if constexpr (G >= 64) v = min(v, __shfl_xor(v, 32, G));
    return v;
}

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

// Wavefront-aggregated appends and counts: one atomic per wavefront instead of
// one per lane (same-address atomics serialise).  Every lane of the wavefront
// that is executing must make the call.
__device__ inline int wave_append(bool want, int *counter) {
    const unsigned long long m = __ballot(want);
    if (m == 0ull) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, (int)__popcll(m));
    base = __shfl(base, leader, 64);
    const int rank = (int)__popcll(m & ((1ull << lane) - 1ull));
    return want ? base + rank : -1;
}

__device__ inline void wave_count(bool pred, int *counter) {
    const unsigned long long m = __ballot(pred);
    if (m != 0ull && lane_id() == __ffsll((long long)m) - 1) atomicAdd(counter, (int)__popcll(m));
}

// sum / maximum over the wavefront, added to an LDS counter by one lane
__device__ inline void wave_add(int v, int *counter) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (v != 0 && lane_id() == 0) atomicAdd(counter, v);
}
__device__ inline void wave_max(int v, int *counter) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    if (v != 0 && lane_id() == 0) atomicMax(counter, v);
}

// q = i / d for 0 <= i < 2^20 and 0 < d < 2^20, from a binary32 reciprocal
// r = 1 / d: the estimate is within one of the quotient and one step fixes it
__device__ inline int div_small(int i, int d, float r) {
    int q = (int)((float)i * r);
    const int m = i - q * d;
    q += (m >= d ? 1 : 0) - (m < 0 ? 1 : 0);
    return q;
}

// readable at shell k: -1 (readable from the start) or filled in a shell < k
__device__ inline bool readable(int32_t s, int k) { return (unsigned)(s + 1) <= (unsigned)k; }

// ---------------------------------------------------------------------------
// Persistent launches without a cooperative dispatch.  The kernels are
// launched as ordinary grids sized to what the device holds at once (the
// cooperative dispatch costs ~17 us more per launch here).  Residency is then
// not promised, so the workgroups that take part are discovered at start-up:
// each one takes a ticket on its XCD group's join word; one leader waits until
// every launched workgroup has joined, or at most join_ticks of the 100 MHz
// constant clock, and closes the poll.  A workgroup that joins after the close
// leaves at once, so every barrier waits only for workgroups that have run,
// hence are resident.  Join words cannot be cleared after a launch (a late
// workgroup may still add to them), so the host deals out kLaunchSlots sets in
// a ring and each launch clears the next launch's set.

// The XCD this workgroup runs on: the hardware XCC id (bits 3:0 of the
// XCC_ID register); workgroups on one XCD share its L2.
__device__ __attribute__((always_inline)) inline int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & (kXcd - 1));
}

struct GridInfo {
    int lw;  // logical index of this workgroup among those taking part
    int n;   // workgroups taking part
    int x;   // XCD group: the XCD the workgroup runs on (hardware XCC id)
};
// what the barriers need, kept in LDS rather than registers: workgroups
// taking part in this workgroup's group, groups with at least one
__shared__ int s_grid_shape[2];

struct LaunchSync {
    unsigned epoch;  // a number the host never reuses for the workspace, never 0
    int slot;        // join-word set of this launch, host ring 0, 1, 2, 0, ...
    int join_ticks;  // longest wait for the launched workgroups to join
};

// Start-up: join, then the leader zeroes the control block (but the join
// words and the published epoch) and the caller's accumulated outputs,
// records the groups' sizes and publishes the epoch; the others wait for it
// before touching any of them.  Returns false in a workgroup that does not
// take part: it must return at once.  Logical indices are consecutive within
// an XCD group, so contiguous ranges of pixels or tiles stay in one L2.
__device__ __attribute__((always_inline)) bool launch_start(int32_t *ctl, const LaunchSync &ls, GridInfo &gi, int32_t *z1, int n1,
                             int32_t *z2, int n2, int32_t *z3, int n3) {
    __shared__ int s_role;  // 1 leader, 0 taking part, -1 not taking part
    __shared__ int s_ticket;
    __shared__ int s_ok;    // 0 after a (never expected) start-up timeout
    __shared__ int s_nx[kXcd];
    const int tid = (int)threadIdx.x, nt = (int)blockDim.x;
    const int x = xcc_id();
    const int slot = ls.slot, next = (ls.slot + 1) % kLaunchSlots;
    if (tid == 0) {
        unsigned *tk = reinterpret_cast<unsigned *>(&ctl[xw(x, XF_TICKET + slot)]);
        const unsigned t = __hip_atomic_fetch_add(tk, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int role = 0;
        if (t & kClosed) {
            role = -1;
        } else if (t == 0u) {
            unsigned *lead = reinterpret_cast<unsigned *>(&ctl[G_LEAD + slot]);
            if (__hip_atomic_fetch_add(lead, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                role = 1;
        }
        s_role = role;
        s_ok = 1;
        s_ticket = (int)(t & (kClosed - 1u));
    }
    __syncthreads();
    if (s_role < 0) return false;
    if (s_role == 1) {
        if (tid == 0) {
            const long long t0 = wall_clock64();
            for (;;) {
                unsigned joined = 0;
#pragma unroll
                for (int y = 0; y < kXcd; ++y)
                    joined += __hip_atomic_load(reinterpret_cast<unsigned *>(&ctl[xw(y, XF_TICKET + slot)]),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                              (kClosed - 1u);
                if (joined >= gridDim.x || wall_clock64() - t0 > (long long)ls.join_ticks) break;
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int y = 0; y < kXcd; ++y)
                s_nx[y] = (int)(__hip_atomic_fetch_or(reinterpret_cast<unsigned *>(&ctl[xw(y, XF_TICKET + slot)]),
                                                      kClosed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                                (kClosed - 1u));
        }
        for (int i = tid; i < kCtlWords; i += nt) {
            const int f = i % kXStride;
            const bool join_word = (i < kXcd * kXStride && f >= XF_TICKET && f < XF_TICKET + kLaunchSlots) ||
                                   (i >= G_LEAD && i < G_LEAD + kLaunchSlots);
            if (i != G_READY && !join_word && (i < G_NX || i >= G_NX + kXcd)) ctl[i] = 0;
        }
        for (int i = tid; i < n1; i += nt) z1[i] = 0;
        for (int i = tid; i < n2; i += nt) z2[i] = 0;
        for (int i = tid; i < n3; i += nt) z3[i] = 0;
        __syncthreads();
        if (tid < kXcd) {
            ctl[xw(tid, XF_TICKET + next)] = 0;
            ctl[G_NX + tid] = s_nx[tid];
        }
        if (tid == 0) ctl[G_LEAD + next] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(&ctl[G_READY], (int32_t)ls.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (tid == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(&ctl[G_READY], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != (int32_t)ls.epoch) {
            if (++spins == kSpinLimit) {  // never expected: leave (the barriers then time out)
                s_ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
        for (int y = 0; y < kXcd; ++y) s_nx[y] = __hip_atomic_load(&ctl[G_NX + y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (!s_ok) return false;
    int n = 0, off = 0, groups = 0;
#pragma unroll
    for (int y = 0; y < kXcd; ++y) {
        if (y < x) off += s_nx[y];
        n += s_nx[y];
        groups += s_nx[y] > 0 ? 1 : 0;
    }
    gi.lw = __builtin_amdgcn_readfirstlane(off + s_ticket);  // uniform: scalar registers
    gi.n = __builtin_amdgcn_readfirstlane(n);
    gi.x = x;
    if (tid == 0) {
        s_grid_shape[0] = s_nx[x];
        s_grid_shape[1] = groups;
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// grid barrier over the workgroups taking part.  Arrivals are counted per XCD
// group first, then per group, so no counter sees more than
// max(n / 8, 8) serialised atomics.  A group is the set of workgroups on one
// XCD, which share that XCD's L2: every wave first waits until its own
// stores and atomics are acknowledged (they are then in the L2), so when the
// group's last workgroup arrives, one agent-scope release by it (an L2
// write-back) publishes the stores of the whole group, instead of one
// write-back per workgroup.  Waiting is a relaxed spin (an acquire load would
// invalidate the caches on every iteration) followed by one acquire.

__device__ __attribute__((always_inline)) void grid_sync(int32_t *ctl, const GridInfo &gi) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are in the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned x = (unsigned)gi.x;
        const unsigned per_group = (unsigned)s_grid_shape[0];
        const unsigned groups = (unsigned)s_grid_shape[1];
        unsigned *gen = (unsigned *)&ctl[G_GEN];
        unsigned *top = (unsigned *)&ctl[G_TOP];
        unsigned *grp = (unsigned *)&ctl[xw((int)x, XF_BAR)];
        const unsigned g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);  // the load completes before the arrival
        const unsigned a = __hip_atomic_fetch_add(grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool last = false;
        if (a == per_group - 1) {
            // every workgroup of the group has its stores in this L2: write it back
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            // the reset must be published before the group arrives at the top
            __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const unsigned b =
                __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = (b == groups - 1);
        }
        if (last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                if (++spins == kSpinLimit) {  // never expected: report and leave
                    __hip_atomic_store(&ctl[G_TIMEOUT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Grid barrier that also sums two per-workgroup values: a (the totals stay
// below 2^32) and a flag (the number of workgroups that raise it).  Arrivals,
// flag count and sum share one 64-bit word per XCD group and one at the top
// (16 | 16 | 32 bits); the last arriver publishes the totals in the same
// 64-bit word as the new generation, so no workgroup loads them afterwards.
struct SyncSum {
    unsigned a;
    unsigned flags;
};

__device__ __attribute__((always_inline)) SyncSum grid_sync_sum(int32_t *ctl, const GridInfo &gi, unsigned a, bool flag) {
    __shared__ unsigned long long s_word;
    typedef unsigned long long u64;
    constexpr u64 kLow48 = (1ull << 48) - 1ull;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores are in the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned x = (unsigned)gi.x;
        const u64 per_group = (u64)s_grid_shape[0];
        const u64 groups = (u64)s_grid_shape[1];
        u64 *gen = reinterpret_cast<u64 *>(&ctl[G_GEN2]);
        u64 *top = reinterpret_cast<u64 *>(&ctl[G_TOP2]);
        u64 *grp = reinterpret_cast<u64 *>(&ctl[xw((int)x, XF_SUM)]);
        const u64 g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 48;
        __builtin_amdgcn_s_waitcnt(0);  // the load completes before the arrival
        const u64 add = (1ull << 48) | ((u64)(flag ? 1u : 0u) << 32) | (u64)a;
        const u64 prior = __hip_atomic_fetch_add(grp, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u64 word = 0;
        bool have = false;
        if ((prior >> 48) == per_group - 1) {
            // every workgroup of the group has its stores in this L2: write it back
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const u64 gsum = (prior + add) & kLow48;
            __hip_atomic_store(grp, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const u64 tadd = (1ull << 48) | gsum;
            const u64 tprior = __hip_atomic_fetch_add(top, tadd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((tprior >> 48) == groups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(top, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                word = (((g + 1ull) & 0xffffull) << 48) | ((tprior + tadd) & kLow48);
                __hip_atomic_store(gen, word, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                have = true;
            }
        }
        if (!have) {
            unsigned spins = 0;
            for (;;) {
                word = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((word >> 48) != g) break;
                if (++spins == kSpinLimit) {  // never expected: report, publish nothing
                    __hip_atomic_store(&ctl[G_TIMEOUT], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    word = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_word = word;
    }
    __syncthreads();
    const u64 w = s_word;
    return SyncSum{(unsigned)(w & 0xffffffffull), (unsigned)((w >> 32) & 0xffffull)};
}

__device__ inline int ld_ctl(const int32_t *ctl, int i) {
    return __hip_atomic_load(&ctl[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int sum_x(const int32_t *ctl, int field) {
    int s = 0;
#pragma unroll
    for (int x = 0; x < kXcd; ++x) s += ld_ctl(ctl, xw(x, field));
    return s;
}

__device__ inline int max_x(const int32_t *ctl, int field) {
    int s = 0;
#pragma unroll
    for (int x = 0; x < kXcd; ++x) s = max(s, ld_ctl(ctl, xw(x, field)));
    return s;
}

// ball offsets {(n, m): 0 < n^2 + m^2 <= eps^2}, m ascending then n, and the
// reciprocal distances 1/|(n, m)| (the rotation preserves them)
__device__ __attribute__((always_inline)) void build_offsets(double eps, short2 *off, double *rinv, int *T) {
    if (threadIdx.x == 0) {
        int R = (int)floor(eps);
        int cnt = 0;
        for (int m = -R; m <= R; ++m)
            for (int n = -R; n <= R; ++n) {
                int r2 = n * n + m * m;
                if (r2 == 0 || (double)r2 > eps * eps) continue;
                if (cnt < kMaxOffsets) {
                    off[cnt] = make_short2((short)n, (short)m);
                    rinv[cnt] = 1.0 / sqrt((double)r2);
                }
                ++cnt;
            }
        *T = cnt < kMaxOffsets ? cnt : kMaxOffsets;
        // padding up to the table size: far outside any image or window (never
        // readable) and of weight 0, so a group reads G * lanes entries unchecked
        for (int t = cnt; t < kMaxOffsets; ++t) {
            off[t] = make_short2((short)kPadOffset, (short)kPadOffset);
            rinv[t] = 0.0;
        }
    }
}

// rotated offset R(n, m), R taking (0, 1) to g/|g| (Sec. 3.1), evaluated as
// ox = n*s + m*c, oy = m*s - n*c with no fused operations
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

// bilinear support of a ghost point at offset (ox, oy) from (X, Y): the pixels
// with a nonzero basis value (|q - p|_inf < 1, eqn:bilinearDef)
struct Support {
    int x0, x1, y0, y1;  // x1 == x0 / y1 == y0 on a lattice line
    double wx0, wx1, wy0, wy1;
};

__device__ inline Support support_of(int X, int Y, double ox, double oy) {
    Support s;
    double fx = floor(ox), fy = floor(oy);
    bool ex = (ox == fx), ey = (oy == fy);
    s.x0 = X + (int)fx;
    s.y0 = Y + (int)fy;
    s.x1 = s.x0 + (ex ? 0 : 1);
    s.y1 = s.y0 + (ey ? 0 : 1);
    if (ex) { s.wx0 = 1.0; s.wx1 = 0.0; } else { double f = ox - fx; s.wx0 = 1.0 - f; s.wx1 = f; }
    if (ey) { s.wy0 = 1.0; s.wy1 = 0.0; } else { double f = oy - fy; s.wy0 = 1.0 - f; s.wy1 = f; }
    return s;
}

}  // namespace gfk
