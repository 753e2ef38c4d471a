// Device-side building blocks shared by the gfx950 kernels.
//
// Cross-wavefront hand-off without flags.  Every value a persistent kernel
// hands from one row to another (entries of F, entries of x and y in the
// triangular solves, adjoints in the reverse sweep) lives in an output array
// that is first filled with a reserved signalling-NaN bit pattern, kPending.
// The producing wavefront overwrites each slot exactly once with its final
// value; a consumer polls the slot itself until it no longer reads kPending.
// No arithmetic result is ever a signalling NaN, so a value that is not
// kPending is the final one: no separate completion flag, no release/acquire
// fence and no second round trip are needed, and every slot is its own
// message.
//
// Coherence across the eight XCDs (each has a private L2): the producer
// writes with agent-scope atomic stores (write-through to the memory-side
// coherence point); a consumer first tries a plain load (it may hit a cache;
// a non-kPending answer is final because the slot holds only kPending or the
// final value during the kernel, and caches are invalidated at kernel
// start), and only if that still shows kPending polls with agent-scope
// atomic loads, which bypass the non-coherent caches.
//
// Every wait is bounded: after a wall-clock budget it sets the control
// block's abort word and the TIMEOUT bit and returns a quiet NaN; every other
// wait notices the abort word within a few polls and gives up too, so all
// waves always drain.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpilu {

constexpr uint64_t kPending = 0x7FF4A5A5A5A5A5A5ull;  // reserved sNaN payload: "not written yet"
constexpr uint64_t kQNaN = 0x7FF8000000000000ull;     // default quiet NaN
constexpr int kWave = 64;

// status bits (sticky until read by the host)
constexpr uint32_t kStTimeout = 1u;
constexpr uint32_t kStReservedNaN = 2u;

// Counters of the row kernels' level-order positions, each on its own 256-byte
// line: one counter serialises its atomics (about 11 ns each), several on
// separate lines proceed in parallel.
constexpr int kTicketParts = 8;
constexpr int kTicketStride = 64;  // uint32 words between two counters

struct Ctl {
    uint32_t ticket;        // next task of the running persistent kernel
    uint32_t abort;         // set once any wait ran out
    uint32_t status;        // kSt* bits
    uint32_t pad;
    unsigned long long bad_row;  // smallest row with a zero final pivot, or ~0
    uint32_t leader;        // 1 + the XCD a one-XCD kernel runs on, 0 = not chosen yet
    uint32_t pad2[57];
    uint32_t part[kTicketParts * kTicketStride];  // position counters (next_pos)
};

// Race check build (compiled with -DTPILU_JITTER, never the product): a
// pseudo-random pause of 0 to 31 x 64 cycles, the same for the whole
// wavefront, before every publishing store and after every coherent load, so
// that hand-offs happen in orders and at times the normal timing never
// produces.  The results must keep their bits.
#ifdef TPILU_JITTER
__device__ __forceinline__ void jitter(uint32_t salt) {
    uint32_t h = (uint32_t)wall_clock64() * 0x9E3779B9u ^ (blockIdx.x + 0x7F4A7C15u) * 0x85EBCA6Bu ^ salt;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    const uint32_t r = __builtin_amdgcn_readfirstlane(h) & 31u;
    for (uint32_t k = 0; k < r; ++k) __builtin_amdgcn_s_sleep(1);
}
#else
__device__ __forceinline__ void jitter(uint32_t) {}
#endif

// The update of Eq. 6b, f - l * u: by default the product and the difference
// are rounded on their own; with kFused as one fused multiply-add (a single
// rounding of the exact f - l * u).  Negating l is exact, so both forms
// are fixed by IEEE-754 alone.
template <bool kFused>
__device__ __forceinline__ double ikj_update(double f, double l, double u) {
    if constexpr (kFused) return __builtin_fma(-l, u, f);
    else return f - l * u;
}

__device__ __forceinline__ uint64_t as_u64(double d) { return __builtin_bit_cast(uint64_t, d); }
__device__ __forceinline__ double as_f64(uint64_t u) { return __builtin_bit_cast(double, u); }

__device__ __forceinline__ uint64_t ld_coherent(const double* p) {
    const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    jitter((uint32_t)v);
    return v;
}
__device__ __forceinline__ uint64_t ld_cached(const double* p) {
    return __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void st_publish(double* p, double v) {
    jitter((uint32_t)(uintptr_t)p);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), as_u64(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_u32_coherent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll slot p until it holds a final value.  `first` is a value already read
// from p (for instance by a prefetch); it is returned at once if final.
// `limit` is the wait budget in wall-clock ticks (s_memrealtime).
__device__ __noinline__ double wait_final_slow(const double* p, Ctl* ctl, uint64_t limit) {
    uint32_t n = 0;
    uint64_t t0 = 0;
    for (;;) {
        uint64_t v = ld_coherent(p);
        if (v != kPending) return as_f64(v);
        if ((n & 31u) == 0u) {
            if ((n & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u) return as_f64(kQNaN);
            const uint64_t now = wall_clock64();
            if (n == 0) {
                t0 = now;
            } else if (now - t0 > limit) {
                atomicOr(&ctl->status, kStTimeout);
                __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return as_f64(kQNaN);
            }
        }
        ++n;
    }
}

__device__ __forceinline__ double wait_final(const double* p, uint64_t first, Ctl* ctl,
                                             uint64_t limit) {
    if (first != kPending) return as_f64(first);
    return wait_final_slow(p, ctl, limit);
}

__device__ __forceinline__ double wait_final(const double* p, Ctl* ctl, uint64_t limit) {
    return wait_final(p, ld_cached(p), ctl, limit);
}

// Make every staged value of a chunk final: the pending ones are re-read
// together, one round trip per round, until none is left; after a timeout or
// an abort they become quiet NaNs.  Unused entries must hold a final value
// and a valid index.
template <int K>
__device__ __forceinline__ void settle(const double* v, const int32_t (&idx)[K], uint64_t (&val)[K], int32_t B,
                                       int32_t col, Ctl* ctl, uint64_t limit) {
    uint32_t n = 0;
    uint64_t t0 = 0;
    for (;;) {
        bool pend = false;
#pragma unroll
        for (int u = 0; u < K; ++u) pend = pend || val[u] == kPending;
        if (!pend) return;
        uint64_t nv[K];
#pragma unroll
        for (int u = 0; u < K; ++u) nv[u] = ld_coherent(v + (int64_t)idx[u] * B + col);
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (val[u] == kPending) val[u] = nv[u];
        if ((n & 31u) == 31u) {
            bool stop = (n & 255u) == 255u && ld_u32_coherent(&ctl->abort) != 0u;
            const uint64_t now = wall_clock64();
            if (n == 31u) {
                t0 = now;
            } else if (now - t0 > limit) {
                atomicOr(&ctl->status, kStTimeout);
                __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                stop = true;
            }
            if (stop) {
#pragma unroll
                for (int u = 0; u < K; ++u)
                    if (val[u] == kPending) val[u] = kQNaN;
                return;
            }
        }
        ++n;
    }
}

// A caller-supplied value that happens to carry the reserved pattern is
// replaced by the quiet NaN (and reported), so it can never be mistaken for
// "not written yet".
__device__ __forceinline__ double sanitize_input(double v, Ctl* ctl) {
    if (as_u64(v) == kPending) {
        atomicOr(&ctl->status, kStReservedNaN);
        return as_f64(kQNaN);
    }
    return v;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// One wavefront per workgroup everywhere a kernel uses wave_sync: the
// barrier then only orders the wave's own LDS traffic.
__device__ __forceinline__ void wave_sync() { __syncthreads(); }

// Optional per-row timeline (wall-clock ticks): the slot for "started" and
// the slot for "published" are chosen by each kernel.
__device__ __forceinline__ void trace_mark(unsigned long long* trace, int64_t slot) {
    if (trace && lane_id() == 0) trace[slot] = wall_clock64();
}

// per-lane form of trace_mark (the lane's own row)
__device__ __forceinline__ void trace_mark_lane(unsigned long long* trace, int64_t slot, bool on) {
    if (trace && on) trace[slot] = wall_clock64();
}

// Value that is the same in every lane, made visibly uniform (SGPR) for the
// compiler.  Only call with all lanes active.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Grab the next task index for the whole wave.  Lane 0 does the atomic and
// broadcasts it through LDS between two barriers: the barriers force every
// lane to be converged here, so the compiler cannot let lane 0 run ahead into
// the next task (a lane-0-only store at the end of a task followed by this
// lane-0-only atomic would otherwise be merged across the loop back-edge).
__device__ __forceinline__ uint32_t wave_ticket(Ctl* ctl) {
    __shared__ uint32_t s_ticket;
    __syncthreads();
    if (lane_id() == 0) s_ticket = atomicAdd(&ctl->ticket, 1u);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(s_ticket);
}

// Positions of a level order handed to wavefronts `group` consecutive ones at a
// time, the wavefront working through its group in order.  Groups are dealt
// round robin to `parts` counters (group g to counter g mod parts; wavefront
// w draws from counter w mod parts), so that wide levels are not held up by
// one counter.  Deadlock-free: a position only depends on earlier ones.  The
// smallest unfinished position is either held by a running wavefront, which
// has finished everything before it in its group and so is working on it,
// or not yet drawn; then every wavefront of its counter holds only smaller,
// finished positions of that counter (a counter deals in increasing order)
// and will draw it next.  Every counter has at least one wavefront
// (parts <= grid), and the waves that are not resident yet only wait for
// resident ones to finish, which needs nothing from them.
struct PosRun {
    uint32_t next = 0, end = 0;
};
__device__ __forceinline__ bool next_pos(Ctl* ctl, uint32_t n, uint32_t group, uint32_t parts, PosRun& r,
                                         uint32_t& pos) {
    if (r.next == r.end) {
        __shared__ uint32_t s_ticket;
        if (parts > gridDim.x) parts = gridDim.x;
        if (parts == 0) parts = 1;
        const uint32_t x = blockIdx.x % parts;
        __syncthreads();
        if (lane_id() == 0) s_ticket = atomicAdd(&ctl->part[x * kTicketStride], 1u);
        __syncthreads();
        const uint64_t v = __builtin_amdgcn_readfirstlane(s_ticket);
        const uint64_t first = (v * parts + x) * group;
        if (first >= n) return false;
        r.next = (uint32_t)first;
        r.end = (uint32_t)(first + group < n ? first + group : n);
    }
    pos = r.next++;
    return true;
}

__device__ __forceinline__ int64_t bcast_i64(int64_t v, int src) {
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(u), src);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(u >> 32), src);
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

__device__ __forceinline__ double bcast_lane(double v, int src) {
    uint64_t u = as_u64(v);
    uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(u), src);
    uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(u >> 32), src);
    return as_f64((static_cast<uint64_t>(hi) << 32) | lo);
}

// Communication scope of the hand-off protocol: across the whole device
// (agent-scope stores, written through to memory, and agent-scope loads),
// inside one XCD (ordinary stores, which stay in the XCD's L2, read back with
// agent-scope loads, which skip the CU's L1 and take a line the L2 holds
// dirty; measured on MI355X at about 0.5 us a round trip against about 0.9
// us device-wide), or inside one workgroup (all waves on one CU, whose caches
// are coherent for them).  A workgroup-scope load may hit the CU's L1 and then
// never sees a store from another CU.
enum class Scope { Device, Xcd, Workgroup };

template <Scope S>
__device__ __forceinline__ uint64_t ld_poll(const double* p) {
    if constexpr (S != Scope::Workgroup) return ld_coherent(p);
    const uint64_t v = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    jitter((uint32_t)v);
    return v;
}

template <Scope S>
__device__ __forceinline__ void st_final(double* p, double v) {
    if constexpr (S == Scope::Device) {
        st_publish(p, v);
    } else {
        jitter((uint32_t)(uintptr_t)p);
        __hip_atomic_store(reinterpret_cast<uint64_t*>(p), as_u64(v), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// XCD the calling wavefront runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ uint32_t xcd_id() {
    return static_cast<uint32_t>(__builtin_amdgcn_s_getreg(20 | (3 << 11))) & 0xFu;
}

// Membership of a one-XCD launch (single-wavefront workgroups): the first
// workgroup to get here names its own XCD, and only workgroups on that XCD
// take part; the others return at once.  Whatever order the hardware deals
// workgroups to XCDs in, the chosen one holds at least that first workgroup,
// so the work is always done.  ctl->leader is cleared before every launch.
__device__ __forceinline__ bool xcd_member(Ctl* ctl) {
    const uint32_t me = xcd_id() + 1u;
    uint32_t l = 0u;
    if (lane_id() == 0) {
        l = __hip_atomic_load(&ctl->leader, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (l == 0u) {
            uint32_t expected = 0u;
            l = __hip_atomic_compare_exchange_strong(&ctl->leader, &expected, me, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    ? me
                    : expected;
        }
    }
    return __builtin_amdgcn_readfirstlane(l) == me;
}

// Running subtraction s <- s - f_k * v_k for k = 0 .. cnt-1 in that order,
// where lane k holds f_k and the address of v_k (cnt <= 64).  The values are
// produced by other rows; the chain advances over every prefix of entries
// whose value is already final, so once the last value arrives only the rest
// of the chain is left to do.  While blocked, every round re-polls all of the
// chunk's pending entries at once (one round trip for all of them) with no
// pause between rounds: entries that land while the chain waits on an earlier
// one are then already in hand when it gets there.  Polling only the blocking
// entry, or pausing between rounds, measured slower.
// The bits are those of the plain sequential loop.  On a watchdog timeout or
// abort the result is a quiet NaN (the call then reports the timeout).
template <Scope S>
__device__ __forceinline__ double chain_sub(double s, int32_t cnt, double f, const double* src, Ctl* ctl,
                                            uint64_t limit) {
    const int lane = lane_id();
    const bool has = lane < cnt;
    uint64_t v = has ? ld_cached(src) : 0ull;
    bool ready = !has || v != kPending;
    double prod = (has && ready) ? f * as_f64(v) : 0.0;
    int32_t k = 0;
    uint32_t polls = 0;
    uint64_t t0 = 0;
    for (;;) {
        const uint64_t pend = ~__ballot(ready) & (k >= kWave ? 0ull : (~0ull << k));
        const int32_t stop = pend ? min((int32_t)__builtin_ctzll(pend), cnt) : cnt;
        for (; k < stop; ++k) s = s - bcast_lane(prod, k);
        if (k >= cnt) break;
        if (!ready) {
            v = ld_poll<S>(src);
            if (v != kPending) {
                ready = true;
                prod = f * as_f64(v);
            }
        }
        if ((polls & 31u) == 0u) {
            if ((polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u) return as_f64(kQNaN);
            const uint64_t now = wall_clock64();
            if (polls == 0) {
                t0 = now;
            } else if (now - t0 > limit) {
                if (lane_id() == 0) {
                    atomicOr(&ctl->status, kStTimeout);
                    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return as_f64(kQNaN);
            }
        }
        ++polls;
    }
    return s;
}

}  // namespace tpilu
