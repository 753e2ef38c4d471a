// Measuring the hand-off between two wavefronts, the cost that bounds every
// dependency-driven kernel of the library from below.
//
// Two wavefronts pass a counter back and forth through global memory with
// the same publish / poll primitives the persistent kernels use: on one XCD
// a plain store read back with agent-scope loads (the line stays in that
// XCD's L2), across XCDs an agent-scope store (written through) read back
// the same way.  Block 0 is the ping side; the first other block that
// finds itself on the required XCD (the same as block 0's, or another one)
// claims the pong side; every other block leaves at once.  Every wait is
// bounded by the watchdog budget: a wait that runs out sets the status word
// and ends both sides, so the launch always drains.
#include "kernels.h"

namespace tpilu {

struct ProbeBuf {
    uint32_t leader;   // 1 + XCD of block 0, 0 until known
    uint32_t claimed;  // pong side taken
    uint32_t status;   // 1 = a wait ran out
    uint32_t pad0[61];
    double a;          // ping -> pong, own 256-byte line
    double pad1[31];
    double b;          // pong -> ping, own line
    double pad2[31];
    unsigned long long ticks;  // wall-clock ticks of the timed rounds
};

constexpr int kProbeWarm = 32;  // untimed rounds first

template <Scope S>
__device__ __forceinline__ bool await_value(const double* p, double want, ProbeBuf* pb, uint64_t limit) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t n = 0;; ++n) {
        if (as_f64(ld_poll<S>(p)) == want) return true;
        if ((n & 63u) == 63u) {
            if (__hip_atomic_load(&pb->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
            if (wall_clock64() - t0 > limit) {
                __hip_atomic_store(&pb->status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
}

template <Scope S>
__global__ __launch_bounds__(64) void k_handoff(ProbeBuf* pb, int32_t rounds, int32_t same_xcd, uint64_t limit) {
    if (lane_id() != 0) return;  // one lane per side: the measured quantity is the hand-off itself
    const uint32_t me = xcd_id() + 1u;
    if (blockIdx.x == 0) {
        __hip_atomic_store(&pb->leader, me, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t t0 = 0;
        for (int32_t i = 1; i <= rounds + kProbeWarm; ++i) {
            if (i == kProbeWarm + 1) t0 = wall_clock64();
            st_final<S>(&pb->a, (double)i);
            if (!await_value<S>(&pb->b, (double)i, pb, limit)) return;
        }
        pb->ticks = wall_clock64() - t0;
        return;
    }
    // wait (bounded) until block 0 has named its XCD
    uint32_t lead = 0;
    const uint64_t t0 = wall_clock64();
    while ((lead = __hip_atomic_load(&pb->leader, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u) {
        if (wall_clock64() - t0 > limit) return;
    }
    if ((me == lead) != (same_xcd != 0)) return;
    uint32_t expected = 0u;
    if (!__hip_atomic_compare_exchange_strong(&pb->claimed, &expected, 1u, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT))
        return;
    for (int32_t i = 1; i <= rounds + kProbeWarm; ++i) {
        if (!await_value<S>(&pb->a, (double)i, pb, limit)) return;
        st_final<S>(&pb->b, (double)i);
    }
}

size_t probe_buf_bytes() { return sizeof(ProbeBuf); }

// buf: probe_buf_bytes() of device memory, zeroed by the caller; the result
// (ticks of `rounds` round trips, status) is read back from it by the caller
hipError_t launch_handoff(void* buf, int32_t rounds, bool same_xcd, uint64_t spin_limit, hipStream_t s) {
    ProbeBuf* pb = static_cast<ProbeBuf*>(buf);
    // 8 blocks per XCD: the one-XCD case always has a partner on block 0's XCD
    const dim3 grid(8 * kXcds);
    if (same_xcd)
        hipLaunchKernelGGL(k_handoff<Scope::Xcd>, grid, dim3(64), 0, s, pb, rounds, 1, spin_limit);
    else
        hipLaunchKernelGGL(k_handoff<Scope::Device>, grid, dim3(64), 0, s, pb, rounds, 0, spin_limit);
    return hipGetLastError();
}

void probe_read(const void* host_copy, unsigned long long* ticks, uint32_t* status) {
    const ProbeBuf* pb = static_cast<const ProbeBuf*>(host_copy);
    *ticks = pb->ticks;
    *status = pb->status;
}

}  // namespace tpilu
