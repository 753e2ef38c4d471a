// The triangular solves of Eq. 1 on one compute unit, for deep, narrow
// dependency graphs (few rows per dependency level, thousands of levels).
//
// There, every level costs one hand-off between rows, and a hand-off through
// the L2 of an XCD takes about 0.23 us on MI355X; through the LDS of one CU
// it takes a few dozen cycles.  A CU has too little issue for a wavefront per
// row (a row's running subtraction is one lane's serial chain, so a
// wavefront would spend ~12 cycles of its SIMD per term), so here a lane
// owns a row: one workgroup of 16 wavefronts takes the level order in slices
// of 64 consecutive positions, wavefront w the slices w, w + 16, w + 32, ...,
// and each lane walks its row's entries in the fixed order (forward:
// ascending column; backward: right to left, then the division), advancing
// as the values it needs become known, 8 entries per load.
//
// Hand-off: the value of position p (its row's result) goes at once to an
// LDS ring slot p mod kRing, and to global memory (the output vector) when the
// wavefront has finished the slice; the ring slot is tagged with
// p under a sequence protocol (tag set to "being written", value, tag = p);
// a reader reads tag, value, tag and takes the value only if both tags equal
// the position it wants.  A smaller tag means the value is not known yet; a
// larger one means the slot was reused by position q + kRing or later, and
// then the value is read from global memory with an agent-scope load.  That
// read is safe: positions q and q + kRing lie in slices kRing / 64 apart, a
// multiple of the 16 wavefronts, so the same wavefront produced both, and a
// wavefront waits for all of its earlier stores before it starts a slice.
//
// Every position depends only on earlier positions, all 16 wavefronts are
// resident (one workgroup) and each takes its slices in order, so the
// smallest unfinished position is always on a running wavefront whose
// inputs are known: no deadlock.  Waits are bounded by the watchdog; on a
// timeout unfinished rows publish a quiet NaN so that the others drain.
#include "kernels.h"

namespace tpilu {

constexpr int kCuWaves = 16;
constexpr int kRing = 4096;  // positions kept in LDS; kRing / 64 must be a multiple of kCuWaves
constexpr int kCuChunk = 16;  // entries of a row per load
static_assert((kRing / kWave) % kCuWaves == 0, "ring reuse must stay within one wavefront");

typedef __attribute__((address_space(3))) volatile double LdsF64;
typedef __attribute__((address_space(3))) volatile int32_t LdsI32;

template <bool kBackward>
__global__ __launch_bounds__(1024) void k_solve_cu(PatDev P, const int32_t* __restrict__ Pq,
                                                   const double* __restrict__ F, const double* __restrict__ in,
                                                   double* out, Ctl* ctl, uint64_t spin_limit) {
    __shared__ double ring_v[kRing];
    __shared__ int32_t ring_t[kRing];
    LdsF64* rv = (LdsF64*)ring_v;
    LdsI32* rt = (LdsI32*)ring_t;
    const int lane = lane_id();
    const int32_t wave = uniform((int32_t)(threadIdx.x >> 6));
    const int32_t n = P.n;
    const int32_t* perm = kBackward ? P.permU : P.permL;
    const int64_t tr0 = kBackward ? 2 * (int64_t)n : 0;
    for (int r = threadIdx.x; r < kRing; r += blockDim.x) rt[r] = -1;
    __syncthreads();
    bool aborted = false;
    for (int32_t s = wave; (int64_t)s * kWave < n; s += kCuWaves) {
        // every store of this wavefront's earlier slices has completed (the
        // ring reuse rule above relies on it)
        __builtin_amdgcn_s_waitcnt(0);
        const int32_t p = s * kWave + lane;
        const bool valid = p < n;
        int32_t i = 0;
        int64_t e = 0, left = 0;
        double acc = 0.0, fii = 1.0;
        if (valid) {
            i = perm ? perm[p] : (kBackward ? n - 1 - p : p);
            const int64_t d = P.diagF[i];
            if (kBackward) {
                e = P.rpF[i + 1] - 1;  // right to left: slots e, e-1, ..., d+1
                left = e - d;
                acc = in[i];
                fii = F[d];
            } else {
                e = P.rpF[i];
                left = d - e;
                acc = sanitize_input(in[i], ctl);
            }
        }
        trace_mark_lane(P.trace, tr0 + i, valid);
        bool done = !valid;
        double res = 0.0;  // the row's result, stored to global memory when the slice ends
        double fv[kCuChunk];
        int32_t qv[kCuChunk];
#pragma unroll
        for (int k = 0; k < kCuChunk; ++k) {
            fv[k] = 0.0;
            qv[k] = 0;
        }
        int32_t cnt = 0, u = 0;
        uint32_t polls = 0;
        uint64_t t0 = 0;
        for (;;) {
            bool prog = false;
            if (!done) {
                if (u == cnt && left > 0) {  // the next entries of the row
                    cnt = (int32_t)min<int64_t>(left, kCuChunk);
#pragma unroll
                    for (int k = 0; k < kCuChunk; ++k) {
                        if (k < cnt) {
                            const int64_t slot = kBackward ? e - k : e + k;
                            fv[k] = F[slot];
                            qv[k] = Pq[slot];
                        }
                    }
                    e = kBackward ? e - cnt : e + cnt;
                    left -= cnt;
                    u = 0;
                }
                // advance over the entries whose values are known, stopping at
                // the first one that is not: a round in which nothing arrived
                // costs one ring read per waiting lane
                while (u < cnt) {
                    const int32_t q = qv[u];
                    const int32_t slot = q & (kRing - 1);
                    const int32_t t1 = rt[slot];
                    const double v = rv[slot];
                    const int32_t t2 = rt[slot];
                    double x;
                    if (t1 == q && t2 == q) {
                        x = v;
                        jitter((uint32_t)q);
                    } else if (t1 > q) {  // reused by a later position: q is in global memory
                        const int32_t row = perm ? perm[q] : (kBackward ? n - 1 - q : q);
                        x = as_f64(ld_coherent(out + row));
                    } else {
                        break;
                    }
                    acc = acc - fv[u] * x;
                    ++u;
                    prog = true;
                }
                if (u == cnt && left == 0) {
                    const double r = kBackward ? acc / fii : acc;
                    res = r;
                    const int32_t slot = p & (kRing - 1);
                    jitter((uint32_t)p);
                    rt[slot] = -2;  // being written
                    rv[slot] = r;
                    rt[slot] = p;
                    trace_mark_lane(P.trace, tr0 + n + i, true);
                    done = true;
                    prog = true;
                }
            }
            if (__all(done)) break;
            if (__any(prog)) {
                polls = 0;
                continue;
            }
            // watchdog over rounds in which no lane advanced
            ++polls;
            if ((polls & 255u) == 0u) {
                bool stop = (polls & 4095u) == 0u && ld_u32_coherent(&ctl->abort) != 0u;
                const uint64_t now = wall_clock64();
                if (polls == 256u) {
                    t0 = now;
                } else if (now - t0 > spin_limit) {
                    if (lane == 0) {
                        atomicOr(&ctl->status, kStTimeout);
                        __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    stop = true;
                }
                if (__any(stop)) {
                    aborted = true;
                    break;
                }
            }
        }
        // Results reach global memory when the whole slice is done.  On this
        // architecture stores and loads share one completion counter, so a
        // store issued in the rounds above would make every later wait for a
        // load wait for the store's acknowledgement from memory as well
        // (about 1 us, once per dependency level); the LDS ring already
        // handed the values over.
        if (valid && done) out[i] = res;
        if (aborted) {
            // release every row that might be waited on: unfinished rows of
            // this and later slices publish a quiet NaN
            for (int32_t s2 = s; (int64_t)s2 * kWave < n; s2 += kCuWaves) {
                const int32_t p2 = s2 * kWave + lane;
                if (p2 >= n || (s2 == s && done)) continue;
                const int32_t i2 = perm ? perm[p2] : (kBackward ? n - 1 - p2 : p2);
                out[i2] = as_f64(kQNaN);
                const int32_t slot = p2 & (kRing - 1);
                rt[slot] = -2;
                rv[slot] = as_f64(kQNaN);
                rt[slot] = p2;
            }
            break;
        }
    }
}

// per F slot: the level-order position of the row its column names
// (strict lower slots: positions of the forward order; upper slots: of the
// backward order; diagonal slots: unused)
__global__ void k_dep_positions(int32_t n, const int64_t* __restrict__ rpF, const int32_t* __restrict__ ciF,
                                const int32_t* __restrict__ diagF, const int32_t* __restrict__ iposL,
                                const int32_t* __restrict__ iposU, int32_t* __restrict__ Pq) {
    for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
        const int64_t a = rpF[i], b = rpF[i + 1], d = diagF[i];
        for (int64_t s = a + threadIdx.x; s < b; s += blockDim.x) {
            const int32_t c = ciF[s];
            Pq[s] = s < d ? iposL[c] : (s > d ? iposU[c] : 0);
        }
    }
}

__global__ void k_inverse_perm(int32_t n, const int32_t* __restrict__ perm, int32_t* __restrict__ ipos) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) ipos[perm[p]] = p;
}

hipError_t launch_dep_positions(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF,
                                const int32_t* permL, const int32_t* permU, int32_t* iposL, int32_t* iposU,
                                int32_t* Pq, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_inverse_perm, dim3((n + 255) / 256), dim3(256), 0, s, n, permL, iposL);
    hipLaunchKernelGGL(k_inverse_perm, dim3((n + 255) / 256), dim3(256), 0, s, n, permU, iposU);
    hipLaunchKernelGGL(k_dep_positions, dim3(std::min(n, 65536)), dim3(256), 0, s, n, rpF, ciF, diagF, iposL,
                       iposU, Pq);
    return hipGetLastError();
}

hipError_t launch_solve_cu(const PatDev& P, const int32_t* Pq, const double* f_val, const double* in, double* out,
                           bool backward, Ctl* ctl, uint64_t spin_limit, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (backward)
        hipLaunchKernelGGL(k_solve_cu<true>, dim3(1), dim3(kCuWaves * kWave), 0, s, P, Pq, f_val, in, out, ctl,
                           spin_limit);
    else
        hipLaunchKernelGGL(k_solve_cu<false>, dim3(1), dim3(kCuWaves * kWave), 0, s, P, Pq, f_val, in, out, ctl,
                           spin_limit);
    return hipGetLastError();
}

}  // namespace tpilu
