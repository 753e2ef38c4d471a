// Phase II on gfx950: row-wise IKJ elimination (Eq. 2 read as running
// updates, Eqs. 6a/6b), bit-identical to the sequential order.
//
// The only order that fixes the bits is, per entry f_jt, its updates in
// ascending pivot h.  A persistent grid hands rows out in dependency-level
// order through atomic task counters (next_pos in dev_common.h), so a
// wavefront only ever waits on rows that some running wavefront already holds
// (no deadlock for any grid size).  One
// wavefront owns row j: it scatters A's row into an LDS working row indexed by
// F slot (fills +0.0), then for every pivot h < j of row j in ascending order
// divides f_jh by the final pivot f_hh and applies that pivot's updates
// f_jt <- f_jt - f_jh * f_ht in parallel over t (distinct targets).  The
// updates come from the schedule built in Phase I, so no search happens here.
// Pivot rows are read straight from the output array F, whose slots start as
// kPending and are overwritten once by their owner (see dev_common.h); the
// static parts of a group of pivots (diag slots, pair lists) and optimistic
// reads of their values are prefetched together so that a pivot only waits
// if its row is still being produced.  No MFMA: this is a sparse gather /
// scatter elimination, not a dense contraction.
#include "kernels.h"

namespace tpilu {

__global__ void k_fill_pending(double* __restrict__ p, int64_t n, Ctl* ctl, int reset_status) {
    if (blockIdx.x == 0 && threadIdx.x < kTicketParts) ctl->part[threadIdx.x * kTicketStride] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->ticket = 0;
        ctl->leader = 0;
        if (reset_status) {
            ctl->abort = 0;
            ctl->status = 0;
            ctl->bad_row = ~0ull;
        }
    }
    const double pend = as_f64(kPending);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = pend;
}

hipError_t launch_fill_pending(double* p, int64_t n, Ctl* ctl, bool reset_status, hipStream_t s) {
    int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(k_fill_pending, dim3(blocks), dim3(256), 0, s, p, n, ctl,
                       reset_status ? 1 : 0);
    return hipGetLastError();
}

// The same for a factorization: only the slots other rows wait on, those of
// U~ (diagonal to row end, every instance), get the marker; the l values
// pass between rows only inside their own row's wavefront, and every row
// writes its L~ part when it finishes.  A wavefront per row at a time.
__global__ void k_fill_pending_upper(double* __restrict__ F, int32_t n, const int64_t* __restrict__ rpF,
                                     const int32_t* __restrict__ diagF, int32_t batch, Ctl* ctl,
                                     int reset_status) {
    if (blockIdx.x == 0 && threadIdx.x < kTicketParts) ctl->part[threadIdx.x * kTicketStride] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->ticket = 0;
        ctl->leader = 0;
        if (reset_status) {
            ctl->abort = 0;
            ctl->status = 0;
            ctl->bad_row = ~0ull;
        }
    }
    const double pend = as_f64(kPending);
    const int32_t waves = (int32_t)(gridDim.x * (blockDim.x / kWave));
    for (int32_t j = (int32_t)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave); j < n; j += waves) {
        const int64_t a = (int64_t)diagF[j] * batch, b = rpF[j + 1] * batch;
        for (int64_t i = a + lane_id(); i < b; i += kWave) F[i] = pend;
    }
}

hipError_t launch_fill_pending_upper(double* f_val, int32_t n, const int64_t* rpF, const int32_t* diagF,
                                     int32_t batch, Ctl* ctl, bool reset_status, hipStream_t s) {
    const int blocks = std::max(1, std::min((n + 3) / 4, 8192));
    hipLaunchKernelGGL(k_fill_pending_upper, dim3(blocks), dim3(256), 0, s, f_val, n, rpF, diagF, batch, ctl,
                       reset_status ? 1 : 0);
    return hipGetLastError();
}

// Wait until pivot i of the staged group is final: its diagonal and every
// value f_ht it contributes.  Each polling round also refreshes the pending
// values of the next few pivots, so pivots whose rows finish while row j
// waits on an earlier one cost no further round trip of their own.  Final
// values are written back into the staged copies; after a watchdog timeout
// or an abort pivot i's diagonal is replaced by a quiet NaN.
constexpr int kLookahead = 16;

__device__ __forceinline__ void wait_pivot(const double* F, int32_t i, int32_t np,
                                           const int32_t* piv_dh, uint64_t* piv_u,
                                           const int32_t* piv_e, const int32_t* pr_q, uint64_t* pr_v,
                                           Ctl* ctl, uint64_t limit) {
    const int lane = lane_id();
    const int32_t xe = min(np, i + kLookahead);
    const int32_t ea = piv_e[i], eb = piv_e[i + 1], ee = piv_e[xe];
    uint32_t polls = 0;
    uint64_t t0 = 0;
    for (;;) {
        bool pend = false;
        for (int32_t x = i + lane; x < xe; x += kWave) {
            if (piv_u[x] == kPending) {
                const uint64_t v = ld_coherent(F + piv_dh[x]);
                if (v != kPending) piv_u[x] = v;
                else if (x == i) pend = true;
            }
        }
        for (int32_t e = ea + lane; e < ee; e += kWave) {
            if (pr_v[e] == kPending) {
                const uint64_t v = ld_coherent(F + pr_q[e]);
                if (v != kPending) pr_v[e] = v;
                else if (e < eb) pend = true;
            }
        }
        if (!__any(pend)) break;
        if ((polls & 31u) == 0u) {
            bool stop = false;
            if ((polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u) stop = true;
            const uint64_t now = wall_clock64();
            if (polls == 0) {
                t0 = now;
            } else if (now - t0 > limit) {
                if (lane == 0) {
                    atomicOr(&ctl->status, kStTimeout);
                    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                stop = true;
            }
            if (stop) {
                if (lane == 0) piv_u[i] = kQNaN;
                break;
            }
        }
        ++polls;
    }
    wave_sync();
}

// ----------------------------------------------------------------------------------
// single instance: one wavefront per row, lanes over the updates of a pivot
// ----------------------------------------------------------------------------------
constexpr int kPivCap = 128;   // pivots staged per group
constexpr int kPairCap = 512;  // update pairs staged per group

template <Scope S, bool kFused = false>
__global__ __launch_bounds__(64) void k_numeric_row(PatDev P, const double* __restrict__ a_val,
                                                    double* F, Ctl* ctl, uint64_t spin_limit,
                                                    int64_t skip_row) {
    extern __shared__ double W[];  // working row, indexed by slot - row start
    __shared__ int32_t piv_e[kPivCap + 1];
    __shared__ int32_t piv_dh[kPivCap];
    __shared__ uint64_t piv_u[kPivCap];
    __shared__ int32_t pr_q[kPairCap];
    __shared__ int32_t pr_p[kPairCap];
    __shared__ uint64_t pr_v[kPairCap];
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const int32_t n = P.n;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, (uint32_t)n, (uint32_t)P.groupL, parts, run, t)) break;
        const int32_t j = P.permL ? P.permL[t] : (int32_t)t;
        trace_mark(P.trace, j);
        // The loads of a row are issued level by level of their address
        // dependencies (row bounds -> pivot offsets and diagonal slots ->
        // pair lists and pivot diagonals -> pivot values), each level in one
        // round trip: a row whose pivots are all final then costs a handful
        // of memory latencies, not one per 64 staged values.
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1];
        const int32_t len = (int32_t)(re - rs);
        const int64_t dj = P.diagF[j];
        const int64_t a0 = P.rpA[j], a1 = P.rpA[j + 1];
        // zeros first, then the values of A (one wavefront: its LDS writes land in order)
        for (int32_t e = lane; e < len; e += kWave) W[e] = 0.0;
        for (int64_t p = a0 + lane; p < a1; p += kWave) W[P.a2f[p] - rs] = sanitize_input(a_val[p], ctl);
        wave_sync();

        int64_t s0 = rs;
        while (s0 < dj) {
            int32_t np = (int32_t)std::min<int64_t>(dj - s0, kPivCap);
            const int64_t e0 = P.sptr[s0];
            {
                constexpr int kSlots = (kPivCap + kWave) / kWave;  // covers i = 0..np
                int64_t off[kSlots];
                int32_t dh[kSlots];
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    const int32_t i = lane + u * kWave;
                    off[u] = i <= np ? P.sptr[s0 + i] : 0;
                    dh[u] = i < np ? P.lsd[s0 + i] : 0;
                }
#pragma unroll
                for (int u = 0; u < kSlots; ++u) {
                    const int32_t i = lane + u * kWave;
                    if (i <= np) piv_e[i] = (int32_t)std::min<int64_t>(off[u] - e0, 0x7fffffff);
                    if (i < np) piv_dh[i] = dh[u];
                }
            }
            wave_sync();
            int32_t fit = 0;
            for (int32_t i = 1 + lane; i <= np; i += kWave) fit += piv_e[i] <= kPairCap ? 1 : 0;
            for (int off = 32; off > 0; off >>= 1) fit += __shfl_xor(fit, off);
            np = uniform(fit > 0 ? fit : 1);
            const int32_t npair = uniform(piv_e[np]);
            const bool big = npair > kPairCap;  // a single pivot with more pairs than fit
            bool all_final = false;
            {
                constexpr int kPS = kPairCap / kWave;
                constexpr int kPv = kPivCap / kWave;
                const int32_t nst = big ? 0 : npair;
                int32_t q[kPS], pp[kPS], dh[kPv];
                bool fin = true;  // every staged value already final
#pragma unroll
                for (int u = 0; u < kPS; ++u) {
                    const int32_t e = lane + u * kWave;
                    q[u] = e < nst ? P.sq[e0 + e] : 0;
                    pp[u] = e < nst ? P.sp[e0 + e] : 0;
                }
#pragma unroll
                for (int u = 0; u < kPv; ++u) {
                    const int32_t i = lane + u * kWave;
                    dh[u] = i < np ? piv_dh[i] : 0;
                }
                uint64_t v[kPS], ud[kPv];
#pragma unroll
                for (int u = 0; u < kPv; ++u) ud[u] = lane + u * kWave < np ? ld_cached(F + dh[u]) : 0ull;
#pragma unroll
                for (int u = 0; u < kPS; ++u) v[u] = lane + u * kWave < nst ? ld_cached(F + q[u]) : 0ull;
#pragma unroll
                for (int u = 0; u < kPv; ++u)
                    if (lane + u * kWave < np) {
                        piv_u[lane + u * kWave] = ud[u];
                        fin = fin && ud[u] != kPending;
                    }
#pragma unroll
                for (int u = 0; u < kPS; ++u) {
                    const int32_t e = lane + u * kWave;
                    if (e < nst) {
                        pr_q[e] = q[u];
                        pr_p[e] = (int32_t)(pp[u] - rs);
                        pr_v[e] = v[u];
                        fin = fin && v[u] != kPending;
                    }
                }
                all_final = !big && __all(fin);
            }
            wave_sync();
            for (int32_t i = 0; i < np; ++i) {
                const int64_t s = s0 + i;
                uint64_t ub = piv_u[i];
                const int32_t ea = piv_e[i], eb = piv_e[i + 1];
                if (all_final) {
                    // nothing to wait for in this group
                } else if (!big) {
                    // the pivot and every value it contributes, polled together
                    bool ok = ub != kPending;
                    for (int32_t e = ea + lane; e < eb; e += kWave) ok = ok && pr_v[e] != kPending;
                    if (!__all(ok)) {
                        wait_pivot(F, i, np, piv_dh, piv_u, piv_e, pr_q, pr_v, ctl, spin_limit);
                        ub = piv_u[i];
                        trace_mark(P.trace, 2 * (int64_t)n + j);
                    }
                } else {
                    ub = as_u64(wait_final(F + piv_dh[i], ub, ctl, spin_limit));
                }
                const double l = W[s - rs] / as_f64(ub);
                if (lane == 0) W[s - rs] = l;
                if (!big) {
                    for (int32_t e = ea + lane; e < eb; e += kWave) {
                        const uint64_t vb = pr_v[e];
                        const double v = as_f64(vb == kPending ? kQNaN : vb);  // pending only after a timeout
                        const int32_t p = pr_p[e];
                        W[p] = ikj_update<kFused>(W[p], l, v);
                    }
                } else {
                    for (int64_t e = e0 + lane; e < e0 + npair; e += kWave) {
                        const int32_t q = P.sq[e];
                        const int32_t p = (int32_t)(P.sp[e] - rs);
                        const double v = wait_final(F + q, ctl, spin_limit);
                        W[p] = ikj_update<kFused>(W[p], l, v);
                    }
                }
                wave_sync();
            }
            s0 += np;
        }
        const int32_t dl = (int32_t)(dj - rs);
        trace_mark(P.trace, 3 * (int64_t)n + j);
        if (lane == 0 && W[dl] == 0.0) atomicMin(&ctl->bad_row, (unsigned long long)j);
        if ((int64_t)j != skip_row) {
            // U part first: later rows wait on it; the L part is only read by later kernels
            for (int32_t e = dl + lane; e < len; e += kWave) st_final<S>(F + rs + e, W[e]);
            for (int32_t e = lane; e < dl; e += kWave) F[rs + e] = W[e];
        }
        trace_mark(P.trace, (int64_t)n + j);
        wave_sync();
    }
}

// ----------------------------------------------------------------------------------
// single instance, dataflow form: lanes own target entries of the row
// ----------------------------------------------------------------------------------
// Walking the pivots of row j one at a time leaves 60 of 64 lanes idle (a
// pivot updates only a handful of entries) and puts every pivot's division
// and LDS round trips on the row's serial path.  Here each lane owns entries
// f_jt of row j (t = lane, lane + 64, ...) and applies their updates itself,
// from a target-major copy of the update schedule: per entry, the pivots h
// that update it in ascending order (the order that fixes the bits).  An
// update needs l_h = f_jh / f_hh, which the lane owning entry h produces once
// f_jh has taken all of its own updates; l values are handed between lanes
// through LDS, initialised to kPending.  A lane finishes its entries in
// ascending order; the smallest unfinished entry of the row only waits on
// pivot rows (never on another lane), so the row always makes progress.
// Values of pivot rows are staged in LDS with optimistic reads; those still
// pending are re-polled (agent scope) a few at a time per lane, all lanes in
// one round trip, only when no lane can progress from LDS alone.  Entries of
// the U part are published the moment they are final, so rows that pivot on
// row j need not wait for the rest of it.
constexpr int kFlowCap = 1024;   // staged updates per chunk of targets (at least the longest L part)
// staged values re-polled per lane and round (at n=160,000 k=2: 1 / 2 / 3 / 4 / 6
// measured 6.12 / 5.44 / 5.19 / 5.25 / 5.44 ms)
constexpr int kFlowLook = 3;

size_t flow_lds_bytes(int32_t max_row, int32_t cap) {
    return (size_t)max_row * 8 * 3 + (size_t)cap * 8 + (size_t)max_row * 4 + (size_t)cap * 8 +
           ((size_t)max_row + 1) * 4;
}

typedef __attribute__((address_space(3))) uint64_t LdsU64;

// kHops: instead of values, every entry carries the length of the longest
// chain of dependencies that ends in it, a hand-off between rows (a pivot-row
// value used by row j) weighing w_hop and an l of row j (a division whose
// result other entries of the row wait for) weighing w_step: the same kernel
// and the same waits, with the update acc - l * v replaced by
// max(acc, l, v + w_hop) and the division by max(acc, u + w_hop) + w_step.
// The largest value over F is the elimination's critical path.
template <Scope S, bool kHops = false, bool kFused = false>
__global__ __launch_bounds__(64) void k_numeric_flow(PatDev P, const double* __restrict__ a_val, double* F,
                                                     Ctl* ctl, uint64_t spin_limit, int64_t skip_row,
                                                     int32_t max_row, int32_t cap, double w_hop = 1.0,
                                                     double w_step = 0.0) {
    extern __shared__ uint64_t lds_u64[];
    double* Wv = reinterpret_cast<double*>(lds_u64);                  // [max_row] initial values
    // arrays that lanes update for one another inside the loops below:
    // volatile, so every read goes to LDS, and typed as LDS so that the reads
    // are LDS instructions rather than generic (flat) loads
    volatile LdsU64* Lb = (volatile LdsU64*)(lds_u64 + max_row);              // [max_row] l of L entries
    volatile LdsU64* Ud = (volatile LdsU64*)(lds_u64 + 2 * (size_t)max_row);  // [max_row] pivot diagonals
    volatile LdsU64* Sv = (volatile LdsU64*)(lds_u64 + 3 * (size_t)max_row);  // [cap] staged f_ht
    int32_t* Uq = reinterpret_cast<int32_t*>(lds_u64 + 3 * (size_t)max_row + cap);  // [max_row]
    int32_t* Ss = Uq + max_row;                                      // [cap] pivot entry of update
    int32_t* Sq = Ss + cap;                                          // [cap] F slot of f_ht
    int32_t* Tb = Sq + cap;                                          // [max_row + 1] chunk offsets
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const int32_t n = P.n;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, (uint32_t)n, (uint32_t)P.groupL, parts, run, t)) break;
        const int32_t j = P.permL ? P.permL[t] : (int32_t)t;
        trace_mark(P.trace, j);
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1];
        const int32_t len = (int32_t)(re - rs);
        const int32_t dl = (int32_t)(P.diagF[j] - rs);
        const bool publish = (int64_t)j != skip_row;
        for (int32_t e = lane; e < len; e += kWave) Wv[e] = 0.0;
        for (int32_t e = lane; e < dl; e += kWave) {
            const int32_t dh = P.lsd[rs + e];
            Uq[e] = dh;
            Ud[e] = ld_cached(F + dh);
            Lb[e] = kPending;
        }
        wave_sync();
        if constexpr (!kHops)
            for (int64_t q = P.rpA[j] + lane; q < P.rpA[j + 1]; q += kWave)
                Wv[P.a2f[q] - rs] = sanitize_input(a_val[q], ctl);
        const int64_t row0 = P.tptr[rs];
        const bool whole = P.tptr[re] - row0 <= cap;
        bool stop = false;
        int32_t p0 = 0;
        while (p0 < len && !stop) {
            // chunk [p0, p1): the most targets whose updates fit the staging arrays
            const int64_t c0 = P.tptr[rs + p0];
            int32_t p1 = len;
            if (!whole) {
                p1 = p0 + 1;
                for (int32_t base = p0 + 1; base <= len; base += kWave) {
                    const int32_t cand = base + lane;
                    const bool ok = cand <= len && P.tptr[rs + cand] - c0 <= cap;
                    const uint64_t m = __ballot(ok);
                    if (m == 0ull) break;
                    p1 = base + 63 - __clzll(m);
                    if (m != ~0ull) break;
                }
            }
            const int32_t nu = (int32_t)(P.tptr[rs + p1] - c0);
            for (int32_t k = lane; k < nu; k += kWave) {
                const int32_t q = P.tq[c0 + k];
                Sq[k] = q;
                Ss[k] = P.tsl[c0 + k];
                Sv[k] = ld_cached(F + q);
            }
            for (int32_t q = p0 + lane; q <= p1; q += kWave) Tb[q - p0] = (int32_t)(P.tptr[rs + q] - c0);
            wave_sync();

            int32_t p = p0 + lane;
            bool have = p < p1;
            int32_t e = 0, ee = 0;
            double acc = 0.0;
            if (have) { e = Tb[p - p0]; ee = Tb[p - p0 + 1]; acc = Wv[p]; }
            uint32_t polls = 0;
            uint64_t t0 = 0;
            for (;;) {
                // progress from LDS alone until no lane can move
                for (;;) {
                    bool prog = false;
                    if (have) {
                        // the entry's updates while their inputs are in LDS.  An
                        // entry mostly takes one or two, so the first is taken
                        // before the loop: in the default rounding that shape
                        // measured 5.78 -> 5.26 ms at n=160,000 k=2; with the
                        // fused update the compiler peels the plain loop itself
                        // (5.24 ms; 5.32 with the peel written out)
                        if constexpr (kFused || kHops) {
                            while (e < ee) {
                                const uint64_t lb = Lb[Ss[e]];
                                const uint64_t vb = Sv[e];
                                if (lb == kPending || vb == kPending) break;
                                if constexpr (kHops)
                                    acc = fmax(acc, fmax(as_f64(lb), as_f64(vb) + w_hop));
                                else
                                    acc = ikj_update<kFused>(acc, as_f64(lb), as_f64(vb));
                                ++e;
                                prog = true;
                            }
                        } else if (e < ee) {
                            const uint64_t lb = Lb[Ss[e]];
                            const uint64_t vb = Sv[e];
                            if (lb != kPending && vb != kPending) {
                                acc = ikj_update<false>(acc, as_f64(lb), as_f64(vb));
                                ++e;
                                prog = true;
                                while (e < ee) {
                                    const uint64_t lb2 = Lb[Ss[e]];
                                    const uint64_t vb2 = Sv[e];
                                    if (lb2 == kPending || vb2 == kPending) break;
                                    acc = ikj_update<false>(acc, as_f64(lb2), as_f64(vb2));
                                    ++e;
                                }
                            }
                        }
                        if (e >= ee) {
                            bool fin = true;
                            if (p < dl) {
                                const uint64_t ub = Ud[p];
                                if (ub == kPending) fin = false;
                                else if constexpr (kHops) Lb[p] = as_u64(fmax(acc, as_f64(ub) + w_hop) + w_step);
                                else Lb[p] = as_u64(acc / as_f64(ub));
                            } else {
                                if (publish) st_final<S>(F + rs + p, acc);
                                if (!kHops && p == dl && acc == 0.0)
                                    atomicMin(&ctl->bad_row, (unsigned long long)j);
                            }
                            if (fin) {
                                prog = true;
                                p += kWave;
                                have = p < p1;
                                if (have) { e = Tb[p - p0]; ee = Tb[p - p0 + 1]; acc = Wv[p]; }
                            }
                        }
                    }
                    if (!__any(prog)) break;
                }
                if (!__any(have)) break;
                // one round trip for every lane's pending inputs
                bool got = false;
                if (have) {
                    // the indices first (LDS, all together), then every load:
                    // no LDS round trip between two loads of one round
                    bool need[kFlowLook];
                    int32_t qi[kFlowLook];
                    uint64_t v[kFlowLook];
#pragma unroll
                    for (int u = 0; u < kFlowLook; ++u) {
                        const int32_t x = e + u;
                        const bool in = x < ee;
                        const int32_t xi = in ? x : 0;  // a staged index either way; unused when !in
                        const uint64_t sv = Sv[xi];
                        qi[u] = Sq[xi];
                        need[u] = in && sv == kPending;
                    }
                    const bool inl = p < dl;
                    const int32_t uq = Uq[inl ? p : 0];
                    const bool needu = inl && Ud[inl ? p : 0] == kPending;
#pragma unroll
                    for (int u = 0; u < kFlowLook; ++u) v[u] = need[u] ? ld_coherent(F + qi[u]) : kPending;
                    const uint64_t vu = needu ? ld_coherent(F + uq) : kPending;
#pragma unroll
                    for (int u = 0; u < kFlowLook; ++u)
                        if (need[u] && v[u] != kPending) { Sv[e + u] = v[u]; got = true; }
                    if (needu && vu != kPending) { Ud[p] = vu; got = true; }
                }
                if (__any(got)) {
                    trace_mark(P.trace, 2 * (int64_t)n + j);
                    polls = 0;
                    continue;
                }
                // watchdog: a stall (rounds with no input arriving) is timed
                // from its 32nd round; the abort flag is read every 256 rounds
                if ((polls & 31u) == 31u) {
                    if ((polls & 255u) == 255u && ld_u32_coherent(&ctl->abort) != 0u) stop = true;
                    const uint64_t now = wall_clock64();
                    if (polls == 31u) {
                        t0 = now;
                    } else if (now - t0 > spin_limit) {
                        if (lane == 0) {
                            atomicOr(&ctl->status, kStTimeout);
                            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        stop = true;
                    }
                    if (__any(stop)) {
                        stop = true;
                        break;
                    }
                }
                ++polls;
            }
            wave_sync();
            p0 = p1;
        }
        trace_mark(P.trace, 3 * (int64_t)n + j);
        if (publish) {
            for (int32_t q = lane; q < dl; q += kWave) {
                const uint64_t lb = Lb[q];
                F[rs + q] = as_f64(lb == kPending ? kQNaN : lb);
            }
            // after an abort, release anything that might still wait on this row
            if (stop)
                for (int32_t q = dl + lane; q < len; q += kWave) st_final<S>(F + rs + q, as_f64(kQNaN));
        }
        trace_mark(P.trace, (int64_t)n + j);
        wave_sync();
    }
}

// ----------------------------------------------------------------------------------
// batches: lanes are instances (values stored entry-major, instance-minor, so a
// wavefront's 64 loads of one entry are one contiguous 512-byte line); the
// pivot loop and the pair lists are uniform across the wavefront
// ----------------------------------------------------------------------------------
constexpr int kBPivCap = 8;
constexpr int kBPairCap = 32;
constexpr int kBAChunk = 8;  // A entries loaded per round trip
// pending pair values re-read per polling round (256 x 128^2 ILU(2) factorization:
// 1 / 2 / 3 / 4 / 8 measured 1.66 / 1.37 / 1.19 / 1.23 / 1.42 ms; 70 x 27-point 20^3
// ILU(2), global working rows: 21.9 / 22.5 / 23.1 / 23.4 / 23.6 ms)
constexpr int kBLook = 3;
constexpr int kBWChunk = 8;  // values loaded per round trip (global working rows, publish, fused forward)

// kGW: the working row lives in global memory (a slice of wrow per
// wavefront, wstride doubles each, same [len][64] layout) instead of LDS, for
// rows too long for LDS.  A lane reads back only what it wrote itself, so
// plain loads and stores in program order are enough.  The update loop then
// reads a pivot's targets a chunk at a time before writing any (one pivot's
// targets are distinct slots), so it pays one latency per chunk rather than
// one per update.  (In LDS the same chunking measured slower.)
//
// xout non-null: the forward substitution (Eq. 3b) is fused in.  Once a row
// has stored its factor, its lane computes x_j = b_j - sum of l_jh x_h over
// the row's L slots in ascending order (the forward kernel's order, so the
// same bits), from the l values still in the working row and the x_h that
// the rows of its pivots published when they finished.  Those rows finished
// before this one, so the extra wait is short and off the chain the factor's
// dependents wait on (the row's U part is published first).
template <bool kGW, Scope S, bool kFused = false>
__global__ __launch_bounds__(64) void k_numeric_batch(PatDev P, const double* __restrict__ a_val,
                                                      int32_t B, double* F, Ctl* ctl,
                                                      uint64_t spin_limit, int64_t skip_row,
                                                      double* __restrict__ wrow, int64_t wstride,
                                                      const double* __restrict__ bvec, double* xout) {
    extern __shared__ double Wl[];  // [len][64]
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    // working-row slice: the block index, or on one XCD (where the members'
    // block indices follow the hardware's dealing) a number drawn from
    // ctl->ticket; members beyond the slices leave (the others do the work)
    uint32_t slot = blockIdx.x;
    if constexpr (kGW && S == Scope::Xcd) {
        slot = wave_ticket(ctl);
        if (slot >= gridDim.x / kXcds) return;
    }
    double* const W = kGW ? wrow + (int64_t)slot * wstride : Wl;
    __shared__ int32_t piv_e[kBPivCap + 1];
    __shared__ int32_t piv_dh[kBPivCap];
    __shared__ int32_t pr_q[kBPairCap];
    __shared__ int32_t pr_p[kBPairCap];
    __shared__ uint64_t vu[kBPivCap * kWave];
    __shared__ uint64_t vv[kBPairCap * kWave];
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, parts, run, t)) break;
        const int32_t jr = (int32_t)(t / (uint32_t)G);
        const int32_t j = P.permL ? P.permL[jr] : jr;
        const int32_t g = (int32_t)(t % (uint32_t)G);
        const int32_t col = g * kWave + lane;
        const bool act = col < B;
        const int32_t colc = act ? col : B - 1;  // an in-bounds column for inactive lanes
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1];
        const int32_t len = (int32_t)(re - rs);
        const int64_t dj = P.diagF[j];
        // Loads are issued a dependency level at a time (A row; pivot offsets
        // and diagonal slots; pair lists; pivot values), each level in one
        // round trip, so a task whose pivots are final costs a few memory
        // latencies rather than one per staged value.
        const int64_t a0 = P.rpA[j], a1 = P.rpA[j + 1];
        for (int32_t e = 0; e < len; ++e) W[e * kWave + lane] = 0.0;
        for (int64_t p0 = a0; p0 < a1; p0 += kBAChunk) {
            // unconditional loads at clamped, in-bounds indices keep the
            // compiler from waiting on each one; the extra values are unused
            int32_t sl[kBAChunk];
            double av[kBAChunk];
#pragma unroll
            for (int u = 0; u < kBAChunk; ++u) {
                const int64_t p = std::min<int64_t>(p0 + u, a1 - 1);
                sl[u] = P.a2f[p] - (int32_t)rs;
                av[u] = a_val[p * B + colc];
            }
#pragma unroll
            for (int u = 0; u < kBAChunk; ++u)
                if (p0 + u < a1 && act) W[(int64_t)sl[u] * kWave + lane] = sanitize_input(av[u], ctl);
        }
        int64_t s0 = rs;
        while (s0 < dj) {
            int32_t np = (int32_t)std::min<int64_t>(dj - s0, kBPivCap);
            const int64_t e0 = P.sptr[s0];
            // lane i: pair offset of pivot i of the group and its diagonal slot
            const int64_t offl = lane <= np ? P.sptr[s0 + lane] - e0 : 0;
            const int32_t dhl = lane < np ? P.lsd[s0 + lane] : 0;
            // offsets never decrease: the pivots whose pairs fit are a prefix
            const int32_t fit = __popcll(__ballot(lane >= 1 && lane <= np && offl <= kBPairCap));
            np = fit > 0 ? fit : 1;
            const int32_t npair = (int32_t)std::min<int64_t>(bcast_i64(offl, np), 0x7fffffff);
            const bool big = npair > kBPairCap;  // a single pivot with more pairs than fit
            wave_sync();
            if (lane <= np) piv_e[lane] = (int32_t)std::min<int64_t>(offl, 0x7fffffff);
            if (lane < np) piv_dh[lane] = dhl;
            const int32_t nst = big ? 0 : npair;
            const int32_t ql = lane < nst ? P.sq[e0 + lane] : 0;
            const int32_t pl = lane < nst ? P.sp[e0 + lane] : 0;
            if (lane < nst) {
                pr_q[lane] = ql;
                pr_p[lane] = (int32_t)(pl - rs);
            }
            // every lane (instance) needs every pivot's and pair's slot: read them
            // out of the lanes that loaded them while the whole wavefront is active
            int32_t dhs[kBPivCap], qs[kBPairCap];
#pragma unroll
            for (int i = 0; i < kBPivCap; ++i) dhs[i] = __builtin_amdgcn_readlane(dhl, i);
#pragma unroll
            for (int e = 0; e < kBPairCap; ++e) qs[e] = __builtin_amdgcn_readlane(ql, e);
            if (act) {
                uint64_t u8[kBPivCap], v32[kBPairCap];
#pragma unroll
                for (int i = 0; i < kBPivCap; ++i) u8[i] = ld_cached(F + (int64_t)dhs[i] * B + col);
#pragma unroll
                for (int e = 0; e < kBPairCap; ++e) v32[e] = ld_cached(F + (int64_t)qs[e] * B + col);
#pragma unroll
                for (int i = 0; i < kBPivCap; ++i)
                    if (i < np) vu[i * kWave + lane] = u8[i];
#pragma unroll
                for (int e = 0; e < kBPairCap; ++e)
                    if (e < nst) vv[e * kWave + lane] = v32[e];
            }
            wave_sync();
            if (act && !big) {
                // Pivots in ascending order, each once its diagonal and all of
                // its pair values are final in this lane's staged copy.  A
                // round of polls re-reads the pivot's diagonal and up to
                // kBLook of its pending pairs together (one round trip), so a
                // pivot row that has just been published costs one latency,
                // not one per value.
                // State of pivot i, carried across polling rounds: its pair
                // range [ea, eb), whether its diagonal is final (ur) and the
                // first pair not yet final (ep).  A round advances ep over the
                // values it brought, in registers, without rescanning LDS.
                int32_t i = 0;
                uint32_t polls = 0;
                uint64_t t0 = 0;
                int32_t ea = piv_e[0], eb = piv_e[1];
                bool ur = vu[lane] != kPending;
                int32_t ep = ea;
                while (ep < eb && vv[ep * kWave + lane] != kPending) ++ep;
                while (i < np) {
                    if (ur && ep == eb) {
                        const int64_t sl = s0 + i - rs;
                        const double l = W[sl * kWave + lane] / as_f64(vu[i * kWave + lane]);
                        W[sl * kWave + lane] = l;
                        if (kGW) {
                            for (int32_t c = ea; c < eb; c += kBWChunk) {
                                double w[kBWChunk];
                                int32_t pc[kBWChunk];
#pragma unroll
                                for (int u = 0; u < kBWChunk; ++u) {
                                    pc[u] = pr_p[std::min(c + u, eb - 1)];
                                    w[u] = W[pc[u] * kWave + lane];
                                }
#pragma unroll
                                for (int u = 0; u < kBWChunk; ++u)
                                    if (c + u < eb)
                                        W[pc[u] * kWave + lane] =
                                            ikj_update<kFused>(w[u], l, as_f64(vv[(c + u) * kWave + lane]));
                            }
                        } else {
                            for (int32_t e = ea; e < eb; ++e) {
                                const int32_t p = pr_p[e];
                                W[p * kWave + lane] =
                                    ikj_update<kFused>(W[p * kWave + lane], l, as_f64(vv[e * kWave + lane]));
                            }
                        }
                        ++i;
                        polls = 0;
                        if (i < np) {
                            ea = eb;
                            eb = piv_e[i + 1];
                            ur = vu[i * kWave + lane] != kPending;
                            ep = ea;
                            while (ep < eb && vv[ep * kWave + lane] != kPending) ++ep;
                        }
                        continue;
                    }
                    const double* du = F + (int64_t)piv_dh[i] * B + col;
                    const uint64_t nu = ld_coherent(du);
                    uint64_t nv[kBLook];
#pragma unroll
                    for (int k = 0; k < kBLook; ++k) {
                        const int32_t e = ep + k;
                        // entries past the pivot's pairs read the diagonal's line again
                        nv[k] = ld_coherent(e < eb ? F + (int64_t)pr_q[e] * B + col : du);
                    }
                    if (!ur && nu != kPending) {
                        vu[i * kWave + lane] = nu;
                        ur = true;
                    }
                    int32_t adv = 0;
#pragma unroll
                    for (int k = 0; k < kBLook; ++k) {
                        const bool fin = ep + k < eb && nv[k] != kPending;
                        if (fin) vv[(ep + k) * kWave + lane] = nv[k];
                        if (fin && adv == k) adv = k + 1;
                    }
                    ep += adv;
                    if (adv == kBLook)
                        while (ep < eb && vv[ep * kWave + lane] != kPending) ++ep;
                    if ((polls & 31u) == 31u) {
                        bool stop = (polls & 255u) == 255u && ld_u32_coherent(&ctl->abort) != 0u;
                        const uint64_t now = wall_clock64();
                        if (polls == 31u) {
                            t0 = now;
                        } else if (now - t0 > spin_limit) {
                            atomicOr(&ctl->status, kStTimeout);
                            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            stop = true;
                        }
                        if (stop) {
                            // give up on this pivot: its values become quiet NaNs
                            if (vu[i * kWave + lane] == kPending) vu[i * kWave + lane] = kQNaN;
                            for (int32_t e = ea; e < eb; ++e)
                                if (vv[e * kWave + lane] == kPending) vv[e * kWave + lane] = kQNaN;
                            ur = true;
                            ep = eb;
                        }
                    }
                    ++polls;
                }
            } else if (act) {
                for (int32_t i = 0; i < np; ++i) {
                    const int64_t sl = s0 + i - rs;
                    const double u = wait_final(F + (int64_t)piv_dh[i] * B + col, vu[i * kWave + lane], ctl,
                                                spin_limit);
                    const double l = W[sl * kWave + lane] / u;
                    W[sl * kWave + lane] = l;
                    if (!big) {
                        for (int32_t e = piv_e[i]; e < piv_e[i + 1]; ++e) {
                            const double v = wait_final(F + (int64_t)pr_q[e] * B + col,
                                                        vv[e * kWave + lane], ctl, spin_limit);
                            const int32_t p = pr_p[e];
                            W[p * kWave + lane] = ikj_update<kFused>(W[p * kWave + lane], l, v);
                        }
                    } else {
                        for (int64_t e = e0; e < e0 + npair; ++e) {
                            const int32_t q = P.sq[e];
                            const int64_t p = P.sp[e] - rs;
                            const double v = wait_final(F + (int64_t)q * B + col, ctl, spin_limit);
                            W[p * kWave + lane] = ikj_update<kFused>(W[p * kWave + lane], l, v);
                        }
                    }
                }
            }
            s0 += np;
        }
        const int32_t dl = (int32_t)(dj - rs);
        if (act && W[dl * kWave + lane] == 0.0) atomicMin(&ctl->bad_row, (unsigned long long)j);
        if (act && (int64_t)j != skip_row) {
            if (kGW) {
                // U part first (the rows waiting on it), then L, a chunk of
                // loads per round trip
                for (int32_t c = dl; c < len + dl; c += kBWChunk) {
                    double w[kBWChunk];
                    int32_t ec[kBWChunk];
#pragma unroll
                    for (int u = 0; u < kBWChunk; ++u) {
                        const int32_t e = std::min(c + u, len + dl - 1);
                        ec[u] = e < len ? e : e - len;
                        w[u] = W[ec[u] * kWave + lane];
                    }
#pragma unroll
                    for (int u = 0; u < kBWChunk; ++u) {
                        if (c + u >= len + dl) continue;
                        if (c + u < len) st_final<S>(F + (rs + ec[u]) * B + col, w[u]);
                        else F[(rs + ec[u]) * B + col] = w[u];
                    }
                }
            } else {
                for (int32_t e = dl; e < len; ++e) st_final<S>(F + (rs + e) * B + col, W[e * kWave + lane]);
                for (int32_t e = 0; e < dl; ++e) F[(rs + e) * B + col] = W[e * kWave + lane];
            }
        }
        if (xout && act) {
            double sx = sanitize_input(bvec[(int64_t)j * B + col], ctl);
            for (int32_t c = 0; c < dl; c += kBWChunk) {
                double fv[kBWChunk];
                uint64_t xv[kBWChunk];
                int32_t hh[kBWChunk];
#pragma unroll
                for (int u = 0; u < kBWChunk; ++u) {
                    const int32_t e = std::min(c + u, dl - 1);
                    hh[u] = P.ciF[rs + e];
                    fv[u] = W[e * kWave + lane];
                    xv[u] = ld_cached(xout + (int64_t)hh[u] * B + col);
                }
#pragma unroll
                for (int u = 0; u < kBWChunk; ++u)
                    if (c + u >= dl) xv[u] = 0ull;
                settle(xout, hh, xv, B, col, ctl, spin_limit);
#pragma unroll
                for (int u = 0; u < kBWChunk; ++u)
                    if (c + u < dl) sx = sx - fv[u] * as_f64(xv[u]);
            }
            if ((int64_t)j != skip_row) st_final<S>(xout + (int64_t)j * B + col, sx);
        }
        wave_sync();
    }
}

int32_t flow_cap(int32_t max_lrow) { return std::max(kFlowCap, max_lrow); }

hipError_t launch_numeric_hops(const PatDev& P, double* f_hops, Ctl* ctl, uint64_t spin_limit, int32_t grid,
                               int32_t max_row, int32_t max_lrow, double w_hop, double w_step, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    const int32_t mr = std::max(max_row, 1), cap = flow_cap(max_lrow);
    hipLaunchKernelGGL((k_numeric_flow<Scope::Device, true>), dim3(grid), dim3(64), flow_lds_bytes(mr, cap), s, P,
                       nullptr, f_hops, ctl, spin_limit, (int64_t)-1, mr, cap, w_hop, w_step);
    return hipGetLastError();
}

// largest value of v[0..n) (non-negative, not NaN) into *out (pre-set to
// 0): non-negative doubles order like their bit patterns
__global__ void k_max_nonneg(const double* __restrict__ v, int64_t n, unsigned long long* out) {
    unsigned long long m = 0ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (unsigned long long)as_u64(v[i]));
    for (int o = kWave / 2; o > 0; o >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, o));
    if (lane_id() == 0) atomicMax(out, m);
}

hipError_t launch_max_nonneg(const double* v, int64_t n, unsigned long long* out, hipStream_t s) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_max_nonneg, dim3(blocks), dim3(256), 0, s, v, n, out);
    return hipGetLastError();
}

bool numeric_flow_fits(int32_t max_row, int32_t max_lrow, size_t lds_limit) {
    return flow_lds_bytes(std::max(max_row, 1), flow_cap(max_lrow)) <= lds_limit;
}

int numeric_grid(int32_t batch, int32_t max_row, int32_t max_lrow, bool flow, int num_cu, bool global_row) {
    // LDS per wavefront bounds how many rows are in flight; aim for the
    // resident maximum so every ready row has a wavefront
    size_t lds;
    if (batch == 1 && flow)
        lds = flow_lds_bytes(std::max(max_row, 1), flow_cap(max_lrow));
    else if (batch == 1)
        lds = (size_t)max_row * 8 + (kPivCap + 1) * 4 + kPivCap * 12 + kPairCap * 16;
    else
        lds = (global_row ? 0 : (size_t)max_row * 8 * kWave) + (kBPivCap + 1) * 4 + kBPivCap * 4 +
              kBPairCap * 8 + (kBPivCap + kBPairCap) * 8 * kWave;
    size_t per_cu = std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
    per_cu = std::min<size_t>(per_cu, 32);
    return (int)(per_cu * (size_t)num_cu);
}

template <bool kFused>
hipError_t launch_numeric_t(const PatDev& P, const double* a_val, int32_t batch, double* f_val,
                          Ctl* ctl, uint64_t spin_limit, int64_t skip_row, int32_t grid,
                          int32_t max_row, int32_t max_lrow, bool flow, bool one_xcd, double* wrow,
                          const double* bvec, double* xout, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    const dim3 g1(one_xcd ? grid * kXcds : grid);
    if (batch == 1 && flow) {
        const int32_t mr = std::max(max_row, 1), cap = flow_cap(max_lrow);
        const size_t lds = flow_lds_bytes(mr, cap);
        if (one_xcd)
            hipLaunchKernelGGL((k_numeric_flow<Scope::Xcd, false, kFused>), g1, dim3(64), lds, s, P, a_val, f_val, ctl, spin_limit,
                               skip_row, mr, cap);
        else
            hipLaunchKernelGGL((k_numeric_flow<Scope::Device, false, kFused>), g1, dim3(64), lds, s, P, a_val, f_val, ctl,
                               spin_limit, skip_row, mr, cap);
    } else if (batch == 1) {
        const size_t lds = (size_t)std::max(max_row, 1) * sizeof(double);
        if (one_xcd)
            hipLaunchKernelGGL((k_numeric_row<Scope::Xcd, kFused>), g1, dim3(64), lds, s, P, a_val, f_val, ctl, spin_limit,
                               skip_row);
        else
            hipLaunchKernelGGL((k_numeric_row<Scope::Device, kFused>), g1, dim3(64), lds, s, P, a_val, f_val, ctl,
                               spin_limit, skip_row);
    } else {
        const int64_t ws = (int64_t)std::max(max_row, 1) * kWave;
        if (wrow) {
            if (one_xcd)
                hipLaunchKernelGGL((k_numeric_batch<true, Scope::Xcd, kFused>), g1, dim3(64), 0, s, P, a_val, batch,
                                   f_val, ctl, spin_limit, skip_row, wrow, ws, bvec, xout);
            else
                hipLaunchKernelGGL((k_numeric_batch<true, Scope::Device, kFused>), g1, dim3(64), 0, s, P, a_val, batch,
                                   f_val, ctl, spin_limit, skip_row, wrow, ws, bvec, xout);
        } else {
            const size_t lds = (size_t)ws * sizeof(double);
            if (one_xcd)
                hipLaunchKernelGGL((k_numeric_batch<false, Scope::Xcd, kFused>), g1, dim3(64), lds, s, P, a_val, batch,
                                   f_val, ctl, spin_limit, skip_row, nullptr, (int64_t)0, bvec, xout);
            else
                hipLaunchKernelGGL((k_numeric_batch<false, Scope::Device, kFused>), g1, dim3(64), lds, s, P, a_val,
                                   batch, f_val, ctl, spin_limit, skip_row, nullptr, (int64_t)0, bvec, xout);
        }
    }
    return hipGetLastError();
}

hipError_t launch_numeric(const PatDev& P, const double* a_val, int32_t batch, double* f_val,
                          Ctl* ctl, uint64_t spin_limit, int64_t skip_row, int32_t grid,
                          int32_t max_row, int32_t max_lrow, bool flow, bool one_xcd, double* wrow,
                          const double* bvec, double* xout, bool fused, hipStream_t s) {
    return fused ? launch_numeric_t<true>(P, a_val, batch, f_val, ctl, spin_limit, skip_row, grid, max_row, max_lrow,
                                          flow, one_xcd, wrow, bvec, xout, s)
                 : launch_numeric_t<false>(P, a_val, batch, f_val, ctl, spin_limit, skip_row, grid, max_row,
                                           max_lrow, flow, one_xcd, wrow, bvec, xout, s);
}

}  // namespace tpilu
