// Applying M^-1 = U~^-1 L~^-1 (Eq. 1) on gfx950.
//
// forward  (Eq. 3b): x_i = b_i - f_ih1 x_h1 - f_ih2 x_h2 - ...   h ascending
// backward:          y_i = (x_i - f_ijm y_jm - ... - f_ij1 y_j1) / f_ii,
//                    j descending (right to left).  The paper leaves the
//                    order of the backward substitution open; right to left
//                    makes the value that arrives last (the nearest row's)
//                    the last term of the chain.
//
// Both are dependency-driven: rows go in ascending order for the forward
// sweep and descending for the backward one.  For one instance a wavefront
// owns a row: its lanes form the products (each rounded on its own) and the
// running subtraction is carried through them strictly in the order above,
// advancing as the needed values arrive, which keeps every bit of the
// sequential result.  With these orders the value that arrives last (the
// nearest row) is the last term of the chain.  Two launch shapes give the
// same bits: a persistent grid over the whole device or one XCD (rows handed
// out by atomic task counters), and for wide levels of short rows a lane per
// row (the one-CU shape for deep, narrow graphs is in k_solve_cu.hip).
// For batches the lanes are instances and each lane runs its own chain.
// x and y start as kPending and each slot is written once.
#include "kernels.h"

namespace tpilu {

// one row of the forward sweep, one wavefront: x_i = b_i - sum_h f_ih x_h,
// h ascending
template <Scope S>
__device__ __forceinline__ void forward_row(const PatDev& P, const double* __restrict__ F,
                                            const double* __restrict__ b, double* x, Ctl* ctl,
                                            uint64_t limit, int32_t i) {
    const int lane = lane_id();
    trace_mark(P.trace, i);
    const int64_t rs = P.rpF[i], dj = P.diagF[i];
    double s = sanitize_input(b[i], ctl);
    for (int64_t c = rs; c < dj; c += kWave) {
        const int32_t cnt = (int32_t)min<int64_t>(kWave, dj - c);
        double f = 0.0;
        const double* src = x;
        if (lane < cnt) {
            f = F[c + lane];
            src = x + P.ciF[c + lane];
        }
        s = chain_sub<S>(s, cnt, f, src, ctl, limit);
    }
    if (lane == 0) st_final<S>(x + i, s);
    trace_mark(P.trace, (int64_t)P.n + i);
}

// one row of the backward sweep: y_i = (x_i - sum_j f_ij y_j) / f_ii with the
// subtractions from right to left (j descending)
template <Scope S>
__device__ __forceinline__ void backward_row(const PatDev& P, const double* __restrict__ F,
                                             const double* __restrict__ x, double* y, Ctl* ctl,
                                             uint64_t limit, int32_t i) {
    const int lane = lane_id();
    trace_mark(P.trace, 2 * (int64_t)P.n + i);
    const int64_t dj = P.diagF[i], re = P.rpF[i + 1];
    const int64_t nu = re - dj - 1;
    // on one XCD the diagonal is read before the chain, so that the division
    // waits on nothing else (random banded ILU(2): 9.4 -> 8.2 ms); device-wide
    // the early read measured slower (Table 3 scale ILU(1): 6.0 -> 6.5 ms)
    double fii = 0.0;
    if constexpr (S == Scope::Xcd) fii = F[dj];
    double s = x[i];
    for (int64_t c = 0; c < nu; c += kWave) {
        const int32_t cnt = (int32_t)min<int64_t>(kWave, nu - c);
        double f = 0.0;
        const double* src = y;
        if (lane < cnt) {
            const int64_t q = re - 1 - (c + lane);
            f = F[q];
            src = y + P.ciF[q];
        }
        s = chain_sub<S>(s, cnt, f, src, ctl, limit);
    }
    if constexpr (S != Scope::Xcd) fii = F[dj];
    const double r = s / fii;
    if (lane == 0) st_final<S>(y + i, r);
    trace_mark(P.trace, 3 * (int64_t)P.n + i);
}

// whole device: persistent grid, rows handed out by the task counters
// S == Scope::Xcd: only the workgroups on one XCD take part, all drawing
// from one counter (which workgroups those are is known only at run time)
template <Scope S>
__global__ __launch_bounds__(64) void k_forward_row(PatDev P, const double* __restrict__ F,
                                                    const double* __restrict__ b, double* x,
                                                    Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, (uint32_t)P.n, (uint32_t)P.groupL, parts, run, t)) break;
        forward_row<S>(P, F, b, x, ctl, spin_limit, P.permL ? P.permL[t] : (int32_t)t);
    }
}

template <Scope S>
__global__ __launch_bounds__(64) void k_backward_row(PatDev P, const double* __restrict__ F,
                                                     const double* __restrict__ x, double* y,
                                                     Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, (uint32_t)P.n, (uint32_t)P.groupU, parts, run, t)) break;
        backward_row<S>(P, F, x, y, ctl, spin_limit, P.permU ? P.permU[t] : P.n - 1 - (int32_t)t);
    }
}

// lane per row, for wide dependency graphs of short rows (many rows per level,
// few entries each): one draw from the task counters hands out 64
// consecutive rows of the level order, one per lane, so the counters are
// taken 64 times less often.  Each lane runs its row's chain in the fixed order
// (forward ascending, backward right to left, then the division), with the
// loads of up to kLaneChunk entries in flight together and every pending one
// re-polled each round; the wavefront goes round until all its lanes have
// published.  A lane may wait on the row of another lane of the same
// wavefront (an earlier position of the level order), which advances in the
// same rounds, so the wavefront cannot deadlock.
constexpr int kLaneChunk = 8;

__device__ __forceinline__ void trace_lane(unsigned long long* trace, int64_t slot, bool on) {
    if (trace && on) trace[slot] = wall_clock64();
}

template <bool kBackward>
__global__ __launch_bounds__(64) void k_solve_lanes(PatDev P, const double* __restrict__ F,
                                                    const double* __restrict__ in, double* out, Ctl* ctl,
                                                    uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t* perm = kBackward ? P.permU : P.permL;
    const int64_t tr0 = kBackward ? 2 * (int64_t)n : 0;
    const uint32_t nchunk = (uint32_t)(((int64_t)n + kWave - 1) / kWave);
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, nchunk, 1u, (uint32_t)P.parts, run, t)) break;
        const int64_t r = (int64_t)t * kWave + lane;
        const bool valid = r < n;
        int32_t i = 0;
        int64_t q = 0, dslot = 0;
        int32_t left = 0;
        double s = 0.0, fii = 1.0;
        if (valid) {
            i = perm ? perm[r] : (kBackward ? n - 1 - (int32_t)r : (int32_t)r);
            dslot = P.diagF[i];
            if (kBackward) {
                q = P.rpF[i + 1] - 1;  // right to left
                left = (int32_t)(q - dslot);
                s = in[i];
                fii = F[dslot];
            } else {
                q = P.rpF[i];
                left = (int32_t)(dslot - q);
                s = sanitize_input(in[i], ctl);
            }
        }
        trace_lane(P.trace, tr0 + i, valid);
        bool done = !valid;
        double fv[kLaneChunk];
        uint64_t xv[kLaneChunk];
        int32_t cc[kLaneChunk];
        int32_t cnt = 0, u = 0;
        uint32_t polls = 0;
        uint64_t t0 = 0;
        for (;;) {
            bool prog = false;
            if (!done) {
                if (u == cnt && left > 0) {  // next chunk of the row
                    cnt = min(left, kLaneChunk);
#pragma unroll
                    for (int k = 0; k < kLaneChunk; ++k) {
                        if (k < cnt) {
                            const int64_t slot = kBackward ? q - k : q + k;
                            cc[k] = P.ciF[slot];
                            fv[k] = F[slot];
                            xv[k] = ld_cached(out + cc[k]);
                        }
                    }
                    q = kBackward ? q - cnt : q + cnt;
                    left -= cnt;
                    u = 0;
                }
                bool blocked = false;
#pragma unroll
                for (int k = 0; k < kLaneChunk; ++k) {
                    if (k >= u && k < cnt && !blocked) {
                        if (xv[k] == kPending) {
                            blocked = true;
                        } else {
                            s = s - fv[k] * as_f64(xv[k]);
                            u = k + 1;
                            prog = true;
                        }
                    }
                }
                if (u == cnt && left == 0) {
                    st_publish(out + i, kBackward ? s / fii : s);
                    trace_lane(P.trace, tr0 + n + i, true);
                    done = true;
                    prog = true;
                } else if (blocked) {
#pragma unroll
                    for (int k = 0; k < kLaneChunk; ++k)
                        if (k >= u && k < cnt && xv[k] == kPending) xv[k] = ld_coherent(out + cc[k]);
                }
            }
            if (__all(done)) break;
            if (__any(prog)) {
                polls = 0;
                continue;
            }
            // watchdog over rounds in which no lane advanced
            ++polls;
            if ((polls & 31u) == 0u) {
                bool stop = (polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u;
                const uint64_t now = wall_clock64();
                if (polls == 32u) {
                    t0 = now;
                } else if (now - t0 > spin_limit) {
                    if (lane == 0) {
                        atomicOr(&ctl->status, kStTimeout);
                        __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    stop = true;
                }
                if (__any(stop)) {
                    // release anything waiting on these rows
                    if (!done) st_publish(out + i, as_f64(kQNaN));
                    break;
                }
            }
        }
    }
}

// batches: lanes are instances; each lane runs the sequential chain of its
// instance; the loads of a chunk of entries are issued before any of them is
// waited on (chunks of 1 / 2 / 3 / 4 / 8 entries measured 0.51 / 0.45 / 0.66 /
// 0.48 / 0.59 ms for the forward sweep of 256 x 128^2 ILU(2), 0.87 / 0.81 / 0.76
// / 0.84 / 1.11 ms for 70 x 27-point 20^3 ILU(2))
constexpr int kSolveChunk = 2;

template <Scope S>
__global__ __launch_bounds__(64) void k_forward_batch(PatDev P, const double* __restrict__ F,
                                                      int32_t B, const double* __restrict__ b,
                                                      double* x, Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, parts, run, t)) break;
        const int32_t ir = (int32_t)(t / (uint32_t)G);
        const int32_t i = P.permL ? P.permL[ir] : ir;
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t rs = P.rpF[i], dj = P.diagF[i];
            double s = sanitize_input(b[(int64_t)i * B + col], ctl);
            for (int64_t c = rs; c < dj; c += kSolveChunk) {
                double fv[kSolveChunk];
                uint64_t xv[kSolveChunk];
                int32_t hh[kSolveChunk];
                // unconditional loads at clamped slots (the extra ones unused)
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    const int64_t cc = std::min<int64_t>(c + u, dj - 1);
                    hh[u] = P.ciF[cc];
                    fv[u] = F[cc * B + col];
                    xv[u] = ld_cached(x + (int64_t)hh[u] * B + col);
                }
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u)
                    if (c + u >= dj) xv[u] = 0ull;
                settle(x, hh, xv, B, col, ctl, spin_limit);
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u)
                    if (c + u < dj) s = s - fv[u] * as_f64(xv[u]);
            }
            st_final<S>(x + (int64_t)i * B + col, s);
        }
    }
}

template <Scope S>
__global__ __launch_bounds__(64) void k_backward_batch(PatDev P, const double* __restrict__ F,
                                                       int32_t B, const double* __restrict__ x,
                                                       double* y, Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, parts, run, t)) break;
        const int32_t ir = (int32_t)(t / (uint32_t)G);
        const int32_t i = P.permU ? P.permU[ir] : n - 1 - ir;
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t dj = P.diagF[i], re = P.rpF[i + 1];
            double s = x[(int64_t)i * B + col];
            const double fii = F[dj * B + col];
            // right to left: slots re-1, re-2, ..., dj+1
            for (int64_t c = re - 1; c > dj; c -= kSolveChunk) {
                double fv[kSolveChunk];
                uint64_t yv[kSolveChunk];
                int32_t jj[kSolveChunk];
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    const int64_t cc = std::max<int64_t>(c - u, dj + 1);
                    jj[u] = P.ciF[cc];
                    fv[u] = F[cc * B + col];
                    yv[u] = ld_cached(y + (int64_t)jj[u] * B + col);
                }
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u)
                    if (c - u <= dj) yv[u] = 0ull;
                settle(y, jj, yv, B, col, ctl, spin_limit);
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u)
                    if (c - u > dj) s = s - fv[u] * as_f64(yv[u]);
            }
            st_final<S>(y + (int64_t)i * B + col, s / fii);
        }
    }
}

// single instance: grid > 0 wavefront per row (one_xcd: grid wavefronts per
// XCD launched, those of one XCD working), grid < 0 lane per row with -grid
// wavefronts (the one-workgroup shape is launch_solve_cu)
hipError_t launch_forward(const PatDev& P, const double* f_val, int32_t batch, const double* b,
                          double* x, Ctl* ctl, uint64_t spin_limit, int32_t grid, bool one_xcd,
                          hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch == 1 && grid < 0)
        hipLaunchKernelGGL(k_solve_lanes<false>, dim3(-grid), dim3(64), 0, s, P, f_val, b, x, ctl, spin_limit);
    else if (batch == 1 && one_xcd)
        hipLaunchKernelGGL(k_forward_row<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, f_val, b, x, ctl,
                           spin_limit);
    else if (batch == 1)
        hipLaunchKernelGGL(k_forward_row<Scope::Device>, dim3(grid), dim3(64), 0, s, P, f_val, b, x, ctl,
                           spin_limit);
    else if (one_xcd)
        hipLaunchKernelGGL(k_forward_batch<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, f_val, batch, b, x, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_forward_batch<Scope::Device>, dim3(grid), dim3(64), 0, s, P, f_val, batch, b, x, ctl, spin_limit);
    return hipGetLastError();
}

hipError_t launch_backward(const PatDev& P, const double* f_val, int32_t batch, const double* x,
                           double* y, Ctl* ctl, uint64_t spin_limit, int32_t grid, bool one_xcd,
                           hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch == 1 && grid < 0)
        hipLaunchKernelGGL(k_solve_lanes<true>, dim3(-grid), dim3(64), 0, s, P, f_val, x, y, ctl, spin_limit);
    else if (batch == 1 && one_xcd)
        hipLaunchKernelGGL(k_backward_row<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, f_val, x, y,
                           ctl, spin_limit);
    else if (batch == 1)
        hipLaunchKernelGGL(k_backward_row<Scope::Device>, dim3(grid), dim3(64), 0, s, P, f_val, x, y, ctl,
                           spin_limit);
    else if (one_xcd)
        hipLaunchKernelGGL(k_backward_batch<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, f_val, batch, x, y, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_backward_batch<Scope::Device>, dim3(grid), dim3(64), 0, s, P, f_val, batch, x, y, ctl, spin_limit);
    return hipGetLastError();
}

}  // namespace tpilu
