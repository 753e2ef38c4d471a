// Phase II on gfx950: row-wise IKJ elimination (Eq. 2 read as running
// updates, Eqs. 5a/5b), bit-identical to the sequential order.
//
// The only order that fixes the bits is, per entry f_jt, its updates in
// ascending pivot h.  A persistent grid hands rows out in ascending order
// through an atomic ticket, so a wavefront only ever waits on rows that some
// running wavefront already holds (no deadlock for any grid size).  One
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
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->ticket = 0;
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

// Wait until pivot row h's diagonal (slot dh) and every value f_ht that the
// pivot contributes (pairs [ea, eb) of the staged group) are final.  All of
// them are polled in the same round, so a row that is waiting on h pays one
// round trip after h is published, not one for the diagonal and another for
// the rest.  Final values are written back into the staged copies.  Returns
// the diagonal's bits (a quiet NaN after a watchdog timeout or abort).
__device__ __forceinline__ uint64_t wait_pivot(const double* F, int32_t dh, uint64_t ub, int32_t ea,
                                               int32_t eb, const int32_t* pr_q, uint64_t* pr_v,
                                               Ctl* ctl, uint64_t limit) {
    const int lane = lane_id();
    uint32_t polls = 0;
    uint64_t t0 = 0;
    for (;;) {
        bool pend = false;
        if (ub == kPending) {
            ub = ld_coherent(F + dh);
            pend = ub == kPending;
        }
        for (int32_t e = ea + lane; e < eb; e += kWave) {
            if (pr_v[e] == kPending) {
                const uint64_t v = ld_coherent(F + pr_q[e]);
                if (v != kPending) pr_v[e] = v;
                else pend = true;
            }
        }
        if (!__any(pend)) return ub;
        if ((polls & 31u) == 0u) {
            if ((polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u) return kQNaN;
            const uint64_t now = wall_clock64();
            if (polls == 0) {
                t0 = now;
            } else if (now - t0 > limit) {
                if (lane == 0) {
                    atomicOr(&ctl->status, kStTimeout);
                    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return kQNaN;
            }
        }
        ++polls;
        __builtin_amdgcn_s_sleep(1);
    }
}

// ----------------------------------------------------------------------------------
// single instance: one wavefront per row, lanes over the updates of a pivot
// ----------------------------------------------------------------------------------
constexpr int kPivCap = 128;   // pivots staged per group
constexpr int kPairCap = 512;  // update pairs staged per group

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
    const int lane = lane_id();
    const int32_t n = P.n;
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= (uint32_t)n) break;
        const int32_t j = P.permL ? P.permL[t] : (int32_t)t;
        trace_mark(P.trace, j);
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1];
        const int32_t len = (int32_t)(re - rs);
        const int64_t dj = P.diagF[j];
        for (int32_t e = lane; e < len; e += kWave) W[e] = 0.0;
        wave_sync();
        for (int64_t p = P.rpA[j] + lane; p < P.rpA[j + 1]; p += kWave)
            W[P.a2f[p] - rs] = sanitize_input(a_val[p], ctl);
        wave_sync();

        int64_t s0 = rs;
        while (s0 < dj) {
            int32_t np = (int32_t)std::min<int64_t>(dj - s0, kPivCap);
            const int64_t e0 = P.sptr[s0];
            for (int32_t i = lane; i <= np; i += kWave) {
                int64_t v = P.sptr[s0 + i] - e0;
                piv_e[i] = (int32_t)std::min<int64_t>(v, 0x7fffffff);
            }
            wave_sync();
            int32_t fit = 0;
            for (int32_t i = 1 + lane; i <= np; i += kWave) fit += piv_e[i] <= kPairCap ? 1 : 0;
            for (int off = 32; off > 0; off >>= 1) fit += __shfl_xor(fit, off);
            np = uniform(fit > 0 ? fit : 1);
            const int32_t npair = uniform(piv_e[np]);
            const bool big = npair > kPairCap;  // a single pivot with more pairs than fit
            for (int32_t i = lane; i < np; i += kWave) {
                const int32_t dh = P.lsd[s0 + i];
                piv_dh[i] = dh;
                piv_u[i] = ld_cached(F + dh);
            }
            if (!big) {
                for (int32_t e = lane; e < npair; e += kWave) {
                    const int32_t q = P.sq[e0 + e];
                    pr_q[e] = q;
                    pr_p[e] = (int32_t)(P.sp[e0 + e] - rs);
                    pr_v[e] = ld_cached(F + q);
                }
            }
            wave_sync();
            for (int32_t i = 0; i < np; ++i) {
                const int64_t s = s0 + i;
                uint64_t ub = piv_u[i];
                const int32_t ea = piv_e[i], eb = piv_e[i + 1];
                if (!big) {
                    // the pivot and every value it contributes, polled together
                    bool ok = ub != kPending;
                    for (int32_t e = ea + lane; e < eb; e += kWave) ok = ok && pr_v[e] != kPending;
                    if (!__all(ok)) ub = wait_pivot(F, piv_dh[i], ub, ea, eb, pr_q, pr_v, ctl, spin_limit);
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
                        W[p] = W[p] - l * v;
                    }
                } else {
                    for (int64_t e = e0 + lane; e < e0 + npair; e += kWave) {
                        const int32_t q = P.sq[e];
                        const int32_t p = (int32_t)(P.sp[e] - rs);
                        const double v = wait_final(F + q, ctl, spin_limit);
                        W[p] = W[p] - l * v;
                    }
                }
                wave_sync();
            }
            s0 += np;
        }
        const int32_t dl = (int32_t)(dj - rs);
        if (lane == 0 && W[dl] == 0.0) atomicMin(&ctl->bad_row, (unsigned long long)j);
        if ((int64_t)j != skip_row) {
            // U part first: later rows wait on it; the L part is only read by later kernels
            for (int32_t e = dl + lane; e < len; e += kWave) st_publish(F + rs + e, W[e]);
            for (int32_t e = lane; e < dl; e += kWave) F[rs + e] = W[e];
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

__global__ __launch_bounds__(64) void k_numeric_batch(PatDev P, const double* __restrict__ a_val,
                                                      int32_t B, double* F, Ctl* ctl,
                                                      uint64_t spin_limit, int64_t skip_row) {
    extern __shared__ double W[];  // [len][64]
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
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= ntask) break;
        const int32_t jr = (int32_t)(t / (uint32_t)G);
        const int32_t j = P.permL ? P.permL[jr] : jr;
        const int32_t g = (int32_t)(t % (uint32_t)G);
        const int32_t col = g * kWave + lane;
        const bool act = col < B;
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1];
        const int32_t len = (int32_t)(re - rs);
        const int64_t dj = P.diagF[j];
        for (int32_t e = 0; e < len; ++e) W[e * kWave + lane] = 0.0;
        for (int64_t p = P.rpA[j]; p < P.rpA[j + 1]; ++p) {
            const int64_t sl = P.a2f[p] - rs;
            if (act) W[sl * kWave + lane] = sanitize_input(a_val[p * B + col], ctl);
        }
        int64_t s0 = rs;
        while (s0 < dj) {
            int32_t np = (int32_t)std::min<int64_t>(dj - s0, kBPivCap);
            const int64_t e0 = P.sptr[s0];
            wave_sync();
            if (lane <= np) piv_e[lane] = (int32_t)std::min<int64_t>(P.sptr[s0 + lane] - e0, 0x7fffffff);
            wave_sync();
            int32_t fit = 0;
            for (int32_t i = 1; i <= np; ++i) fit += piv_e[i] <= kBPairCap ? 1 : 0;
            np = uniform(fit > 0 ? fit : 1);
            const int32_t npair = uniform(piv_e[np]);
            const bool big = npair > kBPairCap;
            if (lane < np) piv_dh[lane] = P.lsd[s0 + lane];
            if (!big && lane < npair) {
                pr_q[lane] = P.sq[e0 + lane];
                pr_p[lane] = (int32_t)(P.sp[e0 + lane] - rs);
            }
            wave_sync();
            if (act) {
                for (int32_t i = 0; i < np; ++i)
                    vu[i * kWave + lane] = ld_cached(F + (int64_t)piv_dh[i] * B + col);
                if (!big)
                    for (int32_t e = 0; e < npair; ++e)
                        vv[e * kWave + lane] = ld_cached(F + (int64_t)pr_q[e] * B + col);
            }
            if (act) {
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
                            W[p * kWave + lane] = W[p * kWave + lane] - l * v;
                        }
                    } else {
                        for (int64_t e = e0; e < e0 + npair; ++e) {
                            const int32_t q = P.sq[e];
                            const int64_t p = P.sp[e] - rs;
                            const double v = wait_final(F + (int64_t)q * B + col, ctl, spin_limit);
                            W[p * kWave + lane] = W[p * kWave + lane] - l * v;
                        }
                    }
                }
            }
            s0 += np;
        }
        const int32_t dl = (int32_t)(dj - rs);
        if (act && W[dl * kWave + lane] == 0.0) atomicMin(&ctl->bad_row, (unsigned long long)j);
        if (act && (int64_t)j != skip_row) {
            for (int32_t e = dl; e < len; ++e) st_publish(F + (rs + e) * B + col, W[e * kWave + lane]);
            for (int32_t e = 0; e < dl; ++e) F[(rs + e) * B + col] = W[e * kWave + lane];
        }
        wave_sync();
    }
}

int numeric_grid(int32_t batch, int32_t max_row, int num_cu) {
    // LDS per wavefront bounds how many rows are in flight; aim for the
    // resident maximum so every ready row has a wavefront
    size_t lds;
    if (batch == 1)
        lds = (size_t)max_row * 8 + (kPivCap + 1) * 4 + kPivCap * 12 + kPairCap * 16;
    else
        lds = (size_t)max_row * 8 * kWave + (kBPivCap + 1) * 4 + kBPivCap * 4 + kBPairCap * 8 +
              (kBPivCap + kBPairCap) * 8 * kWave;
    size_t per_cu = std::max<size_t>(1, (160 * 1024) / std::max<size_t>(lds, 1));
    per_cu = std::min<size_t>(per_cu, 32);
    return (int)(per_cu * (size_t)num_cu);
}

hipError_t launch_numeric(const PatDev& P, const double* a_val, int32_t batch, double* f_val,
                          Ctl* ctl, uint64_t spin_limit, int64_t skip_row, int32_t grid,
                          int32_t max_row, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch == 1) {
        size_t lds = (size_t)std::max(max_row, 1) * sizeof(double);
        hipLaunchKernelGGL(k_numeric_row, dim3(grid), dim3(64), lds, s, P, a_val, f_val, ctl,
                           spin_limit, skip_row);
    } else {
        size_t lds = (size_t)std::max(max_row, 1) * sizeof(double) * kWave;
        hipLaunchKernelGGL(k_numeric_batch, dim3(grid), dim3(64), lds, s, P, a_val, batch, f_val,
                           ctl, spin_limit, skip_row);
    }
    return hipGetLastError();
}

}  // namespace tpilu
