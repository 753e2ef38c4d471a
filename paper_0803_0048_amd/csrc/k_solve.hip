// Applying M^-1 = U~^-1 L~^-1 (Eq. 1) on gfx950.
//
// forward  (Eq. 3b): x_i = b_i - f_ih1 x_h1 - f_ih2 x_h2 - ...   h ascending
// backward:          y_i = (x_i - f_ij1 y_j1 - f_ij2 y_j2 - ...) / f_ii, j ascending
//
// Both are dependency-driven persistent kernels (rows handed out through an
// atomic ticket: ascending for the forward sweep, descending for the
// backward sweep).  For one instance a wavefront owns a row: its lanes form
// the products f_ih * x_h in parallel (each rounded on its own) as the x_h
// arrive, and the running subtraction is then carried through the products
// strictly in ascending column order, which keeps every bit of the
// sequential result.  For batches the lanes are instances and each lane runs
// its own chain.  x and y start as kPending and each slot is written once.
#include "kernels.h"

namespace tpilu {

__global__ __launch_bounds__(64) void k_forward_row(PatDev P, const double* __restrict__ F,
                                                    const double* __restrict__ b, double* x,
                                                    Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= (uint32_t)n) break;
        const int32_t i = (int32_t)t;
        const int64_t rs = P.rpF[i], dj = P.diagF[i];
        const int32_t nl = (int32_t)(dj - rs);
        double s = sanitize_input(b[i], ctl);
        for (int32_t c = 0; c < nl; c += kWave) {
            const int32_t e = c + lane;
            double prod = 0.0;
            if (e < nl) {
                const int32_t h = P.ciF[rs + e];
                const double f = F[rs + e];
                const double xv = wait_final(x + h, ctl, spin_limit);
                prod = f * xv;
            }
            const int32_t cnt = min(kWave, nl - c);
            for (int32_t k = 0; k < cnt; ++k) s = s - bcast_lane(prod, k);
        }
        if (lane == 0) st_publish(x + i, s);
    }
}

__global__ __launch_bounds__(64) void k_backward_row(PatDev P, const double* __restrict__ F,
                                                     const double* __restrict__ x, double* y,
                                                     Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= (uint32_t)n) break;
        const int32_t i = n - 1 - (int32_t)t;
        const int64_t dj = P.diagF[i], re = P.rpF[i + 1];
        const int32_t nu = (int32_t)(re - dj - 1);
        double s = x[i];
        for (int32_t c = 0; c < nu; c += kWave) {
            const int32_t e = c + lane;
            double prod = 0.0;
            if (e < nu) {
                const int32_t jc = P.ciF[dj + 1 + e];
                const double f = F[dj + 1 + e];
                const double yv = wait_final(y + jc, ctl, spin_limit);
                prod = f * yv;
            }
            const int32_t cnt = min(kWave, nu - c);
            for (int32_t k = 0; k < cnt; ++k) s = s - bcast_lane(prod, k);
        }
        const double r = s / F[dj];
        if (lane == 0) st_publish(y + i, r);
    }
}

// batches: lanes are instances; each lane runs the sequential chain of its
// instance; the loads of a chunk of entries are issued before any of them is
// waited on
constexpr int kSolveChunk = 8;

__global__ __launch_bounds__(64) void k_forward_batch(PatDev P, const double* __restrict__ F,
                                                      int32_t B, const double* __restrict__ b,
                                                      double* x, Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)n * (uint32_t)G;
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= ntask) break;
        const int32_t i = (int32_t)(t / (uint32_t)G);
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t rs = P.rpF[i], dj = P.diagF[i];
            double s = sanitize_input(b[(int64_t)i * B + col], ctl);
            for (int64_t c = rs; c < dj; c += kSolveChunk) {
                double fv[kSolveChunk];
                uint64_t xv[kSolveChunk];
                int32_t hh[kSolveChunk];
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    if (c + u < dj) {
                        hh[u] = P.ciF[c + u];
                        fv[u] = F[(c + u) * B + col];
                        xv[u] = ld_cached(x + (int64_t)hh[u] * B + col);
                    }
                }
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    if (c + u < dj) {
                        const double xx = wait_final(x + (int64_t)hh[u] * B + col, xv[u], ctl, spin_limit);
                        s = s - fv[u] * xx;
                    }
                }
            }
            st_publish(x + (int64_t)i * B + col, s);
        }
    }
}

__global__ __launch_bounds__(64) void k_backward_batch(PatDev P, const double* __restrict__ F,
                                                       int32_t B, const double* __restrict__ x,
                                                       double* y, Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)n * (uint32_t)G;
    for (;;) {
        const uint32_t t = wave_ticket(ctl);
        if (t >= ntask) break;
        const int32_t i = n - 1 - (int32_t)(t / (uint32_t)G);
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t dj = P.diagF[i], re = P.rpF[i + 1];
            double s = x[(int64_t)i * B + col];
            for (int64_t c = dj + 1; c < re; c += kSolveChunk) {
                double fv[kSolveChunk];
                uint64_t yv[kSolveChunk];
                int32_t jj[kSolveChunk];
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    if (c + u < re) {
                        jj[u] = P.ciF[c + u];
                        fv[u] = F[(c + u) * B + col];
                        yv[u] = ld_cached(y + (int64_t)jj[u] * B + col);
                    }
                }
#pragma unroll
                for (int u = 0; u < kSolveChunk; ++u) {
                    if (c + u < re) {
                        const double yy = wait_final(y + (int64_t)jj[u] * B + col, yv[u], ctl, spin_limit);
                        s = s - fv[u] * yy;
                    }
                }
            }
            st_publish(y + (int64_t)i * B + col, s / F[dj * B + col]);
        }
    }
}

int solve_grid(int32_t batch, int num_cu) {
    (void)batch;
    return 16 * num_cu;
}

hipError_t launch_forward(const PatDev& P, const double* f_val, int32_t batch, const double* b,
                          double* x, Ctl* ctl, uint64_t spin_limit, int32_t grid, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch == 1)
        hipLaunchKernelGGL(k_forward_row, dim3(grid), dim3(64), 0, s, P, f_val, b, x, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_forward_batch, dim3(grid), dim3(64), 0, s, P, f_val, batch, b, x, ctl,
                           spin_limit);
    return hipGetLastError();
}

hipError_t launch_backward(const PatDev& P, const double* f_val, int32_t batch, const double* x,
                           double* y, Ctl* ctl, uint64_t spin_limit, int32_t grid, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch == 1)
        hipLaunchKernelGGL(k_backward_row, dim3(grid), dim3(64), 0, s, P, f_val, x, y, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_backward_batch, dim3(grid), dim3(64), 0, s, P, f_val, batch, x, y, ctl,
                           spin_limit);
    return hipGetLastError();
}

}  // namespace tpilu
