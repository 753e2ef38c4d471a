// Reverse mode on gfx950: adjoint of b -> y = U~^-1 L~^-1 b and of the
// elimination that produced F (reverse sweep of Eqs. 6a/6b).
//
// The sequential reverse sweep undoes rows in descending order; the pivot h
// of row j then scatters fbar_ht -= fbar_jt * l into row h.  A scatter from
// many rows at once would need floating-point atomics and lose the order, so
// the GPU turns it into a gather: row h, once every row j > h that pivots on
// it is done, pulls those contributions itself in descending j -- the same
// order as the sequential sweep, hence the same bits.  "Rows that pivot on
// h" is column h of the strict lower part (a CSC built once per pattern),
// and the (t) positions come from the Phase II update schedule.  Values
// handed between rows (lbar of every pivot, final adjoints of every row)
// travel through kPending-initialised arrays as in the forward kernels.
//
// Batches use one task per (row, instance), instances strided in memory.
// Tasks are handed out by dependency level of the transposed sweep (rows of
// one level hold no dependencies on each other), so the rows in flight at any
// moment are ones whose inputs are about to be ready.
#include "kernels.h"

namespace tpilu {

// ----------------------------------------------------------------------------------
// CSC of the strict lower and strict upper parts of F
// ----------------------------------------------------------------------------------
__global__ void k_tcount(int32_t n, const int64_t* __restrict__ rpF, const int32_t* __restrict__ ciF,
                         const int32_t* __restrict__ diagF, int32_t* cntL, int32_t* cntU) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t d = diagF[r];
    for (int64_t s = rpF[r]; s < rpF[r + 1]; ++s) {
        if (s < d) atomicAdd(&cntL[ciF[s]], 1);
        else if (s > d) atomicAdd(&cntU[ciF[s]], 1);
    }
}

hipError_t launch_transpose_count(int32_t n, const int64_t* rpF, const int32_t* ciF,
                                  const int32_t* diagF, int32_t* cntL, int32_t* cntU,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_tcount, dim3((n + 255) / 256), dim3(256), 0, s, n, rpF, ciF, diagF, cntL, cntU);
    return hipGetLastError();
}

__global__ void k_tfill(int32_t n, const int64_t* __restrict__ rpF, const int32_t* __restrict__ ciF,
                        const int32_t* __restrict__ diagF, const int64_t* __restrict__ tpL,
                        int32_t* tsL, int32_t* trL, const int64_t* __restrict__ tpU, int32_t* tsU,
                        int32_t* trU, int32_t* curL, int32_t* curU) {
    int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t d = diagF[r];
    for (int64_t s = rpF[r]; s < rpF[r + 1]; ++s) {
        const int32_t c = ciF[s];
        if (s < d) {
            const int64_t pos = tpL[c] + atomicAdd(&curL[c], 1);
            tsL[pos] = (int32_t)s;
            trL[pos] = r;
        } else if (s > d) {
            const int64_t pos = tpU[c] + atomicAdd(&curU[c], 1);
            tsU[pos] = (int32_t)s;
            trU[pos] = r;
        }
    }
}

hipError_t launch_transpose_fill(int32_t n, const int64_t* rpF, const int32_t* ciF,
                                 const int32_t* diagF, const int64_t* tpL, int32_t* tsL,
                                 int32_t* trL, const int64_t* tpU, int32_t* tsU, int32_t* trU,
                                 int32_t* curL, int32_t* curU, hipStream_t s) {
    hipLaunchKernelGGL(k_tfill, dim3((n + 255) / 256), dim3(256), 0, s, n, rpF, ciF, diagF, tpL, tsL,
                       trL, tpU, tsU, trU, curL, curU);
    return hipGetLastError();
}

// sort each column's entries by row (insertion sort; columns are short)
__global__ void k_tsort(int32_t n, const int64_t* __restrict__ tp, int32_t* ts, int32_t* tr) {
    int32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t a = tp[c], b = tp[c + 1];
    for (int64_t i = a + 1; i < b; ++i) {
        const int32_t kr = tr[i], ks = ts[i];
        int64_t j = i - 1;
        while (j >= a && tr[j] > kr) {
            tr[j + 1] = tr[j];
            ts[j + 1] = ts[j];
            --j;
        }
        tr[j + 1] = kr;
        ts[j + 1] = ks;
    }
}

hipError_t launch_sort_columns(int32_t n, const int64_t* tp, int32_t* ts, int32_t* tr,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_tsort, dim3((n + 255) / 256), dim3(256), 0, s, n, tp, ts, tr);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// transposed solves
// ----------------------------------------------------------------------------------
// z = U~^-T ybar: i ascending, z_i = (ybar_i - sum_{j<i} f_ji z_j) / f_ii
// (S == Scope::Xcd: single instance, every wavefront on one XCD, as the
// forward and backward solves)
template <Scope S>
__global__ __launch_bounds__(64) void k_adj_solve_u(PatDev P, AdjPat T, const double* __restrict__ F,
                                                    int32_t B, const double* __restrict__ ybar,
                                                    double* z, Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)B;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, parts, run, t)) break;
        const int32_t i = T.permUT[t / (uint32_t)B];
        const int32_t b = (int32_t)(t % (uint32_t)B);
        // rows j < i of column i, taken in ascending j
        const int64_t a0 = T.tpU[i], a1 = T.tpU[i + 1];
        double s = sanitize_input(ybar[(int64_t)i * B + b], ctl);
        double fii = 0.0;  // read before the chain on one XCD, after it device-wide
        if constexpr (S == Scope::Xcd) fii = F[(int64_t)P.diagF[i] * B + b];
        for (int64_t c = a0; c < a1; c += kWave) {
            const int32_t cnt = (int32_t)min<int64_t>(kWave, a1 - c);
            double f = 0.0;
            const double* src = z;
            if (lane < cnt) {
                f = F[(int64_t)T.tsU[c + lane] * B + b];
                src = z + (int64_t)T.trU[c + lane] * B + b;
            }
            s = chain_sub<S>(s, cnt, f, src, ctl, spin_limit);
        }
        if constexpr (S != Scope::Xcd) fii = F[(int64_t)P.diagF[i] * B + b];
        const double r = s / fii;
        if (lane == 0) st_final<S>(z + (int64_t)i * B + b, r);
    }
}

// w = L~^-T z: i descending, w_i = z_i - sum_{j>i} f_ji w_j, j descending
template <Scope S>
__global__ __launch_bounds__(64) void k_adj_solve_l(PatDev P, AdjPat T, const double* __restrict__ F,
                                                    int32_t B, const double* __restrict__ z,
                                                    double* w, Ctl* ctl, uint64_t spin_limit) {
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(ctl)) return;
    }
    const uint32_t parts = S == Scope::Xcd ? 1u : (uint32_t)P.parts;
    const int lane = lane_id();
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)B;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, parts, run, t)) break;
        const int32_t i = T.permLT[t / (uint32_t)B];
        const int32_t b = (int32_t)(t % (uint32_t)B);
        // rows j > i of column i, taken in descending j
        const int64_t a0 = T.tpL[i], a1 = T.tpL[i + 1];
        double s = z[(int64_t)i * B + b];
        for (int64_t c = 0; c < a1 - a0; c += kWave) {
            const int32_t cnt = (int32_t)min<int64_t>(kWave, a1 - a0 - c);
            double f = 0.0;
            const double* src = w;
            if (lane < cnt) {
                const int64_t a = a1 - 1 - (c + lane);
                f = F[(int64_t)T.tsL[a] * B + b];
                src = w + (int64_t)T.trL[a] * B + b;
            }
            s = chain_sub<S>(s, cnt, f, src, ctl, spin_limit);
        }
        if (lane == 0) st_final<S>(w + (int64_t)i * B + b, s);
    }
}

// ----------------------------------------------------------------------------------
// batches: one wavefront per (row, group of 64 instances), lanes = instances, each
// lane running the row's sequential chain for its own instance (values are stored
// entry-major, instance-minor, so the 64 lanes read one contiguous line per entry).
// One draw from the task counters covers a row for 64 instances instead of one.
// ----------------------------------------------------------------------------------
constexpr int kAdjChunk = 8;  // chain entries whose inputs are loaded together

__global__ __launch_bounds__(64) void k_adj_solve_u_batch(PatDev P, AdjPat T, const double* __restrict__ F,
                                                          int32_t B, const double* __restrict__ ybar,
                                                          double* z, Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, (uint32_t)P.parts, run, t)) break;
        const int32_t i = T.permUT[t / (uint32_t)G];
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t a0 = T.tpU[i], a1 = T.tpU[i + 1];
            double s = sanitize_input(ybar[(int64_t)i * B + col], ctl);
            const double fii = F[(int64_t)P.diagF[i] * B + col];
            for (int64_t c = a0; c < a1; c += kAdjChunk) {  // rows j < i of column i, ascending
                double fv[kAdjChunk];
                uint64_t zv[kAdjChunk];
                int32_t jj[kAdjChunk];
                // unconditional loads at clamped entries (the extra ones unused),
                // pending values re-read together
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u) {
                    const int64_t cc = std::min<int64_t>(c + u, a1 - 1);
                    jj[u] = T.trU[cc];
                    fv[u] = F[(int64_t)T.tsU[cc] * B + col];
                    zv[u] = ld_cached(z + (int64_t)jj[u] * B + col);
                }
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u)
                    if (c + u >= a1) zv[u] = 0ull;
                settle(z, jj, zv, B, col, ctl, spin_limit);
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u)
                    if (c + u < a1) s = s - fv[u] * as_f64(zv[u]);
            }
            st_publish(z + (int64_t)i * B + col, s / fii);
        }
    }
}

__global__ __launch_bounds__(64) void k_adj_solve_l_batch(PatDev P, AdjPat T, const double* __restrict__ F,
                                                          int32_t B, const double* __restrict__ z,
                                                          double* w, Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, (uint32_t)P.parts, run, t)) break;
        const int32_t i = T.permLT[t / (uint32_t)G];
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        if (col < B) {
            const int64_t a0 = T.tpL[i], a1 = T.tpL[i + 1];
            double s = z[(int64_t)i * B + col];
            for (int64_t c = a1 - 1; c >= a0; c -= kAdjChunk) {  // rows j > i of column i, descending
                double fv[kAdjChunk];
                uint64_t wv[kAdjChunk];
                int32_t jj[kAdjChunk];
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u) {
                    const int64_t cc = std::max<int64_t>(c - u, a0);
                    jj[u] = T.trL[cc];
                    fv[u] = F[(int64_t)T.tsL[cc] * B + col];
                    wv[u] = ld_cached(w + (int64_t)jj[u] * B + col);
                }
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u)
                    if (c - u < a0) wv[u] = 0ull;
                settle(w, jj, wv, B, col, ctl, spin_limit);
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u)
                    if (c - u >= a0) s = s - fv[u] * as_f64(wv[u]);
            }
            st_publish(w + (int64_t)i * B + col, s);
        }
    }
}

hipError_t launch_adj_solve_u(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* ybar, double* z, Ctl* ctl,
                              uint64_t spin_limit, int32_t grid, bool one_xcd, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch > 1)
        hipLaunchKernelGGL(k_adj_solve_u_batch, dim3(grid), dim3(64), 0, s, P, T, f_val, batch, ybar, z, ctl,
                           spin_limit);
    else if (one_xcd)
        hipLaunchKernelGGL(k_adj_solve_u<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, T, f_val, batch,
                           ybar, z, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_adj_solve_u<Scope::Device>, dim3(grid), dim3(64), 0, s, P, T, f_val, batch, ybar, z,
                           ctl, spin_limit);
    return hipGetLastError();
}

hipError_t launch_adj_solve_l(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* z, double* w, Ctl* ctl,
                              uint64_t spin_limit, int32_t grid, bool one_xcd, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (batch > 1)
        hipLaunchKernelGGL(k_adj_solve_l_batch, dim3(grid), dim3(64), 0, s, P, T, f_val, batch, z, w, ctl,
                           spin_limit);
    else if (one_xcd)
        hipLaunchKernelGGL(k_adj_solve_l<Scope::Xcd>, dim3(grid * kXcds), dim3(64), 0, s, P, T, f_val, batch, z,
                           w, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_adj_solve_l<Scope::Device>, dim3(grid), dim3(64), 0, s, P, T, f_val, batch, z, w,
                           ctl, spin_limit);
    return hipGetLastError();
}

// fbar_ij = -(z_i y_j) on U~ (j >= i); fbar_ih = -(w_i x_h) below the diagonal
__global__ void k_adj_fbar(PatDev P, int32_t B, const double* __restrict__ x,
                           const double* __restrict__ y, const double* __restrict__ z,
                           const double* __restrict__ w, double* __restrict__ fbar) {
    const int64_t task = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (task >= (int64_t)P.n * B) return;
    const int32_t i = (int32_t)(task / B);
    const int32_t b = (int32_t)(task % B);
    const int64_t rs = P.rpF[i], re = P.rpF[i + 1], d = P.diagF[i];
    const double wi = w[(int64_t)i * B + b], zi = z[(int64_t)i * B + b];
    for (int64_t q = rs; q < d; ++q) fbar[q * B + b] = -(wi * x[(int64_t)P.ciF[q] * B + b]);
    for (int64_t q = d; q < re; ++q) fbar[q * B + b] = -(zi * y[(int64_t)P.ciF[q] * B + b]);
}

hipError_t launch_adj_fbar(const PatDev& P, int32_t batch, const double* x, const double* y,
                           const double* z, const double* w, double* fbar, hipStream_t s) {
    const int64_t tasks = (int64_t)P.n * batch;
    if (tasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_fbar, dim3((unsigned)((tasks + 255) / 256)), dim3(256), 0, s, P, batch,
                       x, y, z, w, fbar);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// reverse sweep of the elimination
// ----------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_adj_numeric(PatDev P, AdjPat T, const double* __restrict__ F,
                                                    int32_t B, const double* __restrict__ fin,
                                                    double* G, double* lbar_out,
                                                    double* __restrict__ abar, Ctl* ctl,
                                                    uint64_t spin_limit) {
    extern __shared__ double W[];
    const int lane = lane_id();
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)B;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, (uint32_t)P.parts, run, t)) break;
        const int32_t j = T.permLT[t / (uint32_t)B];
        const int32_t b = (int32_t)(t % (uint32_t)B);
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1], dj = P.diagF[j];
        const int32_t len = (int32_t)(re - rs);
        for (int32_t e = lane; e < len; e += kWave) W[e] = sanitize_input(fin[(rs + e) * B + b], ctl);
        wave_sync();
        const double ujj = F[dj * B + b];
        // contributions of the rows i > j that pivot on j, in descending i
        for (int64_t a = T.tpL[j + 1] - 1; a >= T.tpL[j]; --a) {
            const int64_t s = T.tsL[a];  // slot of f_ij in row i
            const double l = F[s * B + b];
            const int64_t e0 = P.sptr[s], e1 = P.sptr[s + 1];
            for (int64_t e = e0 + lane; e < e1; e += kWave) {
                const int32_t q = P.sq[e];  // slot in row j
                const int32_t p = P.sp[e];  // slot in row i
                const double gv = wait_final(G + (int64_t)p * B + b, ctl, spin_limit);
                W[q - rs] = W[q - rs] - gv * l;
            }
            if (lane == 0) {
                const double lb = wait_final(lbar_out + s * B + b, ctl, spin_limit);
                double tmp = lb * l;
                tmp = tmp / ujj;
                W[dj - rs] = W[dj - rs] - tmp;
            }
            wave_sync();
        }
        // own pivots, descending
        for (int64_t s = dj - 1; s >= rs; --s) {
            double lb = W[s - rs];
            const int64_t e0 = P.sptr[s], e1 = P.sptr[s + 1];
            for (int64_t c = e0; c < e1; c += kWave) {
                const int64_t e = c + lane;
                double prod = 0.0;
                if (e < e1) prod = W[P.sp[e] - rs] * F[(int64_t)P.sq[e] * B + b];
                const int32_t cnt = (int32_t)min<int64_t>(kWave, e1 - c);
                for (int32_t k = 0; k < cnt; ++k) lb = lb - bcast_lane(prod, k);
            }
            if (lane == 0) {
                st_publish(lbar_out + s * B + b, lb);
                W[s - rs] = lb / F[(int64_t)P.lsd[s] * B + b];
            }
            wave_sync();
        }
        for (int64_t p = P.rpA[j] + lane; p < P.rpA[j + 1]; p += kWave)
            abar[p * B + b] = W[P.a2f[p] - rs];
        for (int32_t e = lane; e < len; e += kWave) st_publish(G + (rs + e) * B + b, W[e]);
        wave_sync();
    }
}

// Reverse sweep for batches: lanes = instances, the working row in LDS as
// [slot][lane]; the same operations in the same order as k_adj_numeric, each
// lane on its own instance.
// Inputs of a task that no other task writes (the row's own pivot
// diagonals and update values, the l of the rows that pivot on it) are staged
// in LDS at the start, a batch of loads per round trip, so that once the last
// dependency has arrived only the polled values remain on the task's path.
constexpr int kAdjPairCap = 32;  // own update pairs staged
constexpr int kAdjRowCap = 16;   // rows pivoting on the task's row staged
constexpr int kAdjLCap = 64;     // own pivots staged
constexpr int kAdjRPairCap = 64; // update pairs of the staged rows

size_t adj_numeric_batch_lds(int32_t max_row, bool stage) {
    const size_t rows = (size_t)std::max(max_row, 1) * (stage ? 2 : 1) + (stage ? kAdjPairCap + kAdjRowCap : 0);
    return rows * sizeof(double) * kWave;
}

__global__ __launch_bounds__(64) void k_adj_numeric_batch(PatDev P, AdjPat T, const double* __restrict__ F,
                                                          int32_t B, const double* __restrict__ fin,
                                                          double* Gv, double* lbar_out,
                                                          double* __restrict__ abar, Ctl* ctl,
                                                          uint64_t spin_limit, int32_t max_row, int32_t stage) {
    extern __shared__ double W[];  // [max_row][64]; staged: Ud [max_row][64], Pv [pairs][64], La [rows][64]
    double* Ud = W + (size_t)std::max(max_row, 1) * kWave;
    double* Pv = Ud + (size_t)std::max(max_row, 1) * kWave;
    double* La = Pv + (size_t)kAdjPairCap * kWave;
    __shared__ int32_t sla[kAdjRowCap];       // slot of f_ij of the staged rows i
    __shared__ int32_t psp[kAdjPairCap];      // own pairs: slot in row j minus its start
    __shared__ int32_t pof[kAdjLCap + 1];     // own pivots: first pair, relative
    __shared__ int32_t rq[kAdjRPairCap];      // pairs of the staged rows: slot in row j minus its start
    __shared__ int32_t rp[kAdjRPairCap];      // ... and slot in row i
    __shared__ int32_t rof[kAdjRowCap + 1];   // first pair of each staged row, relative
    const int lane = lane_id();
    const int32_t G = (B + kWave - 1) / kWave;
    const uint32_t ntask = (uint32_t)P.n * (uint32_t)G;
    PosRun run;
    for (;;) {
        uint32_t t;
        if (!next_pos(ctl, ntask, 1u, (uint32_t)P.parts, run, t)) break;
        const int32_t j = T.permLT[t / (uint32_t)G];
        const int32_t col = (int32_t)(t % (uint32_t)G) * kWave + lane;
        const int64_t rs = P.rpF[j], re = P.rpF[j + 1], dj = P.diagF[j];
        const int32_t len = (int32_t)(re - rs);
        const int64_t a0 = T.tpL[j], a1 = T.tpL[j + 1];
        const int64_t q0 = P.sptr[rs], q1 = P.sptr[dj];
        const bool st_own = stage && q1 - q0 <= kAdjPairCap && dj - rs <= kAdjLCap;
        bool st_rows = stage && a1 - a0 <= kAdjRowCap;
        // uniform metadata first, with the whole wavefront active
        if (st_own) {
            for (int64_t e = q0 + lane; e < q1; e += kWave) psp[e - q0] = P.sp[e] - (int32_t)rs;
            for (int64_t sl = rs + lane; sl <= dj; sl += kWave) pof[sl - rs] = (int32_t)(P.sptr[sl] - q0);
        }
        if (st_rows) {
            // lane k < a1 - a0: row a0 + k, its slot and its pair range
            const int32_t k = lane;
            const bool in = k < a1 - a0;
            const int32_t slk = in ? T.tsL[a0 + k] : 0;
            const int64_t pb = in ? P.sptr[slk] : 0, pe = in ? P.sptr[slk + 1] : 0;
            // exclusive prefix of the pair counts, lanes in order
            int32_t cnt = (int32_t)(pe - pb), pre = cnt;
            for (int off = 1; off < kWave; off <<= 1) {
                const int32_t o = __shfl_up(pre, off);
                if (k >= off) pre += o;
            }
            const int32_t total = __shfl(pre, kWave - 1);
            pre -= cnt;
            if (total > kAdjRPairCap) {
                st_rows = false;
            } else {
                if (in) {
                    sla[k] = slk;
                    rof[k] = pre;
                }
                if (k == 0) rof[a1 - a0] = total;
                wave_sync();
                for (int32_t r = 0; r < (int32_t)(a1 - a0); ++r) {
                    const int64_t b0 = P.sptr[sla[r]];
                    const int32_t o0 = rof[r], o1 = rof[r + 1];
                    if (lane < o1 - o0) {
                        rq[o0 + lane] = P.sq[b0 + lane] - (int32_t)rs;
                        rp[o0 + lane] = P.sp[b0 + lane];
                    }
                }
            }
        }
        wave_sync();
        if (col < B) {
            for (int32_t e0 = 0; e0 < len; e0 += kAdjChunk) {
                double v[kAdjChunk];
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u) v[u] = fin[(rs + std::min(e0 + u, len - 1)) * B + col];
#pragma unroll
                for (int u = 0; u < kAdjChunk; ++u)
                    if (e0 + u < len) W[(e0 + u) * kWave + lane] = sanitize_input(v[u], ctl);
            }
            const double ujj = F[dj * B + col];
            if (stage) {
                for (int64_t c = rs; c < dj; c += kAdjChunk) {
                    double v[kAdjChunk];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        v[u] = F[(int64_t)P.lsd[std::min<int64_t>(c + u, dj - 1)] * B + col];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        if (c + u < dj) Ud[(c + u - rs) * kWave + lane] = v[u];
                }
            }
            if (st_own) {
                for (int64_t c = q0; c < q1; c += kAdjChunk) {
                    double v[kAdjChunk];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        v[u] = F[(int64_t)P.sq[std::min<int64_t>(c + u, q1 - 1)] * B + col];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        if (c + u < q1) Pv[(c + u - q0) * kWave + lane] = v[u];
                }
            }
            if (st_rows) {
                for (int64_t c = a0; c < a1; c += kAdjChunk) {
                    double v[kAdjChunk];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        v[u] = F[(int64_t)sla[std::min<int64_t>(c + u, a1 - 1) - a0] * B + col];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        if (c + u < a1) La[(c + u - a0) * kWave + lane] = v[u];
                }
            }
            // contributions of the rows i > j that pivot on j, in descending i
            for (int64_t a = a1 - 1; a >= a0; --a) {
                const int64_t sl = st_rows ? sla[a - a0] : T.tsL[a];  // slot of f_ij in row i
                const double l = st_rows ? La[(a - a0) * kWave + lane] : F[sl * B + col];
                const uint64_t lb0 = ld_cached(lbar_out + sl * B + col);
                if (st_rows) {
                    const int32_t o0 = rof[a - a0], o1 = rof[a - a0 + 1];
                    for (int32_t c = o0; c < o1; c += kAdjChunk) {
                        uint64_t gv[kAdjChunk];
                        int32_t pp[kAdjChunk];
#pragma unroll
                        for (int u = 0; u < kAdjChunk; ++u) {
                            pp[u] = rp[std::min(c + u, o1 - 1)];
                            gv[u] = ld_cached(Gv + (int64_t)pp[u] * B + col);
                        }
#pragma unroll
                        for (int u = 0; u < kAdjChunk; ++u)
                            if (c + u >= o1) gv[u] = 0ull;
                        settle(Gv, pp, gv, B, col, ctl, spin_limit);
#pragma unroll
                        for (int u = 0; u < kAdjChunk; ++u) {
                            if (c + u < o1) {
                                const int32_t q = rq[c + u] * kWave + lane;
                                W[q] = W[q] - as_f64(gv[u]) * l;
                            }
                        }
                    }
                    const double lb = wait_final(lbar_out + sl * B + col, lb0, ctl, spin_limit);
                    double tmp = lb * l;
                    tmp = tmp / ujj;
                    W[(dj - rs) * kWave + lane] = W[(dj - rs) * kWave + lane] - tmp;
                    continue;
                }
                const int64_t e0 = P.sptr[sl], e1 = P.sptr[sl + 1];
                for (int64_t c = e0; c < e1; c += kAdjChunk) {
                    uint64_t gv[kAdjChunk];
                    int32_t pq[kAdjChunk], pp[kAdjChunk];
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u) {
                        const int64_t cc = std::min<int64_t>(c + u, e1 - 1);
                        pq[u] = P.sq[cc];  // slot in row j
                        pp[u] = P.sp[cc];  // slot in row i
                        gv[u] = ld_cached(Gv + (int64_t)pp[u] * B + col);
                    }
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u)
                        if (c + u >= e1) gv[u] = 0ull;
                    settle(Gv, pp, gv, B, col, ctl, spin_limit);
#pragma unroll
                    for (int u = 0; u < kAdjChunk; ++u) {
                        if (c + u < e1) {
                            const int64_t q = (pq[u] - rs) * kWave + lane;
                            W[q] = W[q] - as_f64(gv[u]) * l;
                        }
                    }
                }
                const double lb = wait_final(lbar_out + sl * B + col, lb0, ctl, spin_limit);
                double tmp = lb * l;
                tmp = tmp / ujj;
                W[(dj - rs) * kWave + lane] = W[(dj - rs) * kWave + lane] - tmp;
            }
            // own pivots, descending
            for (int64_t sl = dj - 1; sl >= rs; --sl) {
                double lb = W[(sl - rs) * kWave + lane];
                if (st_own) {
                    for (int32_t e = pof[sl - rs]; e < pof[sl - rs + 1]; ++e)
                        lb = lb - W[psp[e] * kWave + lane] * Pv[e * kWave + lane];
                } else {
                    for (int64_t e = P.sptr[sl]; e < P.sptr[sl + 1]; ++e)
                        lb = lb - W[(P.sp[e] - rs) * kWave + lane] * F[(int64_t)P.sq[e] * B + col];
                }
                st_publish(lbar_out + sl * B + col, lb);
                const double u = stage ? Ud[(sl - rs) * kWave + lane] : F[(int64_t)P.lsd[sl] * B + col];
                W[(sl - rs) * kWave + lane] = lb / u;
            }
            for (int64_t p = P.rpA[j]; p < P.rpA[j + 1]; ++p)
                abar[p * B + col] = W[(P.a2f[p] - rs) * kWave + lane];
            for (int32_t e = 0; e < len; ++e) st_publish(Gv + (rs + e) * B + col, W[e * kWave + lane]);
        }
        wave_sync();
    }
}

hipError_t launch_adj_numeric(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* fbar_in, double* G, double* lbar,
                              double* abar, Ctl* ctl, uint64_t spin_limit, int32_t grid,
                              int32_t max_row, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    const bool stage = adj_numeric_batch_lds(max_row, true) <= 64 * 1024;  // rows of up to 40 entries
    const size_t lds_batch = adj_numeric_batch_lds(max_row, stage);
    if (batch > 1 && lds_batch <= 64 * 1024) {  // rows of up to 128 entries
        hipLaunchKernelGGL(k_adj_numeric_batch, dim3(grid), dim3(64), lds_batch, s, P, T, f_val, batch, fbar_in,
                           G, lbar, abar, ctl, spin_limit, max_row, stage ? 1 : 0);
    } else {
        size_t lds = (size_t)std::max(max_row, 1) * sizeof(double);
        hipLaunchKernelGGL(k_adj_numeric, dim3(grid), dim3(64), lds, s, P, T, f_val, batch, fbar_in, G,
                           lbar, abar, ctl, spin_limit);
    }
    return hipGetLastError();
}

}  // namespace tpilu
