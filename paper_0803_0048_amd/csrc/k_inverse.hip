// Level-based incomplete inverses (Sec. 3.5) on gfx950.
//
// L~^-1 keeps the strict lower pattern of F: its entry at (i, t) is -beta_it
// with beta_it = f_it - sum over pivots h of row i with t < h, taken in
// ascending h, of f_ih beta_ht (Eqs. 5, 6c, 6d).  U~^-1 keeps the upper
// pattern: row i is (e_i - sum over pivots j > i of row i, right to left, of
// u_ij (row j of the inverse)) / u_ii, rows from the last to the first.
// Both are stored in G, an array shaped like F.
//
// Phase I part (once per pattern): for every kept entry (i, t), the list of
// its updates -- the row-local slot of the multiplier (f_ih or u_ij) and the
// slot of the partner entry (beta_ht or g_jt) in the other row -- in the
// order above.  One wavefront per row: row i's columns sit in LDS and every
// column of a pivot row's half is binary-searched there.
//
// Values: a persistent grid walks the rows in dependency-level order (the
// forward DAG for L~, the backward DAG for U~) through the task counters.
// Unlike the elimination, the entries of one row do not depend on each other
// here, so each lane owns entries of the row and runs their chains alone:
// loads of up to kInvChunk partners in flight together, pending ones (rows
// still being produced) re-polled every round, the row's entries published
// the moment they are final.  G starts as kPending.
//
// Applying them (Eq. 3a): x_i = sum_{t<i} G_it p_t + p_i, y_i = sum_{t>=i}
// G_it x_t, each row summed from +0.0 in ascending column order, either by one
// thread per row or by a wavefront per row (products in parallel, added in
// that order); both give the same bits.
#include "kernels.h"

namespace tpilu {

// ----------------------------------------------------------------------------------
// update lists
// ----------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_isched(int32_t n, const int64_t* __restrict__ rpF,
                                               const int32_t* __restrict__ ciF,
                                               const int32_t* __restrict__ diagF, int upper, int pass,
                                               int32_t* __restrict__ tcount, const int64_t* __restrict__ tptr,
                                               int32_t* __restrict__ ps, int32_t* __restrict__ pq) {
    extern __shared__ int64_t ish[];
    const int lane = lane_id();
    for (int32_t j = blockIdx.x; j < n; j += gridDim.x) {
        const int64_t rs = rpF[j], re = rpF[j + 1];
        const int32_t len = (int32_t)(re - rs), dl = (int32_t)(diagF[j] - rs);
        int64_t* Tp = ish;                                          // [len]
        int32_t* cols = reinterpret_cast<int32_t*>(ish + len);     // [len]
        int32_t* cur = cols + len;                                  // [len]
        for (int32_t e = lane; e < len; e += kWave) {
            cols[e] = ciF[rs + e];
            cur[e] = 0;
            if (pass == 1) Tp[e] = tptr[rs + e];
        }
        wave_sync();
        // pivots in the order the lists come out: ascending for L~, descending for U~
        const int32_t np = upper ? len - dl - 1 : dl;
        const int32_t lo0 = upper ? dl : 0, hi0 = upper ? len - 1 : dl - 1;
        for (int32_t k = 0; k < np; ++k) {
            const int32_t sl = upper ? len - 1 - k : k;
            const int32_t h = cols[sl];
            const int64_t a = upper ? (int64_t)diagF[h] : rpF[h];
            const int64_t b = upper ? rpF[h + 1] : (int64_t)diagF[h];
            for (int64_t q0 = a; q0 < b; q0 += kWave) {
                const int64_t q = q0 + lane;
                int32_t pos = -1;
                if (q < b) {
                    const int32_t t = ciF[q];
                    int32_t lo = lo0, hi = hi0;
                    while (lo <= hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        const int32_t c = cols[mid];
                        if (c == t) { pos = mid; break; }
                        if (c < t) lo = mid + 1;
                        else hi = mid - 1;
                    }
                }
                if (pos >= 0) {
                    // the targets of one pivot are distinct, so no two lanes share pos
                    if (pass == 1) {
                        const int64_t o = Tp[pos] + cur[pos];
                        ps[o] = sl;
                        pq[o] = (int32_t)q;
                    }
                    cur[pos] = cur[pos] + 1;
                }
            }
            wave_sync();
        }
        if (pass == 0)
            for (int32_t e = lane + lo0; e <= hi0; e += kWave) tcount[rs + e] = cur[e];
        wave_sync();
    }
}

size_t isched_lds_bytes(int32_t max_row) { return (size_t)std::max(max_row, 1) * 16; }

hipError_t launch_isched(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF, int upper,
                         int pass, int32_t* tcount, const int64_t* tptr, int32_t* ps, int32_t* pq,
                         int32_t max_row, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_isched, dim3(std::min(n, 65536)), dim3(64), isched_lds_bytes(max_row), s, n, rpF, ciF,
                       diagF, upper, pass, tcount, tptr, ps, pq);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// values
// ----------------------------------------------------------------------------------
// entries whose partner values are loaded together (random banded n=160,000
// ILU(2), both halves: 2 / 4 / 8 measured 6.2 / 6.3 / 7.1 ms)
constexpr int kInvChunk = 2;

template <bool kUpper>
__global__ __launch_bounds__(64) void k_inverse(PatDev P, InvSched S, const double* __restrict__ F, double* G,
                                                Ctl* ctl, uint64_t spin_limit) {
    const int lane = lane_id();
    const int32_t n = P.n;
    const int32_t* perm = kUpper ? P.permU : P.permL;
    PosRun run;
    for (;;) {
        uint32_t tk;
        if (!next_pos(ctl, (uint32_t)n, (uint32_t)(kUpper ? P.groupU : P.groupL), (uint32_t)P.parts, run, tk)) break;
        const int32_t i = perm ? perm[tk] : (kUpper ? n - 1 - (int32_t)tk : (int32_t)tk);
        const int64_t rs = P.rpF[i], dj = P.diagF[i];
        const int64_t p0 = kUpper ? dj : rs, p1 = kUpper ? P.rpF[i + 1] : dj;
        const double uii = kUpper ? F[dj] : 1.0;
        bool stop = false;
        for (int64_t pb = p0; pb < p1 && !stop; pb += kWave) {
            const int64_t p = pb + lane;
            bool done = p >= p1;
            int64_t e = 0, ee = 0;
            double acc = 0.0;
            if (!done) {
                e = S.ptr[p];
                ee = S.ptr[p + 1];
                acc = kUpper ? (p == dj ? 1.0 : 0.0) : F[p];
            }
            double fv[kInvChunk];
            uint64_t gv[kInvChunk];
            int32_t gq[kInvChunk];
            int32_t cnt = 0, u = 0;
            uint32_t polls = 0;
            uint64_t t0 = 0;
            for (;;) {
                bool prog = false;
                if (!done) {
                    if (u == cnt && e < ee) {
                        cnt = (int32_t)min<int64_t>(kInvChunk, ee - e);
#pragma unroll
                        for (int k = 0; k < kInvChunk; ++k) {
                            if (k < cnt) {
                                fv[k] = F[rs + S.s[e + k]];
                                gq[k] = S.q[e + k];
                                gv[k] = ld_cached(G + gq[k]);
                            }
                        }
                        e += cnt;
                        u = 0;
                    }
                    bool blocked = false;
#pragma unroll
                    for (int k = 0; k < kInvChunk; ++k) {
                        if (k >= u && k < cnt && !blocked) {
                            if (gv[k] == kPending) {
                                blocked = true;
                            } else {
                                // L~: the partner holds -beta_ht; beta_ht = -(that) exactly
                                const double g = kUpper ? as_f64(gv[k]) : -as_f64(gv[k]);
                                acc = acc - fv[k] * g;
                                u = k + 1;
                                prog = true;
                            }
                        }
                    }
                    if (u == cnt && e >= ee) {
                        st_publish(G + p, kUpper ? acc / uii : -acc);
                        done = true;
                        prog = true;
                    } else if (blocked) {
#pragma unroll
                        for (int k = 0; k < kInvChunk; ++k)
                            if (k >= u && k < cnt && gv[k] == kPending) gv[k] = ld_coherent(G + gq[k]);
                    }
                }
                if (__all(done)) break;
                if (__any(prog)) {
                    polls = 0;
                    continue;
                }
                ++polls;
                if ((polls & 31u) == 0u) {
                    bool halt = (polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u;
                    const uint64_t now = wall_clock64();
                    if (polls == 32u) {
                        t0 = now;
                    } else if (now - t0 > spin_limit) {
                        if (lane == 0) {
                            atomicOr(&ctl->status, kStTimeout);
                            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        halt = true;
                    }
                    if (__any(halt)) {
                        stop = true;
                        break;
                    }
                }
            }
        }
        if (stop)  // after an abort, release anything that might wait on this row
            for (int64_t p = p0 + lane; p < p1; p += kWave) st_publish(G + p, as_f64(kQNaN));
    }
}

hipError_t launch_inverse(const PatDev& P, const InvSched& S, const double* f_val, double* g_val, bool upper,
                          Ctl* ctl, uint64_t spin_limit, int32_t grid, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (upper)
        hipLaunchKernelGGL(k_inverse<true>, dim3(grid), dim3(64), 0, s, P, S, f_val, g_val, ctl, spin_limit);
    else
        hipLaunchKernelGGL(k_inverse<false>, dim3(grid), dim3(64), 0, s, P, S, f_val, g_val, ctl, spin_limit);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------------
// applying them: two products
// ----------------------------------------------------------------------------------
// one wavefront per row: products in parallel, their sum in order (one
// lane's chain broadcast across the wavefront; best for long, uneven rows)
template <bool kUpper>
__global__ __launch_bounds__(64) void k_apply_inverse_wave(PatDev P, const double* __restrict__ G,
                                                           const double* __restrict__ in, double* __restrict__ out) {
    const int lane = lane_id();
    for (int32_t i = blockIdx.x; i < P.n; i += gridDim.x) {
        const int64_t dj = P.diagF[i];
        const int64_t a = kUpper ? dj : P.rpF[i], b = kUpper ? P.rpF[i + 1] : dj;
        double s = 0.0;
        for (int64_t c = a; c < b; c += kWave) {
            const int32_t cnt = (int32_t)min<int64_t>(kWave, b - c);
            double prod = 0.0;
            if (lane < cnt) prod = G[c + lane] * in[P.ciF[c + lane]];
            for (int32_t k = 0; k < cnt; ++k) s = s + bcast_lane(prod, k);
        }
        if (!kUpper) s = s + in[i];
        if (lane == 0) out[i] = s;
    }
}

// 64 rows per wavefront, lane r owning row r0 + r and adding its products in
// order.  The wavefront stages the next kTile entries of all 64 rows in LDS
// with coalesced loads (each load instruction covers kTile consecutive
// entries of 64 / kTile rows), then every lane walks its own row there: the
// in-order sum of a row is one lane's chain, so the wavefront's 64 chains run
// side by side instead of one at a time.
// kTile entries per row per staging round (at most 32: one bit per staged
// slice in `on`): 8 for short rows (a round of 16 mostly stages nothing;
// 7-point 64^3 ILU(1), about 6 entries per half: 0.021 ms with 8, 0.042 with
// 16, both products), else 32 (27-point 50^3 ILU(3), about 82 per half: 0.084
// ms with 32, 0.101 with 16; random banded n=160,000 ILU(2): 0.220 / 0.237 ms).
// Rows in their natural order, 64 consecutive ones to a wavefront: their
// entries and the in_j they gather lie close together.  (Sorting the rows by
// length so that a wavefront's lanes finish together measured slower on every
// pattern tried, even and uneven alike.)
template <bool kUpper, int kTile>
__global__ __launch_bounds__(64) void k_apply_inverse_tile(PatDev P, const double* __restrict__ G,
                                                      const double* __restrict__ in, double* __restrict__ out) {
    constexpr int kTileStride = kTile + 1;  // odd stride: lanes reading their rows hit distinct banks
    __shared__ double tv[kWave * kTileStride];  // the staged products g_ij * in_j
    const int lane = lane_id();
    for (int64_t r0 = (int64_t)blockIdx.x * kWave; r0 < P.n; r0 += (int64_t)gridDim.x * kWave) {
        const bool has = r0 + lane < P.n;
        const int64_t i = has ? r0 + lane : 0;
        int64_t a = 0, b = 0;
        if (has) {
            const int64_t dj = P.diagF[i];
            a = kUpper ? dj : P.rpF[i];
            b = kUpper ? P.rpF[i + 1] : dj;
        }
        int64_t len = b - a, maxlen = len;
        for (int off = 32; off > 0; off >>= 1) maxlen = max(maxlen, (int64_t)__shfl_xor(maxlen, off));
        double s = 0.0;
        for (int64_t k0 = 0; k0 < maxlen; k0 += kTile) {
            // stage the products of entries k0 .. k0+kTile-1 of every row:
            // instruction u takes rows u*(64/kTile) .. +(64/kTile)-1, kTile
            // consecutive entries each, so both the entries and the gathered
            // in_j of one row (sorted columns, often close together) come in
            // whole lines; each lane then adds its own row's products in order
            // in three phases (column and value loads of every u, then the
            // gathers, then the products), so a round costs two memory
            // latencies; entries past a row's end load a clamped, in-bounds
            // slot and are not stored
            int32_t cu[kTile];
            double gu[kTile];
            uint32_t on = 0u;
            const int kk = lane % kTile;  // entry of the row's slice
#pragma unroll
            for (int u = 0; u < kTile; ++u) {
                const int rr = u * (kWave / kTile) + lane / kTile;  // row of the tile
                const int64_t ar = __shfl(a, rr), br = __shfl(b, rr);
                const int64_t e = ar + k0 + kk;
                if (e < br) on |= 1u << u;
                const int64_t ec = e < br ? e : (br > ar ? br - 1 : 0);
                cu[u] = P.ciF[ec];
                gu[u] = G[ec];
            }
#pragma unroll
            for (int u = 0; u < kTile; ++u) gu[u] = gu[u] * in[cu[u]];
#pragma unroll
            for (int u = 0; u < kTile; ++u)
                if (on & (1u << u)) tv[(u * (kWave / kTile) + lane / kTile) * kTileStride + kk] = gu[u];
            wave_sync();
            const int32_t cnt = (int32_t)max<int64_t>(0, min<int64_t>(kTile, len - k0));
#pragma unroll
            for (int kk = 0; kk < kTile; ++kk)
                if (kk < cnt) s = s + tv[lane * kTileStride + kk];
            wave_sync();
        }
        if (has) {
            if (!kUpper) s = s + in[i];
            out[i] = s;
        }
    }
}

// one thread per row: the row's products and their sum in order, no
// cross-lane traffic (rows of a wavefront are consecutive, so each thread's
// consecutive entries share cache lines across iterations)
template <bool kUpper>
__global__ __launch_bounds__(256) void k_apply_inverse_rows(PatDev P, const double* __restrict__ G,
                                                            const double* __restrict__ in,
                                                            double* __restrict__ out) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P.n) return;
    const int64_t dj = P.diagF[i];
    const int64_t a = kUpper ? dj : P.rpF[i], b = kUpper ? P.rpF[i + 1] : dj;
    double s = 0.0;
    for (int64_t q = a; q < b; ++q) s = s + G[q] * in[P.ciF[q]];
    if (!kUpper) s = s + in[i];
    out[i] = s;
}

hipError_t launch_apply_inverse(const PatDev& P, const double* g_val, const double* b, double* x, double* y,
                                int shape, hipStream_t s) {
    if (P.n <= 0) return hipSuccess;
    if (shape == kProdThreadRows) {
        const int grid = (P.n + 255) / 256;
        hipLaunchKernelGGL(k_apply_inverse_rows<false>, dim3(grid), dim3(256), 0, s, P, g_val, b, x);
        hipLaunchKernelGGL(k_apply_inverse_rows<true>, dim3(grid), dim3(256), 0, s, P, g_val, x, y);
    } else if (shape == kProdTile || shape == kProdTileShort) {
        const int grid = std::min((P.n + kWave - 1) / kWave, 65536);
        if (shape == kProdTileShort) {
            hipLaunchKernelGGL((k_apply_inverse_tile<false, 8>), dim3(grid), dim3(64), 0, s, P, g_val, b, x);
            hipLaunchKernelGGL((k_apply_inverse_tile<true, 8>), dim3(grid), dim3(64), 0, s, P, g_val, x, y);
        } else {
            hipLaunchKernelGGL((k_apply_inverse_tile<false, 32>), dim3(grid), dim3(64), 0, s, P, g_val, b, x);
            hipLaunchKernelGGL((k_apply_inverse_tile<true, 32>), dim3(grid), dim3(64), 0, s, P, g_val, x, y);
        }
    } else {
        const int grid = std::min(P.n, 65536);
        hipLaunchKernelGGL(k_apply_inverse_wave<false>, dim3(grid), dim3(64), 0, s, P, g_val, b, x);
        hipLaunchKernelGGL(k_apply_inverse_wave<true>, dim3(grid), dim3(64), 0, s, P, g_val, x, y);
    }
    return hipGetLastError();
}

}  // namespace tpilu
