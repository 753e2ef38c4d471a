// Phase I on gfx950: the level-of-fill pattern (Def. 2.3, Algorithm 1), the
// map from A's entries to F's slots, and the per-row update schedule that
// Phase II replays.
//
// Algorithm 1 merges rows in ascending order, so row j can only be built
// after every row it pivots on.  On the GPU every row is built on its own,
// from the graph of A, using the fill-path form of the same levels: level(i,j)
// equals the least number of interior vertices of a path i -> j in the graph
// of A (edge u -> v for every stored a_uv) whose interior vertices are all
// smaller than min(i, j).  (Each term level(i,h) + level(h,j) + 1 of Def. 2.3
// joins a path to h and a path from h through vertex h itself, which is
// smaller than both ends.)  Algorithm 1 only minimises over entries that are
// themselves kept, but a path through an entry of level > k is already too
// long, so the two agree on every entry of level <= k.  Rows are therefore
// independent (the observation Sec. 3.3 makes for k = 1 holds for every k in
// this form) and one wavefront builds one row:
//
//   frontier_1 = { (v, v) : a_iv stored, v < i }      (vertex, largest interior)
//   depth d = 1..k:  every (v, M) in frontier_d and stored a_vj with j > M
//                    gives entry (i, j) a level candidate d;
//                    frontier_{d+1} = { (w, max(M, w)) : a_vw stored, w < i },
//                    keeping per w the smallest M, and dropping w when a
//                    shorter walk already reached it with an interior maximum
//                    no larger (that state can only lead to higher levels).
//   level 0 for every stored a_ij.
//
// Per-row sets live in LDS hash maps; a row that does not fit is redone by
// the same code with the maps in global memory sized for any row.
#include "kernels.h"

namespace tpilu {

// ------------------------------------------------------------------------------------
// validation
// ------------------------------------------------------------------------------------
__global__ void k_validate(int32_t n, int64_t nnz, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, uint32_t* status) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i > n) return;
    uint32_t bad = 0;
    if (i == 0 && rp[0] != 0) bad |= kValBadRowptr;
    if (i == n) {
        if (rp[n] != nnz) bad |= kValBadRowptr;
    } else {
        int64_t a = rp[i], b = rp[i + 1];
        if (a > b || a < 0 || b > nnz) {
            bad |= kValBadRowptr;
        } else {
            bool diag = false;
            int32_t prev = -1;
            for (int64_t p = a; p < b; ++p) {
                int32_t c = ci[p];
                if (c < 0 || c >= n) { bad |= kValBadCol; break; }
                if (c <= prev) bad |= kValUnsorted;
                if (c == i) diag = true;
                prev = c;
            }
            if (!diag) bad |= kValNoDiag;
        }
    }
    if (bad) atomicOr(status, bad);
}

hipError_t launch_validate(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                           uint32_t* status, hipStream_t s) {
    int64_t threads = (int64_t)n + 1;
    int blocks = (int)((threads + 255) / 256);
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, s, n, nnz, rp, ci, status);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// hash maps (open addressing, linear probing) keyed by a vertex, value = min
// ------------------------------------------------------------------------------------
constexpr int32_t kEmpty = -1;
constexpr int32_t kBig = 0x7fffffff;

__device__ __forceinline__ uint32_t hslot(int32_t key, uint32_t mask) {
    uint32_t h = static_cast<uint32_t>(key) * 0x9E3779B1u;
    h ^= h >> 15;
    return h & mask;
}

// insert key (if absent) and lower its value to min(value, val); false if full
__device__ __forceinline__ bool map_min(int32_t* keys, int32_t* vals, uint32_t mask, int32_t key,
                                        int32_t val) {
    uint32_t h = hslot(key, mask);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        int32_t old = atomicCAS(&keys[h], kEmpty, key);
        if (old == kEmpty || old == key) {
            atomicMin(&vals[h], val);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

// map_min on the endpoint map of an LDS tier: an insert that finds no slot
// within kProbeMax probes fails, which the row then reports as overflowing
// (and the next tier builds it).  A linear-probing table near full makes
// every probe sequence long; giving up early keeps a row that will not fit
// from paying for a full table.
constexpr uint32_t kProbeMax = 64;
__device__ __forceinline__ bool map_min_bounded(int32_t* keys, int32_t* vals, uint32_t mask, int32_t key,
                                                int32_t val, uint32_t max_probe) {
    uint32_t h = hslot(key, mask);
    const uint32_t lim = min(max_probe, mask + 1u);
    for (uint32_t probe = 0; probe < lim; ++probe) {
        int32_t old = atomicCAS(&keys[h], kEmpty, key);
        if (old == kEmpty || old == key) {
            atomicMin(&vals[h], val);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

__device__ __forceinline__ int32_t map_get(const int32_t* keys, const int32_t* vals, uint32_t mask,
                                           int32_t key) {
    uint32_t h = hslot(key, mask);
    for (uint32_t probe = 0; probe <= mask; ++probe) {
        int32_t k = keys[h];
        if (k == key) return vals[h];
        if (k == kEmpty) return kBig;
        h = (h + 1) & mask;
    }
    return kBig;
}

struct SymWs {
    int32_t *ek, *ev;  // endpoint map: column -> level
    int32_t *bk, *bv;  // best interior maximum per vertex over all depths so far
    int32_t *ck, *cv;  // candidates of the next frontier
    int32_t *fv[2], *fm[2];  // frontier lists (vertex, interior maximum)
    int32_t *ok, *ol;  // compacted row (column, level)
    int32_t* ctr;      // [0],[1] frontier sizes, [2] overflow, [3] output size
    uint32_t emask, fmask, fcap;
    uint32_t eprobe;   // most probes of an endpoint insert before the row counts as overflowing
    uint32_t* bm;      // LDS tiers: the space of ok, reused as a bitmap of bm_bits columns
    uint32_t bm_bits;  //   (0: the global tier, which sorts its compacted row instead)
};

constexpr int32_t kSymSortMax = 512;  // longest row the sorting network orders

// exclusive prefix sum over the wavefront's lanes
__device__ __forceinline__ int32_t wave_excl_sum(int32_t v, int32_t& total) {
    const int lane = lane_id();
    int32_t x = v;
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    total = __shfl(x, kWave - 1);
    return x - v;
}

// Write row i of F (column, level) in ascending column order straight from
// the endpoint map: the map's columns are marked in a bitmap over a window
// of bm_bits columns, each lane takes a block of the window's words, a
// prefix over the lanes' bit counts gives every block its first output
// position, and the lane emits its block's columns in order, looking each
// level up in the map.  Windows follow each other from the row's smallest
// column to its largest.  O(row + column range / 32), against the
// O(row log^2 row) of a sorting network.
__device__ __forceinline__ void sym_emit_sorted(int32_t i, const int64_t* __restrict__ rpF, int32_t* __restrict__ ciF,
                                uint8_t* __restrict__ lvF, int32_t* __restrict__ diagF, const SymWs& W) {
    const int lane = lane_id();
    int32_t cmin = kBig, cmax = -1;
    for (uint32_t sl = lane; sl <= W.emask; sl += kWave) {
        const int32_t c = W.ek[sl];
        if (c != kEmpty) {
            cmin = min(cmin, c);
            cmax = max(cmax, c);
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        cmin = min(cmin, __shfl_xor(cmin, off));
        cmax = max(cmax, __shfl_xor(cmax, off));
    }
    const int64_t base = rpF[i];
    int64_t out = base;
    for (int64_t w0 = cmin; w0 <= cmax; w0 += W.bm_bits) {
        const int32_t span = (int32_t)min<int64_t>(W.bm_bits, (int64_t)cmax - w0 + 1);
        const int32_t nw = (span + 31) >> 5;
        for (int32_t x = lane; x < nw; x += kWave) W.bm[x] = 0u;
        wave_sync();
        for (uint32_t sl = lane; sl <= W.emask; sl += kWave) {
            const int32_t c = W.ek[sl];
            if (c != kEmpty && c >= w0 && c < w0 + span) {
                const int32_t o = (int32_t)(c - w0);
                atomicOr(&W.bm[o >> 5], 1u << (o & 31));
            }
        }
        wave_sync();
        const int32_t per = (nw + kWave - 1) / kWave;
        const int32_t wb = min(lane * per, nw), we = min(wb + per, nw);
        int32_t mine = 0;
        for (int32_t x = wb; x < we; ++x) mine += __popc(W.bm[x]);
        int32_t total = 0;
        int64_t r = out + wave_excl_sum(mine, total);
        for (int32_t x = wb; x < we; ++x) {
            uint32_t bits = W.bm[x];
            while (bits) {
                const int32_t b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const int32_t c = (int32_t)(w0 + x * 32 + b);
                const int32_t lev = map_get(W.ek, W.ev, W.emask, c);
                ciF[r] = c;
                lvF[r] = static_cast<uint8_t>(min(lev, 255));
                if (c == i) diagF[i] = static_cast<int32_t>(r);
                ++r;
            }
        }
        out += total;
        wave_sync();
    }
}

__device__ __forceinline__ void sym_row(int32_t i, const int64_t* __restrict__ rpA,
                                        const int32_t* __restrict__ ciA, int32_t k, int mode,
                                        int32_t* __restrict__ cnt, const int64_t* __restrict__ rpF,
                                        int32_t* __restrict__ ciF, uint8_t* __restrict__ lvF,
                                        int32_t* __restrict__ diagF, const SymWs& W) {
    const int lane = lane_id();
    for (uint32_t s = lane; s <= W.emask; s += kWave) { W.ek[s] = kEmpty; W.ev[s] = kBig; }
    for (uint32_t s = lane; s <= W.fmask; s += kWave) {
        W.bk[s] = kEmpty; W.bv[s] = kBig; W.ck[s] = kEmpty; W.cv[s] = kBig;
    }
    if (lane < 4) W.ctr[lane] = 0;
    wave_sync();
    const int64_t a0 = rpA[i], a1 = rpA[i + 1];
    for (int64_t p = a0 + lane; p < a1; p += kWave) {
        int32_t c = ciA[p];
        bool ok = map_min_bounded(W.ek, W.ev, W.emask, c, 0, W.eprobe);
        if (c < i) {
            int32_t slot = atomicAdd(&W.ctr[0], 1);
            if (slot < (int32_t)W.fcap) { W.fv[0][slot] = c; W.fm[0][slot] = c; }
            else ok = false;
            ok = map_min(W.bk, W.bv, W.fmask, c, c) && ok;
        }
        if (!ok) W.ctr[2] = 1;
    }
    wave_sync();
    int cur = 0;
    for (int32_t d = 1; d <= k; ++d) {
        const int32_t nf = uniform(min(W.ctr[cur], (int32_t)W.fcap));
        if (nf == 0 || uniform(W.ctr[2])) break;
        // endpoints reachable from this frontier in one more edge
        for (int32_t f = lane; f < nf; f += kWave) {
            if (W.ctr[2]) break;  // overflowing: the next tier builds this row
            int32_t v = (cur ? W.fv[1] : W.fv[0])[f], M = (cur ? W.fm[1] : W.fm[0])[f];
            for (int64_t p = rpA[v]; p < rpA[v + 1]; ++p) {
                int32_t j = ciA[p];
                if (j > M && !map_min_bounded(W.ek, W.ev, W.emask, j, d, W.eprobe)) {
                    W.ctr[2] = 1;
                    break;
                }
            }
        }
        if (d == k) break;
        wave_sync();
        if (uniform(W.ctr[2])) break;
        // next frontier
        for (int32_t f = lane; f < nf; f += kWave) {
            int32_t v = (cur ? W.fv[1] : W.fv[0])[f], M = (cur ? W.fm[1] : W.fm[0])[f];
            for (int64_t p = rpA[v]; p < rpA[v + 1]; ++p) {
                int32_t w = ciA[p];
                if (w < i && !map_min(W.ck, W.cv, W.fmask, w, max(M, w))) W.ctr[2] = 1;
            }
        }
        const int nxt = cur ^ 1;
        if (lane == 0) W.ctr[nxt] = 0;
        wave_sync();
        for (uint32_t s = lane; s <= W.fmask; s += kWave) {
            int32_t w = W.ck[s];
            if (w == kEmpty) continue;
            int32_t c = W.cv[s];
            W.ck[s] = kEmpty;
            W.cv[s] = kBig;
            if (c < map_get(W.bk, W.bv, W.fmask, w)) {
                bool ok = map_min(W.bk, W.bv, W.fmask, w, c);
                int32_t slot = atomicAdd(&W.ctr[nxt], 1);
                if (slot < (int32_t)W.fcap) { (nxt ? W.fv[1] : W.fv[0])[slot] = w; (nxt ? W.fm[1] : W.fm[0])[slot] = c; }
                else ok = false;
                if (!ok) W.ctr[2] = 1;
            }
        }
        wave_sync();
        cur = nxt;
    }
    wave_sync();
    if (uniform(W.ctr[2])) {
        if (mode == 0 && lane == 0) cnt[i] = -1;
        return;
    }
    if (W.bm_bits) {
        int32_t mine = 0;
        for (uint32_t sl = lane; sl <= W.emask; sl += kWave) mine += W.ek[sl] != kEmpty;
        for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
        if (mode == 0) {
            if (lane == 0) cnt[i] = mine;
            return;
        }
        // long rows: through the bitmap; short ones: the sorting network
        // below costs less than a pass over the column range
        if (mine > kSymSortMax) {
            sym_emit_sorted(i, rpF, ciF, lvF, diagF, W);
            return;
        }
    }
    // compact the row
    for (uint32_t s = lane; s <= W.emask; s += kWave) {
        int32_t c = W.ek[s];
        if (c != kEmpty) {
            int32_t idx = atomicAdd(&W.ctr[3], 1);
            W.ok[idx] = c;
            W.ol[idx] = W.ev[s];
        }
    }
    wave_sync();
    const int32_t len = uniform(W.ctr[3]);
    if (mode == 0) {
        if (lane == 0) cnt[i] = len;
        return;
    }
    // sort (column, level) by column: bitonic network over the next power of
    // two, padded with kBig (it fits: the map's capacity is a power of two)
    uint32_t np2 = 1;
    while (np2 < (uint32_t)len) np2 <<= 1;
    for (uint32_t e = len + lane; e < np2; e += kWave) { W.ok[e] = kBig; W.ol[e] = 0; }
    wave_sync();
    for (uint32_t kk = 2; kk <= np2; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
            for (uint32_t e = lane; e < np2; e += kWave) {
                const uint32_t f = e ^ jj;
                if (f > e) {
                    const int32_t a = W.ok[e], b = W.ok[f];
                    if ((a > b) == ((e & kk) == 0)) {
                        W.ok[e] = b;
                        W.ok[f] = a;
                        const int32_t la = W.ol[e];
                        W.ol[e] = W.ol[f];
                        W.ol[f] = la;
                    }
                }
            }
            wave_sync();
        }
    }
    const int64_t base = rpF[i];
    for (int32_t e = lane; e < len; e += kWave) {
        const int32_t key = W.ok[e];
        ciF[base + e] = key;
        lvF[base + e] = static_cast<uint8_t>(min(W.ol[e], 255));
        if (key == i) diagF[i] = static_cast<int32_t>(base + e);
    }
}

// kEnd: capacity of the endpoint map (and of the compacted row)
template <int kEnd>
__global__ __launch_bounds__(64) void k_sym_rows_lds(int32_t n, const int64_t* __restrict__ rpA,
                                                     const int32_t* __restrict__ ciA, int32_t k,
                                                     const int32_t* __restrict__ row_list,
                                                     int32_t n_rows, int mode,
                                                     int32_t* __restrict__ cnt,
                                                     const int64_t* __restrict__ rpF,
                                                     int32_t* __restrict__ ciF,
                                                     uint8_t* __restrict__ lvF,
                                                     int32_t* __restrict__ diagF,
                                                     const uint8_t* __restrict__ tier_of, int tier) {
    __shared__ int32_t ek[kEnd], ev[kEnd];
    __shared__ int32_t bk[kSymFrontCap], bv[kSymFrontCap], ck[kSymFrontCap], cv[kSymFrontCap];
    __shared__ int32_t f0v[kSymFrontCap], f0m[kSymFrontCap], f1v[kSymFrontCap], f1m[kSymFrontCap];
    __shared__ int32_t ok[kEnd], ol[kEnd];
    __shared__ int32_t ctr[4];
    SymWs W;
    W.ek = ek; W.ev = ev; W.bk = bk; W.bv = bv; W.ck = ck; W.cv = cv;
    W.fv[0] = f0v; W.fm[0] = f0m; W.fv[1] = f1v; W.fm[1] = f1m;
    W.ok = ok; W.ol = ol; W.ctr = ctr;
    W.emask = kEnd - 1; W.fmask = kSymFrontCap - 1; W.fcap = kSymFrontCap;
    W.eprobe = kProbeMax;
    W.bm = reinterpret_cast<uint32_t*>(ok);
    W.bm_bits = (uint32_t)kEnd * 32u;
    for (int32_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
        int32_t i = row_list ? row_list[r] : r;
        if (mode == 1 && tier_of && tier_of[i] != tier) continue;  // built by another tier
        sym_row(i, rpA, ciA, k, mode, cnt, rpF, ciF, lvF, diagF, W);
        wave_sync();
    }
    (void)n;
}

__host__ __device__ size_t sym_global_scratch_ints(int32_t n, uint32_t gcap) {
    // ek ev (gcap) bk bv ck cv (gcap) f0v f0m f1v f1m (n) ok ol (gcap) ctr (4, padded)
    return (size_t)gcap * 8 + (size_t)n * 4 + 64;
}

__global__ __launch_bounds__(64) void k_sym_rows_global(int32_t n, const int64_t* __restrict__ rpA,
                                                        const int32_t* __restrict__ ciA, int32_t k,
                                                        const int32_t* __restrict__ row_list,
                                                        int32_t n_rows, int mode,
                                                        int32_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ rpF,
                                                        int32_t* __restrict__ ciF,
                                                        uint8_t* __restrict__ lvF,
                                                        int32_t* __restrict__ diagF,
                                                        int32_t* gscratch, uint32_t gcap,
                                                        const uint8_t* __restrict__ tier_of) {
    int32_t* base = gscratch + (size_t)blockIdx.x * sym_global_scratch_ints(n, gcap);
    SymWs W;
    W.ek = base; W.ev = base + gcap;
    W.bk = base + 2 * (size_t)gcap; W.bv = base + 3 * (size_t)gcap;
    W.ck = base + 4 * (size_t)gcap; W.cv = base + 5 * (size_t)gcap;
    W.ok = base + 6 * (size_t)gcap; W.ol = base + 7 * (size_t)gcap;
    int32_t* fl = base + 8 * (size_t)gcap;
    W.fv[0] = fl; W.fm[0] = fl + n; W.fv[1] = fl + 2 * (size_t)n; W.fm[1] = fl + 3 * (size_t)n;
    W.ctr = fl + 4 * (size_t)n;
    W.emask = gcap - 1; W.fmask = gcap - 1; W.fcap = (uint32_t)n;
    W.eprobe = gcap;  // sized for any row (gcap >= 2n + 2): never gives up
    W.bm = nullptr;
    W.bm_bits = 0;
    for (int32_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
        int32_t i = row_list ? row_list[r] : r;
        if (mode == 1 && tier_of && tier_of[i] != 2) continue;
        sym_row(i, rpA, ciA, k, mode, cnt, rpF, ciF, lvF, diagF, W);
        wave_sync();
    }
}

hipError_t launch_sym_rows(int tier, int32_t n, const int64_t* rpA, const int32_t* ciA,
                           int32_t k, const int32_t* row_list, int32_t n_rows, int mode,
                           int32_t* cnt, const int64_t* rpF, int32_t* ciF, uint8_t* lvF,
                           int32_t* diagF, const uint8_t* tier_of, int32_t* gscratch, uint32_t gcap,
                           int32_t grid, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    if (tier == 2) {
        hipLaunchKernelGGL(k_sym_rows_global, dim3(grid), dim3(64), 0, s, n, rpA, ciA, k,
                           row_list, n_rows, mode, cnt, rpF, ciF, lvF, diagF, gscratch, gcap, tier_of);
    } else if (tier == 1) {
        hipLaunchKernelGGL(k_sym_rows_lds<kSymEndCapLong>, dim3(grid), dim3(64), 0, s, n, rpA, ciA, k,
                           row_list, n_rows, mode, cnt, rpF, ciF, lvF, diagF, tier_of, 1);
    } else {
        hipLaunchKernelGGL(k_sym_rows_lds<kSymEndCap>, dim3(grid), dim3(64), 0, s, n, rpA, ciA, k,
                           row_list, n_rows, mode, cnt, rpF, ciF, lvF, diagF, tier_of, 0);
    }
    return hipGetLastError();
}

// Routing of rows to the tiers before the count pass.  ub_i = |row i of A| +
// sum over stored a_ih, h < i, of the entries of row h right of h: every
// position of level <= 1 of row i is one of those terms (Def. 2.3 with one
// interior vertex), so for k = 1 it bounds the row's length, counting
// duplicates.  Rows whose bound passes `limit` go straight to the larger
// maps of tier 1: built in tier 0 they would only fill its map and be given
// up.  The routing only changes where a row is built, never what it holds
// (a row tier 1 cannot hold still goes on to the global tier).
__global__ void k_row_upper(int32_t n, const int64_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
                            int32_t* __restrict__ nup) {
    const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    int64_t lo = rpA[h], hi = rpA[h + 1];
    const int64_t end = hi;
    while (lo < hi) {  // first entry right of the diagonal
        const int64_t mid = (lo + hi) >> 1;
        if (ciA[mid] <= h) lo = mid + 1;
        else hi = mid;
    }
    nup[h] = (int32_t)(end - lo);
}

__global__ void k_route_rows(int32_t n, const int64_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
                             const int32_t* __restrict__ nup, int64_t limit, int32_t* __restrict__ list0,
                             int32_t* __restrict__ list1, int32_t* __restrict__ counts, uint8_t* __restrict__ tier_of) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t a0 = rpA[i], a1 = rpA[i + 1];
    int64_t ub = a1 - a0;
    for (int64_t p = a0; p < a1 && ub <= limit; ++p) {
        const int32_t h = ciA[p];
        if (h >= i) break;
        ub += nup[h];
    }
    if (ub > limit) {
        list1[atomicAdd(&counts[1], 1)] = i;
        tier_of[i] = 1;
    } else {
        list0[atomicAdd(&counts[0], 1)] = i;
    }
}

hipError_t launch_route_rows(int32_t n, const int64_t* rpA, const int32_t* ciA, int32_t* nup, int64_t limit,
                             int32_t* list0, int32_t* list1, int32_t* counts, uint8_t* tier_of, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_upper, dim3((n + 255) / 256), dim3(256), 0, s, n, rpA, ciA, nup);
    hipLaunchKernelGGL(k_route_rows, dim3((n + 255) / 256), dim3(256), 0, s, n, rpA, ciA, nup, limit, list0, list1,
                       counts, tier_of);
    return hipGetLastError();
}

int64_t sym_route_limit() { return (int64_t)(kSymEndCap - kSymEndCap / 8) * 5 / 4; }

__global__ void k_collect_overflow(int32_t n_rows, const int32_t* __restrict__ list,
                                   const int32_t* __restrict__ cnt, int32_t* row_list, int32_t* n_over,
                                   uint8_t* tier_of, int tier) {
    const int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rows) return;
    const int32_t i = list ? list[r] : r;
    if (cnt[i] < 0) {
        row_list[atomicAdd(n_over, 1)] = i;
        tier_of[i] = static_cast<uint8_t>(tier);
    }
}

hipError_t launch_collect_overflow(int32_t n_rows, const int32_t* list, const int32_t* cnt, int32_t* row_list,
                                   int32_t* n_over, uint8_t* tier_of, int tier, hipStream_t s) {
    if (n_rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_collect_overflow, dim3((n_rows + 255) / 256), dim3(256), 0, s, n_rows, list, cnt,
                       row_list, n_over, tier_of, tier);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// exclusive scan int32 -> int64 (three passes, 1024 elements per block)
// ------------------------------------------------------------------------------------
constexpr int kScanTile = 1024;

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[256];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int e = threadIdx.x; e < kScanTile; e += 256) {
        int64_t idx = base + e;
        if (idx < n) acc += in[idx];
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(1024) void k_scan_blocks(int64_t* bsum, int64_t nb) {
    // exclusive scan of nb block sums in place; bsum[nb] = total
    __shared__ int64_t sh[1024];
    int64_t per = (nb + 1023) / 1024;
    int64_t lo = threadIdx.x * per, hi = min(nb, lo + per);
    int64_t acc = 0;
    for (int64_t e = lo; e < hi; ++e) acc += bsum[e];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 1; w < 1024; w <<= 1) {
        int64_t v = (int)threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = threadIdx.x ? sh[threadIdx.x - 1] : 0;
    for (int64_t e = lo; e < hi; ++e) {
        int64_t v = bsum[e];
        bsum[e] = run;
        run += v;
    }
    if (threadIdx.x == 1023) bsum[nb] = sh[1023];
}

__global__ __launch_bounds__(256) void k_scan_final(const int32_t* __restrict__ in, int64_t n,
                                                    const int64_t* __restrict__ boff,
                                                    int64_t* __restrict__ out, int64_t nb) {
    __shared__ int64_t sh[256];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t v[4];
    int64_t loc = 0;
    for (int e = 0; e < 4; ++e) {
        int64_t idx = base + threadIdx.x * 4 + e;
        v[e] = idx < n ? in[idx] : 0;
        loc += v[e];
    }
    sh[threadIdx.x] = loc;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {
        int64_t t = (int)threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = boff[blockIdx.x] + (threadIdx.x ? sh[threadIdx.x - 1] : 0);
    for (int e = 0; e < 4; ++e) {
        int64_t idx = base + threadIdx.x * 4 + e;
        if (idx < n) out[idx] = run;
        run += v[e];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = boff[nb];
}

hipError_t launch_scan(const int32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s) {
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, tmp, (int64_t)0);
        hipLaunchKernelGGL(k_scan_final, dim3(1), dim3(256), 0, s, in, n, tmp, out, (int64_t)0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(256), 0, s, in, n, tmp, out, nb);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// A -> F slot map: merge of two sorted rows, one thread per row
// ------------------------------------------------------------------------------------
__global__ void k_a2f(int32_t n, const int64_t* __restrict__ rpA, const int32_t* __restrict__ ciA,
                      const int64_t* __restrict__ rpF, const int32_t* __restrict__ ciF,
                      int32_t* __restrict__ a2f, uint32_t* status) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t q = rpF[i], qe = rpF[i + 1];
    for (int64_t p = rpA[i]; p < rpA[i + 1]; ++p) {
        int32_t c = ciA[p];
        while (q < qe && ciF[q] < c) ++q;
        if (q < qe && ciF[q] == c) {
            a2f[p] = static_cast<int32_t>(q);
        } else {
            a2f[p] = -1;
            atomicOr(status, kValBadCol);
        }
    }
}

hipError_t launch_a2f(int32_t n, const int64_t* rpA, const int32_t* ciA, const int64_t* rpF,
                      const int32_t* ciF, int32_t* a2f, uint32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_a2f, dim3((n + 255) / 256), dim3(256), 0, s, n, rpA, ciA, rpF, ciF, a2f,
                       status);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Update schedule.  For every pivot slot s = (j, h) of F (h < j), the pairs
// (q, p) with q the slot of f_ht in row h and p the slot of f_jt in row j,
// for every t > h stored in both rows, in ascending t.  Phase II replays them
// (f_jt <- f_jt - f_jh * f_ht); their number is the number of updates.
// One wavefront per row j; row j's columns are staged in LDS and every
// candidate t of the pivot row is binary-searched there, inside one bucket of
// a directory over [c_min, c_max].  A column's bucket is (t - c_min) * mul >>
// 24 with mul = floor(kSchedDir * 2^24 / range), computed once per row (the
// same monotone map builds the directory and finds the bucket, so no
// candidate is missed); a 64-bit division per candidate cost more than the
// search itself.
// ------------------------------------------------------------------------------------
constexpr int kSchedDir = 1024;  // buckets of the column directory of row j
constexpr int kSchedUnroll = 8;  // 64-column chunks of a pivot row loaded per round

__device__ __forceinline__ int32_t sched_bucket(int64_t off, uint64_t mul) {
    return static_cast<int32_t>((static_cast<uint64_t>(off) * mul) >> 24);
}

// Modes: 0 counts the pairs of every pivot slot (scount) and records its
// pivot's diagonal slot (lsd); 1 writes them at sptr (the scan of the
// counts); 2 does both in one pass: the counts as mode 0, and the pairs, in
// order, to a pool.  A wavefront takes the pool a chunk of pool.chunk pairs
// at a time (one atomic per chunk) and writes each round's pairs straight
// into its chunk; a run of one row's pairs inside one chunk is a segment
// (row, index of its first pair within the row, pool position, count),
// closed when the row ends or the chunk is full.  k_sched_copy then moves
// each segment to sptr[first slot of its row] + that index.  If the pool or
// the segment list is too small, mode 2 raises *overflow and stops storing
// (the counts stay exact): the caller then runs mode 1.  Mode 3 only adds
// the sampled rows' pair count into sample[0] and their candidate count into
// sample[2] (rows j with j % stride == 0), to size the pool and to decide
// whether one pass pays.
// DirT: uint16_t when every row has fewer than 65536 entries (half the LDS
// of int32_t, which keeps more wavefronts resident: random n=160,000 ILU(1),
// rows of ~1,250 entries, 400 -> 332 ms with 1,024 buckets; 256 buckets of
// int32_t took 400 ms, 1,024 of int32_t 398 ms, 4,096 of uint16_t 412 ms).
// split > 1 (mode 3): each sampled row is shared by `split` wavefronts, each
// taking every split-th block of 64 pivots, so the few sampled rows still
// fill the device.
template <typename DirT>
__global__ __launch_bounds__(64) void k_sched(int32_t n, const int64_t* __restrict__ rpF,
                                              const int32_t* __restrict__ ciF,
                                              const int32_t* __restrict__ diagF, int mode,
                                              int32_t* __restrict__ scount, int32_t* __restrict__ lsd,
                                              const int64_t* __restrict__ sptr,
                                              int32_t* __restrict__ sq, int32_t* __restrict__ sp,
                                              SchedPool pool, int32_t max_row, int32_t stride,
                                              int32_t split) {
    extern __shared__ int32_t colsj[];
    // Row j's sorted columns get a directory: bucket b of [c_min, c_max]
    // holds the columns at positions dir[b] .. dir[b+1]-1, so a candidate t
    // is searched among a handful of columns instead of the whole row.
    __shared__ DirT dir[kSchedDir + 1];
    // the pivots of the row, 64 at a time: diagonal slot and row end of each
    __shared__ int32_t pdh[kWave], phe[kWave];
    __shared__ int64_t pout[kWave];
    const int lane = lane_id();
    const bool counts = mode == 0 || mode == 2;
    int64_t cbase = -1;          // mode 2: pool position of the wavefront's chunk (-2: pool exhausted)
    int32_t used = 0, seg0 = 0;  // pairs used in the chunk; start of the open segment
    const int64_t nsampled = ((int64_t)n + stride - 1) / stride;
    for (int64_t task = blockIdx.x; task < nsampled * split; task += gridDim.x) {
        const int32_t j = (int32_t)((task / split) * stride);
        const int32_t part = (int32_t)(task % split);
        const int64_t rs = rpF[j], re = rpF[j + 1];
        const int32_t len = static_cast<int32_t>(re - rs);
        const int64_t dj = diagF[j];
        // mode 2: the open segment is [seg0, used) of the current chunk
        int64_t row_done = 0;  // pairs of this row in closed segments
        auto close_seg = [&]() {
            if (cbase >= 0 && used > seg0) {
                unsigned long long g = 0;
                if (lane == 0) g = atomicAdd(pool.ctr + 1, 1ull);
                g = __shfl(g, 0);
                if (g < (unsigned long long)pool.seg_cap) {
                    if (lane == 0) pool.seg[g] = make_longlong4(j, row_done, cbase + seg0, used - seg0);
                } else if (lane == 0) {
                    atomicOr(pool.overflow, 1u);
                }
                row_done += used - seg0;
            }
            seg0 = used;
        };
        for (int32_t e = lane; e < len; e += kWave) colsj[e] = ciF[rs + e];
        if (counts)
            for (int64_t s = dj + lane; s < re; s += kWave) scount[s] = 0;
        wave_sync();
        const int32_t cmin = colsj[0];
        const int64_t range = (int64_t)colsj[len - 1] - cmin + 1;
        // off < range < 2^31 and mul <= 2^34: the product fits in 64 bits,
        // and the bucket of any off < range is below kSchedDir
        const uint64_t mul = ((uint64_t)kSchedDir << 24) / (uint64_t)range;
        for (int32_t b = lane; b <= kSchedDir; b += kWave) {
            // first position whose bucket is >= b
            int32_t lo = 0, hi = len;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                const int64_t bm = sched_bucket((int64_t)colsj[mid] - cmin, mul);
                if (bm < b) lo = mid + 1;
                else hi = mid;
            }
            dir[b] = (DirT)lo;
        }
        wave_sync();
        for (int64_t s0 = rs + (int64_t)part * kWave; s0 < dj; s0 += (int64_t)kWave * split) {
            const int32_t np = static_cast<int32_t>(min<int64_t>(kWave, dj - s0));
            if (lane < np) {
                const int32_t h = ciF[s0 + lane];
                const int32_t dh = diagF[h];
                pdh[lane] = dh;
                phe[lane] = static_cast<int32_t>(rpF[h + 1]);
                pout[lane] = mode == 1 ? sptr[s0 + lane] : 0;
                if (counts) lsd[s0 + lane] = dh;
            }
            wave_sync();
            for (int32_t p = 0; p < np; ++p) {
                const int64_t s = s0 + p;
                const int64_t dh = pdh[p], he = phe[p];
                const int64_t out = pout[p];
                const int32_t lo0 = static_cast<int32_t>(s - rs) + 1;
                int32_t found = 0;
                // kSchedUnroll chunks of the pivot row per round: their column
                // loads are issued together (clamped, in bounds; extras unused)
                for (int64_t q0 = dh + 1; q0 < he; q0 += kSchedUnroll * kWave) {
                    int32_t tv[kSchedUnroll];
#pragma unroll
                    for (int u = 0; u < kSchedUnroll; ++u)
                        tv[u] = ciF[min<int64_t>(q0 + u * kWave + lane, he - 1)];
#pragma unroll
                    for (int u = 0; u < kSchedUnroll; ++u) {
                        const int64_t q = q0 + u * kWave + lane;
                        int32_t pos = -1;
                        const int64_t off = (int64_t)tv[u] - cmin;
                        if (q < he && off >= 0 && off < range) {
                            const int32_t t = tv[u];
                            const int32_t b = sched_bucket(off, mul);
                            int32_t lo = max(lo0, (int32_t)dir[b]), hi = (int32_t)dir[b + 1] - 1;
                            while (lo <= hi) {
                                const int32_t mid = (lo + hi) >> 1;
                                const int32_t c = colsj[mid];
                                if (c == t) { pos = mid; break; }
                                if (c < t) lo = mid + 1;
                                else hi = mid - 1;
                            }
                        }
                        const uint64_t m = __ballot(pos >= 0);
                        if (mode == 1 && pos >= 0) {
                            const int32_t rank = __popcll(m & ((1ull << lane) - 1ull));
                            sq[out + found + rank] = static_cast<int32_t>(q);
                            sp[out + found + rank] = static_cast<int32_t>(rs + pos);
                        }
                        if (mode == 2 && m && cbase != -2) {
                            const int32_t c = __popcll(m);
                            if (cbase < 0 || used + c > pool.chunk) {
                                close_seg();
                                unsigned long long at = 0;
                                if (lane == 0) at = atomicAdd(pool.ctr, (unsigned long long)pool.chunk);
                                at = __shfl(at, 0);
                                if (at + (unsigned long long)pool.chunk > (unsigned long long)pool.cap) {
                                    if (lane == 0) atomicOr(pool.overflow, 1u);
                                    cbase = -2;
                                } else {
                                    cbase = (int64_t)at;
                                }
                                used = 0;
                                seg0 = 0;
                            }
                            if (cbase >= 0) {
                                if (pos >= 0) {
                                    const int32_t rank = __popcll(m & ((1ull << lane) - 1ull));
                                    pool.q[cbase + used + rank] = static_cast<int32_t>(q);
                                    pool.p[cbase + used + rank] = static_cast<int32_t>(rs + pos);
                                }
                                used += c;
                            }
                        }
                        found += __popcll(m);
                    }
                }
                if (counts && lane == 0) scount[s] = found;
                if (mode == 3 && lane == 0) {
                    if (found) atomicAdd(pool.sample, (unsigned long long)found);
                    if (he > dh + 1) atomicAdd(pool.sample + 2, (unsigned long long)(he - dh - 1));
                }
            }
            wave_sync();
        }
        if (mode == 2) close_seg();
        wave_sync();
    }
}

// mode 2's segments to their places: one wavefront per segment
__global__ __launch_bounds__(64) void k_sched_copy(SchedPool pool, int64_t nseg, const int64_t* __restrict__ rpF,
                                                   const int64_t* __restrict__ sptr, int32_t* __restrict__ sq,
                                                   int32_t* __restrict__ sp) {
    const int lane = lane_id();
    for (int64_t g = blockIdx.x; g < nseg; g += gridDim.x) {
        const longlong4 d = pool.seg[g];
        const int64_t dst = sptr[rpF[d.x]] + d.y;
        for (int64_t e = lane; e < d.w; e += kWave) {
            sq[dst + e] = pool.q[d.z + e];
            sp[dst + e] = pool.p[d.z + e];
        }
    }
}

hipError_t launch_sched_copy(const SchedPool& pool, int64_t nseg, const int64_t* rpF, const int64_t* sptr,
                             int32_t* sq, int32_t* sp, hipStream_t s) {
    if (nseg <= 0) return hipSuccess;
    const int grid = (int)std::min<int64_t>(nseg, 65536);
    hipLaunchKernelGGL(k_sched_copy, dim3(grid), dim3(64), 0, s, pool, nseg, rpF, sptr, sq, sp);
    return hipGetLastError();
}

hipError_t launch_sched(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF,
                        int mode, int32_t* scount, int32_t* lsd, const int64_t* sptr,
                        int32_t* sq, int32_t* sp, int32_t max_row, hipStream_t s, const SchedPool* pool,
                        int32_t stride) {
    const int32_t mr = max(max_row, 1);
    size_t lds = (size_t)mr * sizeof(int32_t);
    stride = max(stride, 1);
    const int32_t split = mode == 3 ? kSchedSampleSplit : 1;
    const int64_t tasks = ((int64_t)n + stride - 1) / stride * split;
    int grid = (int)std::min<int64_t>(tasks, 65536);
    if (grid <= 0) return hipSuccess;
    const SchedPool none{};
    if (mr < 65536)
        hipLaunchKernelGGL(k_sched<uint16_t>, dim3(grid), dim3(64), lds, s, n, rpF, ciF, diagF, mode, scount,
                           lsd, sptr, sq, sp, pool ? *pool : none, mr, stride, split);
    else
        hipLaunchKernelGGL(k_sched<int32_t>, dim3(grid), dim3(64), lds, s, n, rpF, ciF, diagF, mode, scount,
                           lsd, sptr, sq, sp, pool ? *pool : none, mr, stride, split);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Target-major copy of the update schedule: for every F slot p of row j, the
// updates it receives (row-local slot of the pivot entry f_jh, slot of f_ht)
// in ascending h.  One wavefront per row.  mode 0 counts per slot into
// tcount; mode 1 fills, walking the pivots in ascending order so that each
// slot's list comes out sorted (a pivot updates distinct slots).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_tsched(int32_t n, const int64_t* __restrict__ rpF,
                                               const int32_t* __restrict__ diagF,
                                               const int64_t* __restrict__ sptr,
                                               const int32_t* __restrict__ sq,
                                               const int32_t* __restrict__ sp, int mode,
                                               int32_t* __restrict__ tcount, const int64_t* __restrict__ tptr,
                                               int32_t* __restrict__ tsl, int32_t* __restrict__ tq) {
    extern __shared__ int64_t tsh[];
    const int lane = lane_id();
    for (int32_t j = blockIdx.x; j < n; j += gridDim.x) {
        const int64_t rs = rpF[j], re = rpF[j + 1], dj = diagF[j];
        const int32_t len = (int32_t)(re - rs), dl = (int32_t)(dj - rs);
        int64_t* Tp = tsh;                                  // [len] tptr of the row's slots
        int64_t* Sp = tsh + len;                            // [dl + 1] sptr of its L slots
        int32_t* cur = reinterpret_cast<int32_t*>(tsh + len + dl + 1);  // [len]
        for (int32_t e = lane; e < len; e += kWave) {
            cur[e] = 0;
            if (mode == 1) Tp[e] = tptr[rs + e];
        }
        for (int32_t e = lane; e <= dl; e += kWave) Sp[e] = sptr[rs + e];
        wave_sync();
        if (mode == 0) {
            for (int64_t e = Sp[0] + lane; e < Sp[dl]; e += kWave) atomicAdd(&cur[sp[e] - rs], 1);
            wave_sync();
            for (int32_t e = lane; e < len; e += kWave) tcount[rs + e] = cur[e];
        } else {
            for (int32_t h = 0; h < dl; ++h) {
                for (int64_t e = Sp[h] + lane; e < Sp[h + 1]; e += kWave) {
                    const int32_t p = (int32_t)(sp[e] - rs);
                    const int64_t pos = Tp[p] + cur[p];
                    cur[p] = cur[p] + 1;
                    tsl[pos] = h;
                    tq[pos] = sq[e];
                }
                wave_sync();
            }
        }
        wave_sync();
    }
}

size_t tsched_lds_bytes(int32_t max_row, int32_t max_lrow) {
    return (size_t)max_row * 8 + ((size_t)max_lrow + 1) * 8 + (size_t)max_row * 4;
}

hipError_t launch_tsched(int32_t n, const int64_t* rpF, const int32_t* diagF, const int64_t* sptr,
                         const int32_t* sq, const int32_t* sp, int mode, int32_t* tcount, const int64_t* tptr,
                         int32_t* tsl, int32_t* tq, int32_t max_row, int32_t max_lrow, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t lds = tsched_lds_bytes(std::max(max_row, 1), max_lrow);
    hipLaunchKernelGGL(k_tsched, dim3(std::min(n, 65536)), dim3(64), lds, s, n, rpF, diagF, sptr, sq, sp, mode,
                       tcount, tptr, tsl, tq);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// pattern statistics
// ------------------------------------------------------------------------------------
__global__ void k_stats(int32_t n, const int64_t* __restrict__ rpF,
                        const int32_t* __restrict__ diagF, PatStats* st) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t rs = rpF[i], re = rpF[i + 1], d = diagF[i];
    atomicMax(&st->max_row, static_cast<int32_t>(re - rs));
    atomicMax(&st->max_lrow, static_cast<int32_t>(d - rs));
    atomicMax(&st->max_upart, static_cast<int32_t>(re - d - 1));
    atomicAdd(&st->nnz_l, static_cast<unsigned long long>(d - rs));
}

hipError_t launch_stats(int32_t n, const int64_t* rpF, const int32_t* diagF, PatStats* st,
                        hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats, dim3((n + 255) / 256), dim3(256), 0, s, n, rpF, diagF, st);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// dependency levels: level_i = 1 + max level_h over the nodes h that node i
// depends on (-1 = not yet known).  Up to two independent graphs are walked in
// one launch (the forward and the backward DAG), alternate wavefronts taking
// nodes of either, so their two dependency chains overlap in time.
// ------------------------------------------------------------------------------------
// The dependencies of node i: mode 0 the strict lower part of row i of F,
// mode 1 the strict upper part, mode 2 entries [ptr[i], ptr[i+1]) of a
// column structure (idx = row indices).
__device__ __forceinline__ void dep_range(const DepGraph& G, int32_t i, int64_t& a, int64_t& b) {
    if (G.mode == 0) { a = G.ptr[i]; b = G.diag[i]; }
    else if (G.mode == 1) { a = G.diag[i] + 1; b = G.ptr[i + 1]; }
    else { a = G.ptr[i]; b = G.ptr[i + 1]; }
}

__device__ __forceinline__ int32_t ld_level(const int32_t* p) {
    const int32_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    jitter((uint32_t)v);
    return v;
}

// watchdog over polling rounds without progress; true = give up
__device__ __forceinline__ bool level_watchdog(uint32_t& polls, uint64_t& t0, Ctl* ctl, uint64_t limit) {
    ++polls;
    if ((polls & 31u) != 0u) return false;
    bool stop = (polls & 255u) == 0u && ld_u32_coherent(&ctl->abort) != 0u;
    const uint64_t now = wall_clock64();
    if (polls == 32u) {
        t0 = now;
    } else if (now - t0 > limit) {
        if (lane_id() == 0) {
            atomicOr(&ctl->status, kStTimeout);
            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        stop = true;
    }
    return __any(stop);
}

// One node, one wavefront.  The maximum does not depend on order, so every
// round re-polls all of a chunk's unknown dependencies at once.
constexpr int kLevelPer = 4;  // dependencies per lane and chunk

// S == Scope::Xcd: every wavefront of the job runs on one XCD and the levels
// are stored with workgroup scope (they stay in that XCD's L2, where the
// agent-scope polls of the job's other wavefronts find them)
template <Scope S>
__device__ __forceinline__ void level_row(const DepGraph& G, int32_t* depth, Ctl* ctl, uint64_t limit, int32_t i) {
    const int lane = lane_id();
    int64_t a, b;
    dep_range(G, i, a, b);
    int32_t best = 0;
    bool stop = false;
    for (int64_t base = a; base < b && !stop; base += kWave * kLevelPer) {
        int32_t src[kLevelPer], dv[kLevelPer];
        bool need[kLevelPer];
#pragma unroll
        for (int u = 0; u < kLevelPer; ++u) {
            const int64_t q = base + u * kWave + lane;
            need[u] = q < b;
            src[u] = need[u] ? G.idx[q] : 0;
            dv[u] = need[u] ? __hip_atomic_load(depth + src[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) : 0;
        }
        uint32_t polls = 0;
        uint64_t t0 = 0;
        for (;;) {
            bool pend = false;
#pragma unroll
            for (int u = 0; u < kLevelPer; ++u) {
                if (need[u]) {
                    if (dv[u] >= 0) {
                        best = max(best, dv[u]);
                        need[u] = false;
                    } else {
                        pend = true;
                    }
                }
            }
            if (!__any(pend)) break;
#pragma unroll
            for (int u = 0; u < kLevelPer; ++u)
                if (need[u]) dv[u] = ld_level(depth + src[u]);
            if (level_watchdog(polls, t0, ctl, limit)) {
                stop = true;
                break;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) best = max(best, __shfl_xor(best, off));
    if (lane == 0) {
        jitter((uint32_t)i);
        if constexpr (S == Scope::Xcd)
            __hip_atomic_store(depth + i, best + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_store(depth + i, best + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// S == Scope::Xcd: each job elects its own XCD through its control block (the
// first of its workgroups to start names it); the job's workgroups elsewhere
// leave at once
template <Scope S>
__global__ __launch_bounds__(64) void k_depth(int32_t n, LevelJob j0, LevelJob j1, int32_t njobs, Ctl* ctl,
                                              uint64_t spin_limit) {
    const LevelJob J = (njobs > 1 && (blockIdx.x & 1)) ? j1 : j0;
    if constexpr (S == Scope::Xcd) {
        if (!xcd_member(J.tctl)) return;
    }
    for (;;) {
        const uint32_t t = wave_ticket(J.tctl);
        if (t >= (uint32_t)n) break;
        const int32_t i = J.desc ? n - 1 - (int32_t)t : (int32_t)t;
        level_row<S>(J.G, J.depth, ctl, spin_limit, i);
    }
}

// Lane per node: a ticket hands a wavefront 64 consecutive nodes (in the
// sweep's order), so the whole graph can be in flight at once and wide
// graphs are not throttled by the ticket.  A lane scans its node's
// dependencies, at most 8 per round, and stops at the first one not known
// yet; the wavefront keeps looping until every lane published, so lanes that
// depend on other lanes of the same wavefront cannot deadlock.
__global__ __launch_bounds__(64) void k_depth_lanes(int32_t n, LevelJob j0, LevelJob j1, int32_t njobs, Ctl* ctl,
                                                    uint64_t spin_limit) {
    const int lane = lane_id();
    const LevelJob J = (njobs > 1 && (blockIdx.x & 1)) ? j1 : j0;
    const int32_t* __restrict__ ciF = J.G.idx;
    for (;;) {
        const uint32_t t = wave_ticket(J.tctl);
        const int64_t r = (int64_t)t * kWave + lane;
        if ((int64_t)t * kWave >= n) break;
        const bool valid = r < n;
        const int32_t i = valid ? (J.desc ? n - 1 - (int32_t)r : (int32_t)r) : 0;
        int64_t q = 0, b = 0;
        if (valid) dep_range(J.G, i, q, b);
        int32_t best = 0;
        bool done = !valid;
        uint32_t polls = 0;
        uint64_t t0 = 0;
        for (;;) {
            bool prog = false;
            if (!done) {
                for (int step = 0; step < 8 && q < b; ++step) {
                    const int32_t* src = J.depth + ciF[q];
                    int32_t d = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
                    if (d < 0) d = ld_level(src);
                    if (d < 0) break;
                    best = max(best, d);
                    ++q;
                    prog = true;
                }
                if (q >= b) {
                    jitter((uint32_t)i);
                    __hip_atomic_store(J.depth + i, best + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    done = true;
                }
            }
            if (__all(done)) break;
            if (__any(prog)) {
                polls = 0;
                continue;
            }
            if (level_watchdog(polls, t0, ctl, spin_limit)) break;
        }
    }
}

// Rows sorted by level (counting sort): hist, scan (shared scan kernel),
// scatter.  The order inside a level is whatever the atomics give; any
// order that lists every level before the next is a valid schedule, and the
// results never depend on it.
__global__ void k_level_hist(int32_t n, const int32_t* __restrict__ depth, int32_t* hist) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&hist[depth[i] - 1], 1);
}

__global__ void k_level_scatter(int32_t n, const int32_t* __restrict__ depth,
                                const int64_t* __restrict__ off, int32_t* cursor, int32_t* perm) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t d = depth[i] - 1;
    perm[off[d] + atomicAdd(&cursor[d], 1)] = i;
}

hipError_t launch_level_order(int32_t n, const int32_t* depth, int32_t max_depth, int32_t* hist,
                              int64_t* off, int64_t* scan_tmp, int32_t* perm, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipError_t e = launch_fill_i32(hist, 2 * (int64_t)max_depth, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_level_hist, dim3((n + 255) / 256), dim3(256), 0, s, n, depth, hist);
    e = launch_scan(hist, max_depth, off, scan_tmp, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_level_scatter, dim3((n + 255) / 256), dim3(256), 0, s, n, depth, off,
                       hist + max_depth, perm);
    return hipGetLastError();
}

hipError_t launch_depth(int32_t n, const LevelJob& j0, const LevelJob* j1, Ctl* ctl, uint64_t spin_limit,
                        int32_t grid, bool one_xcd, hipStream_t s) {
    if (n <= 0 || grid == 0) return hipSuccess;
    const int32_t njobs = j1 ? 2 : 1;
    const LevelJob b = j1 ? *j1 : j0;
    if (grid < 0)
        hipLaunchKernelGGL(k_depth_lanes, dim3(-grid * njobs), dim3(64), 0, s, n, j0, b, njobs, ctl, spin_limit);
    else if (one_xcd)
        hipLaunchKernelGGL(k_depth<Scope::Xcd>, dim3(grid * njobs * kXcds), dim3(64), 0, s, n, j0, b, njobs, ctl,
                           spin_limit);
    else
        hipLaunchKernelGGL(k_depth<Scope::Device>, dim3(grid * njobs), dim3(64), 0, s, n, j0, b, njobs, ctl,
                           spin_limit);
    return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_max_i32(const int32_t* __restrict__ p, int64_t n, int32_t* out) {
    int32_t m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, p[i]);
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
    if (lane_id() == 0) atomicMax(out, m);
}

hipError_t launch_max_i32(const int32_t* p, int64_t n, int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_max_i32, dim3(blocks), dim3(256), 0, s, p, n, out);
    return hipGetLastError();
}

}  // namespace tpilu
