// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev_common.h"

namespace tpilu {

// ---- symbolic phase --------------------------------------------------------
// status bits written by k_validate
constexpr uint32_t kValBadRowptr = 1u, kValBadCol = 2u, kValUnsorted = 4u, kValNoDiag = 8u;

hipError_t launch_validate(int32_t n, int64_t nnz, const int64_t* rp, const int32_t* ci,
                           uint32_t* status, hipStream_t s);

// LDS capacities of the symbolic paths: tier 0 for rows of up to about a
// thousand entries, tier 1 (80 KB of LDS per wavefront) up to about four
// thousand; longer rows use maps in global memory (tier 2)
constexpr int kSymEndCap = 1024;      // endpoint map (row of F being built), tier 0
constexpr int kSymEndCapLong = 4096;  // the same, tier 1
constexpr int kSymFrontCap = 512;     // frontier maps and lists

// Count (mode 0) or fill (mode 1) the level-<=k pattern of rows [0, n) (or of
// the rows in row_list when non-null) with the maps of `tier`; a row that
// does not fit gets cnt = -1 (mode 0).  In mode 1 a row is only built by the
// tier that tier_of (nullable: tier 0 for all) records for it.
hipError_t launch_sym_rows(int tier, int32_t n, const int64_t* rpA, const int32_t* ciA,
                           int32_t k, const int32_t* row_list, int32_t n_rows, int mode,
                           int32_t* cnt, const int64_t* rpF, int32_t* ciF, uint8_t* lvF,
                           int32_t* diagF, const uint8_t* tier_of, int32_t* gscratch, uint32_t gcap,
                           int32_t grid, hipStream_t s);
__host__ __device__ size_t sym_global_scratch_ints(int32_t n, uint32_t gcap);  // per block

// rows (of `list`, or 0..n_rows-1) with cnt < 0 -> row_list, *n_over; tier_of[row] = tier
// rows whose one-step bound passes `limit` into list1 (and tier_of 1),
// the others into list0; counts[0], counts[1] are their running sizes (pre-set)
hipError_t launch_route_rows(int32_t n, const int64_t* rpA, const int32_t* ciA, int32_t* nup, int64_t limit,
                             int32_t* list0, int32_t* list1, int32_t* counts, uint8_t* tier_of, hipStream_t s);
int64_t sym_route_limit();
hipError_t launch_collect_overflow(int32_t n_rows, const int32_t* list, const int32_t* cnt, int32_t* row_list,
                                   int32_t* n_over, uint8_t* tier_of, int tier, hipStream_t s);

// exclusive scan of int32 counts into int64 offsets out[0..n], out[n] = total
hipError_t launch_scan(const int32_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
size_t scan_tmp_elems(int64_t n);

hipError_t launch_a2f(int32_t n, const int64_t* rpA, const int32_t* ciA, const int64_t* rpF,
                      const int32_t* ciF, int32_t* a2f, uint32_t* status, hipStream_t s);

// update schedule: mode 0 counts matches per L slot (and writes lsd = diag
// slot of the pivot), mode 1 writes the (q, p) pairs
// the pool of the one-pass schedule (k_sched mode 2) and the sample counter
// of mode 3; seg entries are (row, index of the first pair within the row,
// pool position, count); ctr[0] = pairs taken (whole chunks), ctr[1] =
// segments taken
struct SchedPool {
    int32_t* q = nullptr;
    int32_t* p = nullptr;
    int64_t cap = 0;
    int32_t chunk = 0;  // pairs a wavefront takes at a time
    longlong4* seg = nullptr;
    int64_t seg_cap = 0;
    unsigned long long* ctr = nullptr;
    uint32_t* overflow = nullptr;
    unsigned long long* sample = nullptr;
};
hipError_t launch_sched(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF,
                        int mode, int32_t* scount, int32_t* lsd, const int64_t* sptr,
                        int32_t* sq, int32_t* sp, int32_t max_row, hipStream_t s,
                        const SchedPool* pool = nullptr, int32_t stride = 1);
constexpr int32_t kSchedSampleStride = 241;  // rows sampled (j % 241 == 0) to size the pool
constexpr int32_t kSchedSampleSplit = 16;   // wavefronts sharing one sampled row
constexpr int64_t kSchedOnePassRatio = 8;   // candidates per pair above which the one-pass schedule runs
hipError_t launch_sched_copy(const SchedPool& pool, int64_t nseg, const int64_t* rpF, const int64_t* sptr,
                             int32_t* sq, int32_t* sp, hipStream_t s);

struct PatStats {
    unsigned long long nnz_l;
    int32_t max_row;
    int32_t max_lrow;
    int32_t max_upart;
    int32_t pad;
};
hipError_t launch_stats(int32_t n, const int64_t* rpF, const int32_t* diagF, PatStats* st,
                        hipStream_t s);

// Dependency graph whose levels are computed: node i depends on idx[a..b)
// with (a, b) from the mode (0 strict lower part of row i, 1 strict upper
// part, 2 a column structure [ptr[i], ptr[i+1])).
struct DepGraph {
    const int64_t* ptr;
    const int32_t* idx;
    const int32_t* diag;
    int mode;
};
// One level computation: the graph, its sweep order (ascending, or descending
// when desc), the level array (pre-filled with -1) and the control block
// whose ticket hands out its nodes.
struct LevelJob {
    DepGraph G;
    int desc;
    int32_t* depth;
    Ctl* tctl;
};
// level of every node (1 + max level of its dependencies) for one job, or two
// independent jobs in one launch (alternate wavefronts; j1 may be null).
// grid > 0: wavefront per node, grid < 0: lane per node; |grid| wavefronts
// per job (one_xcd, wavefront per node: grid wavefronts per XCD launched,
// those of one XCD per job working).  Abort and watchdog state live in ctl.
hipError_t launch_depth(int32_t n, const LevelJob& j0, const LevelJob* j1, Ctl* ctl, uint64_t spin_limit,
                        int32_t grid, bool one_xcd, hipStream_t s);
// perm = nodes sorted by level (counting sort); levels are 1 .. max_depth
// (depth[i] >= 1); hist needs 2 * max_depth ints
hipError_t launch_level_order(int32_t n, const int32_t* depth, int32_t max_depth, int32_t* hist,
                              int64_t* off, int64_t* scan_tmp, int32_t* perm, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_max_i32(const int32_t* p, int64_t n, int32_t* out, hipStream_t s);

// ---- numeric phase -------------------------------------------------------------
struct PatDev {
    int32_t n;
    int32_t nnz_a;
    int32_t nnz_f;
    const int64_t* rpA;
    const int32_t* ciA;
    const int64_t* rpF;
    const int32_t* ciF;
    const int32_t* diagF;
    const int32_t* a2f;
    const int32_t* lsd;   // per F slot (L part): diag slot of the pivot
    const int64_t* sptr;  // per F slot: start of its update pairs; [nnz_f + 1]
    const int32_t* sq;    // pair: slot of f_ht in row h
    const int32_t* sp;    // pair: slot of f_jt in row j
    unsigned long long* trace;  // nullable: per-row start/finish ticks
    const int32_t* permL;       // nullable: rows in order of forward dependency level
    const int32_t* permU;       // nullable: rows in order of backward dependency level
    int32_t groupL, groupU;     // positions of permL / permU per ticket (>= 1)
    int32_t parts;              // position counters the row kernels draw from (1..kTicketParts, <= grid)
    const int64_t* tptr;  // per F slot: start of the updates it receives; [nnz_f + 1]
    const int32_t* tsl;   // update: row-local slot of the pivot entry f_jh (ascending h per target)
    const int32_t* tq;    // update: slot of f_ht in row h
};

// fill `n` doubles with kPending; thread 0 also resets ctl->ticket (and, if
// reset_status, the sticky status words)
hipError_t launch_fill_pending(double* p, int64_t n, Ctl* ctl, bool reset_status, hipStream_t s);
// the same for the U~ slots of a factor (rows diag..end, batch values per
// slot); the L~ slots are left as they are (the elimination writes them)
hipError_t launch_fill_pending_upper(double* f_val, int32_t n, const int64_t* rpF, const int32_t* diagF,
                                     int32_t batch, Ctl* ctl, bool reset_status, hipStream_t s);

constexpr int32_t kXcds = 8;  // XCDs of an MI355X

// flow: the single-instance dataflow kernel (needs the target-major schedule
// and numeric_flow_fits); otherwise the pivot-serial one.  one_xcd (single
// instance): grid wavefronts per XCD launched, those of one XCD working.
// wrow (batches only): non-null puts every wavefront's working row in global
// memory, grid x max_row x 64 doubles, instead of LDS.  xout (batches only):
// non-null fuses the forward substitution x = L~^-1 bvec in (xout pre-filled
// with kPending).  fused: every update of Eq. 6b as one fused multiply-add.
hipError_t launch_numeric(const PatDev& P, const double* a_val, int32_t batch, double* f_val,
                          Ctl* ctl, uint64_t spin_limit, int64_t skip_row, int32_t grid,
                          int32_t max_row, int32_t max_lrow, bool flow, bool one_xcd, double* wrow,
                          const double* bvec, double* xout, bool fused, hipStream_t s);
int numeric_grid(int32_t batch, int32_t max_row, int32_t max_lrow, bool flow, int num_cu, bool global_row = false);
// the dataflow kernel in critical-path mode: f_len (pre-filled with
// kPending) receives, per entry, the length of the longest dependency chain
// ending in it, a row-to-row hand-off weighing w_hop and an l of a row
// (strict lower slots: when that l is ready) w_step
hipError_t launch_numeric_hops(const PatDev& P, double* f_len, Ctl* ctl, uint64_t spin_limit, int32_t grid,
                               int32_t max_row, int32_t max_lrow, double w_hop, double w_step, hipStream_t s);
hipError_t launch_max_nonneg(const double* v, int64_t n, unsigned long long* out, hipStream_t s);
bool numeric_flow_fits(int32_t max_row, int32_t max_lrow, size_t lds_limit);
// target-major update schedule (mode 0 count per slot, mode 1 fill); LDS of
// tsched_lds_bytes per wavefront
hipError_t launch_tsched(int32_t n, const int64_t* rpF, const int32_t* diagF, const int64_t* sptr,
                         const int32_t* sq, const int32_t* sp, int mode, int32_t* tcount, const int64_t* tptr,
                         int32_t* tsl, int32_t* tq, int32_t max_row, int32_t max_lrow, hipStream_t s);
size_t tsched_lds_bytes(int32_t max_row, int32_t max_lrow);

// ---- triangular solves -------------------------------------------------------------
// single instance: grid > 0 wavefront per row (one_xcd: grid wavefronts on
// one XCD), < 0 lane per row with -grid wavefronts (the one-CU shape is
// launch_solve_cu); batches: lanes = instances with grid wavefronts
hipError_t launch_forward(const PatDev& P, const double* f_val, int32_t batch, const double* b,
                          double* x, Ctl* ctl, uint64_t spin_limit, int32_t grid, bool one_xcd,
                          hipStream_t s);
hipError_t launch_backward(const PatDev& P, const double* f_val, int32_t batch, const double* x,
                           double* y, Ctl* ctl, uint64_t spin_limit, int32_t grid, bool one_xcd,
                           hipStream_t s);

// ---- the solves on one CU (lane per row, hand-off through an LDS ring) ----------
// Pq[slot] = level-order position of the row named by the slot's column
// (forward order for strict lower slots, backward order for upper ones)
hipError_t launch_dep_positions(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF,
                                const int32_t* permL, const int32_t* permU, int32_t* iposL, int32_t* iposU,
                                int32_t* Pq, hipStream_t s);
// forward (x = L~^-1 b: in = b, out = x) or backward (y = U~^-1 x: in = x,
// out = y), single instance, one workgroup; out needs no pending fill
hipError_t launch_solve_cu(const PatDev& P, const int32_t* Pq, const double* f_val, const double* in, double* out,
                           bool backward, Ctl* ctl, uint64_t spin_limit, hipStream_t s);

// ---- Krylov building blocks ---------------------------------------------------
constexpr int kDotLanes = 16384;  // fixed shape of every inner product
constexpr int kDotBlocks = 64;
constexpr int kDotThreads = 256;

hipError_t launch_spmv(int32_t n, const int64_t* rp, const int32_t* ci, const double* v,
                       const double* x, const double* b_minus, double* y, hipStream_t s);
hipError_t launch_dot_partial(int64_t n, const double* x, const double* y, double* partial,
                              hipStream_t s);
hipError_t launch_dot_final(const double* partial, double* out, int sqrt_it, hipStream_t s);

struct GmresDev;  // defined in the Krylov unit
hipError_t launch_gm_axpy_h(int64_t n, const double* partial, double* hslot, double* w,
                            const double* v, hipStream_t s);
hipError_t launch_gm_norm_scale(int64_t n, const double* partial, double* hslot, const double* w,
                                double* vnext, hipStream_t s);
hipError_t launch_gm_start(int64_t n, const double* partial, double* beta_slot, double* g0,
                           const double* r, double* v0, hipStream_t s);
hipError_t launch_gm_givens(double* H, double* cs, double* sn, double* g, int32_t m, int32_t j,
                            double tol, int32_t* iters, int32_t maxit, double* hist,
                            int32_t* stop, hipStream_t s);
// rho, c, s of the rotation of every pair (a_i, b_i), with the same device
// code as the GMRES step
hipError_t launch_givens_batch(int64_t n, const double* a, const double* b, double* rho, double* c, double* s,
                               hipStream_t st);
hipError_t launch_gm_backsub(const double* H, const double* g, double* yv, int32_t m, int32_t jj,
                             hipStream_t s);
hipError_t launch_gm_combine(int64_t n, const double* V, const double* yv, int32_t jj, double* u,
                             hipStream_t s);
hipError_t launch_axpy1(int64_t n, double* x, const double* z, hipStream_t s);
hipError_t launch_sub(int64_t n, const double* b, const double* ax, double* r, hipStream_t s);

// ---- adjoint -------------------------------------------------------------------
struct AdjPat {
    const int64_t* tpL;   // CSC of the strict lower part: column c -> entries
    const int32_t* tsL;   //   F slots of column c's entries, rows ascending
    const int32_t* trL;   //   and their rows
    const int64_t* tpU;   // CSC of the strict upper part
    const int32_t* tsU;
    const int32_t* trU;
    const int32_t* permUT;  // rows by level of the U~^T solve (row i waits on column i of U~)
    const int32_t* permLT;  // rows by level of the L~^T solve and of the reverse sweep
                            // (row i waits on the rows of column i of L~)
};
hipError_t launch_transpose_count(int32_t n, const int64_t* rpF, const int32_t* ciF,
                                  const int32_t* diagF, int32_t* cntL, int32_t* cntU,
                                  hipStream_t s);
hipError_t launch_transpose_fill(int32_t n, const int64_t* rpF, const int32_t* ciF,
                                 const int32_t* diagF, const int64_t* tpL, int32_t* tsL,
                                 int32_t* trL, const int64_t* tpU, int32_t* tsU, int32_t* trU,
                                 int32_t* curL, int32_t* curU, hipStream_t s);
hipError_t launch_sort_columns(int32_t n, const int64_t* tp, int32_t* ts, int32_t* tr,
                               hipStream_t s);

// one_xcd (single instance): grid wavefronts per XCD launched, those of one
// XCD working
hipError_t launch_adj_solve_u(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* ybar, double* z, Ctl* ctl,
                              uint64_t spin_limit, int32_t grid, bool one_xcd, hipStream_t s);
hipError_t launch_adj_solve_l(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* z, double* w, Ctl* ctl,
                              uint64_t spin_limit, int32_t grid, bool one_xcd, hipStream_t s);
hipError_t launch_adj_fbar(const PatDev& P, int32_t batch, const double* x, const double* y,
                           const double* z, const double* w, double* fbar, hipStream_t s);
hipError_t launch_adj_numeric(const PatDev& P, const AdjPat& T, const double* f_val,
                              int32_t batch, const double* fbar_in, double* G, double* lbar,
                              double* abar, Ctl* ctl, uint64_t spin_limit, int32_t grid,
                              int32_t max_row, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);

// ---- BiCGSTAB steps ----------------------------------------------------------------------
// device scalar slots
enum { kBiRho = 0, kBiRhoOld = 1, kBiAlpha = 2, kBiOmega = 3, kBiRv = 4, kBiTt = 5, kBiSlots = 8 };
enum { kBiOpRho = 0, kBiOpP = 1, kBiOpAlpha = 2, kBiOpS = 3, kBiOpXHalf = 4, kBiOpOmega = 5, kBiOpXR = 6 };
// one step of the iteration (see k_krylov.hip for the operands of each op)
hipError_t launch_bi(int op, int64_t n, int first, const double* pa, const double* pb, double* sc, double* x,
                     double* r, const double* a1, const double* a2, const double* a3, const double* a4,
                     hipStream_t s);

// ---- level-based incomplete inverses ---------------------------------------------------
// per kept entry p of F's pattern: its updates [ptr[p], ptr[p+1]), each the
// row-local slot of the multiplier (s) and the slot of the partner entry in
// the other row (q); ascending pivot order for the strict lower part,
// descending for the upper part
struct InvSched {
    const int64_t* ptr;
    const int32_t* s;
    const int32_t* q;
};
// upper 0: lists of the strict lower entries, 1: of the upper entries; pass 0
// counts into tcount, pass 1 fills (tptr = scan of the counts)
hipError_t launch_isched(int32_t n, const int64_t* rpF, const int32_t* ciF, const int32_t* diagF, int upper,
                         int pass, int32_t* tcount, const int64_t* tptr, int32_t* ps, int32_t* pq,
                         int32_t max_row, hipStream_t s);
size_t isched_lds_bytes(int32_t max_row);
// one half of G from F (G pre-filled with kPending; ctl ticket reset)
hipError_t launch_inverse(const PatDev& P, const InvSched& S, const double* f_val, double* g_val, bool upper,
                          Ctl* ctl, uint64_t spin_limit, int32_t grid, hipStream_t s);
// x = L~~^-1 b, y = U~~^-1 x; thread_rows: one thread per row, else a wavefront
// shapes of the two products of the incomplete inverses
// (kProdTile stages 32 entries per row and round, kProdTileShort 8)
enum { kProdWaveRows = 0, kProdThreadRows = 1, kProdTile = 2, kProdTileShort = 3 };
hipError_t launch_apply_inverse(const PatDev& P, const double* g_val, const double* b, double* x, double* y,
                                int shape, hipStream_t s);

// ---- hand-off probe -------------------------------------------------------------------
size_t probe_buf_bytes();
// two wavefronts (on one XCD, or on two different XCDs) pass a counter back
// and forth `rounds` times through global memory; buf (probe_buf_bytes(),
// zeroed) receives the wall-clock ticks and a status word
hipError_t launch_handoff(void* buf, int32_t rounds, bool same_xcd, uint64_t spin_limit, hipStream_t s);
void probe_read(const void* host_copy, unsigned long long* ticks, uint32_t* status);

}  // namespace tpilu
