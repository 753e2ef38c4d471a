// Host runtime of the gfx950 ILU(k) library: contexts, pattern handles, the
// orchestration of the kernels behind every C entry point, the GMRES driver
// and batched graph capture.  Everything here is host code; every step of
// the numeric path runs in the kernels of the k_*.hip units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpilu.h"
#include "kernels.h"

using namespace tpilu;

struct tpilu_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    tpilu_alloc_fn alloc = nullptr;
    tpilu_free_fn free_fn = nullptr;
    void* user = nullptr;
    int num_cu = 256;
    uint64_t spin_limit = 1000000000ull;  // wait budget in wall-clock ticks (set from the clock rate)
    uint64_t ticks_per_us = 100;
    int64_t skip_row = -1;
    int32_t grid_override = 0;
    int solver = 0;  // 0 auto, 1 wavefront per row, 2 one workgroup, 3 lane per row
    int numeric = 0;  // 0 auto, 1 dataflow, 2 pivot-serial
    bool fused = false;  // numeric updates as one fused multiply-add
    int placement = 0;  // row kernels: 0 auto, 1 whole device, 2 one XCD
    int32_t group = 0;  // level-order positions per ticket of the row kernels; 0 auto
    int32_t tickets = 0;  // position counters of the row kernels; 0 auto
    bool timing = false;
    unsigned long long* trace = nullptr;  // per-row timeline buffer (device, 2n), or null
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
    // second stream (default priority) for work that overlaps the main one
    hipStream_t aux = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    double* scratch = nullptr;  // device address of the no-alloc scratch on this device
    hipError_t scratch_err = hipSuccess;
    std::string err;
    ~tpilu_ctx_s() {
        if (aux) (void)hipStreamDestroy(aux);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        for (auto& v : ev)
            for (auto& p : v) {
                (void)hipEventDestroy(p.first);
                (void)hipEventDestroy(p.second);
            }
    }
};

// ---------------------------------------------------------------------------
// Fixed scratch for tpilu_apply_noalloc: the intermediate vector x of the two
// substitutions lives in this file-scope device array, one copy per device,
// held until the process ends.  Host code never uses the array's name as an
// address (in host code it names a host-side stand-in): the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current and kept in scratch_addr.
constexpr int64_t kScratchDoubles = int64_t(1) << 22;  // 32 MiB: n * batch <= 4,194,304
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_addr[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// the first time and cached; nullptr (and the error in *err) if it failed.
double* scratch_on(int device, hipError_t* err) {
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    if (!scratch_addr[device] && scratch_err[device] == hipSuccess) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
            (void)hipGetLastError();
        } else {
            scratch_addr[device] = static_cast<double*>(p);
        }
    }
    *err = scratch_err[device];
    return scratch_addr[device];
}

namespace {

constexpr uint64_t kDefaultWaitUs = 10000000ull;  // 10 s per dependency wait

// Wavefronts of the wavefront-per-row solves.  Every waiting wavefront polls
// the memory side, so past the parallelism a dependency graph can use, more
// wavefronts only slow each hand-off down; long rows, on the other hand,
// keep a wavefront busy and want more rows in flight.  Measured on MI355X
// (forward solve, best grid): random banded n=160,000 ILU(2), 13 rows per
// level, 12 ms at 128-192 and 33 ms at 8192; the same ILU(1), 46 rows per
// level and 18 entries per row half: 3.1 ms at 256, 3.5 at 1024; paper-scale
// random ILU(1), 40 rows per level and 640 entries per half: 5.2 ms at 1024,
// 22 at 192; 27-point 50^3 ILU(3): 1.9 ms at 1024, 3.2 at 256.
constexpr int32_t kSolveWavesNarrow = 192;   // fewer than kNarrowWidth rows per level
constexpr int32_t kSolveWavesMid = 256;      // fewer than 64 rows per level, short rows
constexpr int32_t kSolveWavesWide = 1024;
// The numeric kernels run every resident wavefront: with their loads batched
// a row is short, and the rows in flight set the rate (1024 wavefronts ->
// resident maximum, pivot-serial: 27-point 90^3 ILU(1) 15.7 -> 8.4 ms,
// 7-point 64^3 ILU(1) 1.9 -> 1.2 ms, paper-scale random ILU(1) 69.7 ->
// 58.5 ms; dataflow: random banded ILU(1) 1.37 -> 0.83 ms, ILU(2) unchanged).
// Dataflow numeric kernel (automatic choice) when the L rows average at least
// kFlowMinL entries, an entry receives fewer than kFlowMaxChain updates on
// average and a dependency level holds fewer than kFlowMaxWidth rows.  On
// narrow graphs the dataflow kernel's short hand-off wins (random banded
// n=160,000: ILU(1) 0.72 vs 5.2 ms, ILU(2) 6.0 vs 22.9 ms); on wide ones the
// pivot-serial kernel's cheaper rows do (27-point 30^3 ILU(1), 71 rows per
// level: 1.28 vs 1.47 ms; 7-point 64^3 ILU(2): 2.19 vs 2.72 ms).
constexpr int64_t kFlowMinL = 4;
constexpr int64_t kFlowMaxChain = 12;
constexpr int64_t kFlowMaxWidth = 64;
constexpr int32_t kAdjointWaves = 512;
constexpr int32_t kAdjointBatchWaves = 1024;  // batched reverse elimination (3-D 7-point 32^3 x16: 1.9 ms, 2.2 at 512)
constexpr int32_t kInverseWaves = 1024;  // incomplete inverses (n=160,000 ILU(2): 7.0 ms, 8.3 at 512)
constexpr int64_t kNarrowWidth = 32;   // n / depth below this: narrow
// Wavefront-per-row solves run on one XCD, where the hand-offs stay in that
// XCD's L2, when the device-wide shape would take at most 256 wavefronts (a
// dependency level of fewer than 32 rows, or fewer than 64 of short rows)
// and a row half holds at most this many entries on average.  Measured on
// MI355X (forward / backward ms, device vs one XCD): random banded n=160,000
// ILU(2) (13 rows per level, 82 entries per half) 11.8 / 12.6 vs 8.4 / 9.3;
// 2-D 64 x 64 ILU(1) 0.18 / 0.19 vs 0.14 / 0.16; Table 3 scale ILU(1) (40
// rows per level, 640 entries per half) 5.2 / 6.0 vs 12.0 / 12.2.
constexpr int64_t kXcdMaxAvg = 128;
constexpr int64_t kLevelLaneMax = 14;  // level computation: lane per node below this many dependencies
constexpr int64_t kLevelWideMax = 60;  // wavefront per node: the wide window below this, else the narrow one
constexpr int32_t kLevelWavesWide = 768;
constexpr int32_t kLevelWavesNarrow = 192;

// TPILU_TRACE=1 in the environment prints every host-side step to stderr.
bool trace_on() {
    static const bool on = [] {
        const char* v = std::getenv("TPILU_TRACE");
        return v && *v && *v != '0';
    }();
    return on;
}
void trace(const char* what, int64_t a = -1, int64_t b = -1) {
    if (!trace_on()) return;
    std::fprintf(stderr, "[tpilu] %s %lld %lld\n", what, (long long)a, (long long)b);
    std::fflush(stderr);
}

struct Alloc {
    tpilu_alloc_fn alloc = nullptr;
    tpilu_free_fn free_fn = nullptr;
    void* user = nullptr;
    void* get(size_t bytes) const {
        if (bytes == 0) bytes = 8;
        if (alloc) return alloc(bytes, user);
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p) const {
        if (!p) return;
        if (free_fn) free_fn(p, user);
        else (void)hipFree(p);
    }
};

// device buffer owned by a handle
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        (void)hipGetLastError();  // a failure of an earlier call must not be reported by this one
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

// Level-order positions a wavefront takes per ticket in the wavefront-per-row
// kernels.  Every ticket is one atomic on one address (about 11 ns each,
// serialised), which on wide levels caps how fast rows can be handed out;
// grouping divides that traffic but runs a group's rows back to back.  The
// numeric kernels overlap a row's work with its wait on earlier levels, so
// there a group costs a whole row time per level (random banded n=160,000
// ILU(2): 8.5 -> 147 ms at 2 rows): always 1.  Solves and inverses gain on wide levels (7-point 64^3,
// ILU(1), 692 rows per level: wavefront-per-row forward 5.5 -> 3.3 ms at 3
// rows, inverse 6.6 -> 4.0 ms at 2 rows) and lose on narrow ones.
enum class RowKernel { Numeric, Solve, Inverse };

int32_t row_group(RowKernel kind, int64_t n, int64_t depth) {
    if (depth <= 0 || kind == RowKernel::Numeric) return 1;
    const int64_t width = std::max<int64_t>(n, 1) / depth;
    if (kind == RowKernel::Solve) return width >= 512 ? 3 : width >= 128 ? 2 : 1;
    return width >= 512 ? 2 : 1;
}

// Wavefronts of the batched kernels (a task is one row for 64 instances).
// Their waits re-read all pending values of a chunk in one round trip and
// their tasks come from the eight counters, and then extra wavefronts cost
// little: measured on MI355X, the batched solves are flat from 256-384
// wavefronts on (2-D 5-point 128^2 ILU(2) x256, x512 ILU(1); 3-D 7-point
// 32^3 ILU(1) x16, 64^3 x64) and the transposed ones best at 1024 (32^3
// x16: 0.59 ms, 0.70 at 512); the numeric kernel improves up to the
// resident maximum.
constexpr int32_t kBatchSolveWaves = 1024;
constexpr int32_t kBatchSolveWavesXcd = 256;  // on one XCD (32 CUs)


struct tpilu_pattern_s {
    Alloc al;
    int device = 0;
    int64_t n = 0, nnz_a = 0, nnz_f = 0, n_updates = 0;
    int32_t k = 0;
    PatStats st{};
    int32_t depth_l = 0, depth_u = 0, overflow_rows = 0, long_rows = 0;
    std::vector<DBuf> owned;
    // device arrays
    int64_t* rpA = nullptr;
    int32_t* ciA = nullptr;
    int64_t* rpF = nullptr;
    int32_t* ciF = nullptr;
    uint8_t* lvF = nullptr;
    int32_t* diagF = nullptr;
    int32_t* a2f = nullptr;
    int32_t* lsd = nullptr;
    int64_t* sptr = nullptr;
    int32_t* sq = nullptr;
    int32_t* sp = nullptr;
    int32_t* depthL = nullptr;  // dependency level of every row, forward sweep
    int32_t* depthU = nullptr;  // and backward sweep
    int32_t* permL = nullptr;   // rows sorted by depthL: the ticket order of numeric and forward
    int32_t* permU = nullptr;   // rows sorted by depthU: the ticket order of backward
    Ctl* ctl = nullptr;
    // adjoint transposes (built on first use)
    bool have_t = false;
    int64_t *tpL = nullptr, *tpU = nullptr;
    int32_t *tsL = nullptr, *trL = nullptr, *tsU = nullptr, *trU = nullptr;
    int32_t *permUT = nullptr, *permLT = nullptr;
    // update lists of the incomplete inverses (built on first use)
    bool have_inv = false;
    int64_t* iptr = nullptr;
    int32_t *is_s = nullptr, *is_q = nullptr;
    int64_t n_inv_updates = 0;
    // per F slot, the level-order position of the row its column names (the
    // one-CU solves); built with the pattern when those are the automatic
    // choice, else on first use
    int32_t* dep_pos = nullptr;
    bool solve_cu = false;  // the automatic solve shape is the one-CU one
    // target-major update schedule (only when the dataflow numeric kernel fits)
    bool flow = false;
    int64_t* tptr = nullptr;
    int32_t *tsl = nullptr, *tq = nullptr;
    // growable workspaces
    DBuf ws_x, ws_z, ws_fin, ws_lbar, ws_gm, ws_bi, ws_wrow;

    void* take(size_t bytes) {
        void* p = al.get(bytes);
        if (p) owned.push_back(DBuf{p, bytes});
        return p;
    }
    double* grow(DBuf& b, size_t bytes) {
        if (b.bytes >= bytes && b.p) return static_cast<double*>(b.p);
        al.put(b.p);
        b.p = al.get(bytes);
        b.bytes = b.p ? bytes : 0;
        return static_cast<double*>(b.p);
    }
    PatDev dev(unsigned long long* trace = nullptr, RowKernel kind = RowKernel::Numeric, int32_t group = 0,
               int32_t tickets = 0) const {
        PatDev d;
        d.trace = trace;
        d.parts = tickets ? tickets : kTicketParts;  // task counters (see next_pos)
        d.groupL = group ? group : row_group(kind, n, depth_l);
        d.groupU = group ? group : row_group(kind, n, depth_u);
        d.n = (int32_t)n;
        d.nnz_a = (int32_t)nnz_a;
        d.nnz_f = (int32_t)nnz_f;
        d.rpA = rpA; d.ciA = ciA; d.rpF = rpF; d.ciF = ciF; d.diagF = diagF; d.a2f = a2f;
        d.lsd = lsd; d.sptr = sptr; d.sq = sq; d.sp = sp;
        d.permL = permL; d.permU = permU;
        d.tptr = tptr; d.tsl = tsl; d.tq = tq;
        return d;
    }
    ~tpilu_pattern_s() {
        for (auto& b : owned) al.put(b.p);
        al.put(ws_x.p); al.put(ws_z.p); al.put(ws_fin.p); al.put(ws_lbar.p); al.put(ws_gm.p); al.put(ws_bi.p);
        al.put(ws_wrow.p);
    }
};

PatDev pdev(tpilu_ctx ctx, tpilu_pattern pat, RowKernel kind = RowKernel::Numeric, bool trace = false) {
    return pat->dev(trace ? ctx->trace : nullptr, kind, ctx->group, ctx->tickets);
}

// A captured batch: its graph, and the intermediate vector and control block
// the captured kernels use, owned by the graph so that no later call on the
// pattern (which may regrow or reuse the pattern's own workspace and control
// block) can touch them.  The pattern's read-only arrays are used too: the
// pattern must outlive the graph.
struct tpilu_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    Alloc al;
    double* x = nullptr;
    Ctl* ctl = nullptr;
    double* wrow = nullptr;  // global working rows of a batch with long rows
    ~tpilu_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        al.put(x);
        al.put(ctl);
        al.put(wrow);
    }
};

namespace {

tpilu_status fail(tpilu_ctx ctx, tpilu_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

#define HIPCHK(ctx, call)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((ctx), TPILU_E_DEVICE,                                                \
                        std::string(#call) + ": " + hipGetErrorString(e_));                   \
    } while (0)

Alloc ctx_alloc(tpilu_ctx c) {
    Alloc a;
    a.alloc = c->alloc;
    a.free_fn = c->free_fn;
    a.user = c->user;
    return a;
}

uint32_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return (uint32_t)std::min<uint64_t>(p, 1ull << 31);
}

// read the control block after the stream drained and turn it into a status
tpilu_status read_ctl(tpilu_ctx ctx, tpilu_pattern pat, int64_t* bad_row, bool clear) {
    Ctl h{};
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(&h, pat->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (clear) {
        Ctl z{};
        z.bad_row = ~0ull;
        HIPCHK(ctx, hipMemcpy(pat->ctl, &z, sizeof(Ctl), hipMemcpyHostToDevice));
    }
    const int64_t bad = h.bad_row == ~0ull ? -1 : (int64_t)h.bad_row;
    if (bad_row) *bad_row = bad;
    if (h.status & kStTimeout)
        return fail(ctx, TPILU_E_TIMEOUT, "a dependency wait ran out (watchdog)");
    if (h.status & kStReservedNaN)
        return fail(ctx, TPILU_E_INVAL, "input holds the reserved NaN bit pattern 0x7FF4A5A5A5A5A5A5");
    if (bad >= 0) return fail(ctx, TPILU_E_ZEROPIVOT, "zero pivot in row " + std::to_string(bad));
    return TPILU_OK;
}

// Brackets one kernel launch with events when timing is on (and the stream is
// not being captured).
struct TimedLaunch {
    tpilu_ctx ctx;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(tpilu_ctx c, int k, bool allowed = true) : ctx(c), kind(k) {
        if (!ctx->timing || !allowed) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        if (hipEventCreate(&a) != hipSuccess) { a = nullptr; return; }
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); a = nullptr; return; }
        (void)hipEventRecord(a, ctx->stream);
    }
    ~TimedLaunch() {
        if (!a) return;
        (void)hipEventRecord(b, ctx->stream);
        ctx->ev[kind].push_back({a, b});
    }
};

tpilu_status check_common(tpilu_ctx ctx, tpilu_pattern pat, int32_t batch) {
    if (!ctx) return TPILU_E_INVAL;
    if (!pat) return fail(ctx, TPILU_E_INVAL, "null pattern");
    if (batch < 1) return fail(ctx, TPILU_E_INVAL, "batch must be >= 1");
    if ((int64_t)pat->n * batch >= (1ll << 31) || pat->nnz_f * (int64_t)batch >= (1ll << 40))
        return fail(ctx, TPILU_E_INVAL, "batch too large");
    return TPILU_OK;
}

constexpr size_t kBatchLdsLimit = 64 * 1024;
size_t batch_numeric_lds(int32_t max_row) {
    return (size_t)std::max(max_row, 1) * 8 * 64 + 24 * 1024;
}

// The batched kernel keeps a row of 64 instances in LDS (512 bytes per
// entry) up to 80 entries (64 KB with its staging); longer rows go to global
// memory: a slice of grid x max_row x 64 doubles.  The grid is the kernel's
// resident maximum, cut so that the slices stay within kBatchRowBytes.
// Measured on MI355X, rows in up to 160 KB of LDS (two wavefronts per CU)
// were slower than in global memory (seven per CU): 27-point 20^3 ILU(2),
// 70 instances, 24.8 vs 22.1 ms; ILU(3), 5 instances, 46.6 vs 44.2 ms;
// 27-point 30^3 ILU(2), 256 instances, 142 vs 107 ms.
constexpr size_t kBatchRowBytes = size_t(1) << 30;
bool batch_global_row(tpilu_ctx, tpilu_pattern pat, int32_t batch) {
    return batch > 1 && batch_numeric_lds(pat->st.max_row) > kBatchLdsLimit;
}
// the batched kernels on one XCD (explicit placement only)
bool batch_one_xcd(tpilu_ctx ctx, int32_t batch) { return batch > 1 && ctx->placement == 2; }
// working wavefronts of a batched factorization (on one XCD: of that XCD)
int batch_numeric_grid(tpilu_ctx ctx, tpilu_pattern pat, int32_t batch) {
    const bool gr = batch_global_row(ctx, pat, batch);
    int grid = ctx->grid_override ? ctx->grid_override
                                  : std::max(1, numeric_grid(batch, pat->st.max_row, pat->st.max_lrow, false,
                                                             ctx->num_cu, gr) /
                                                    (batch_one_xcd(ctx, batch) ? kXcds : 1));
    if (gr && !ctx->grid_override) {
        const size_t per = (size_t)std::max(pat->st.max_row, 1) * 64 * sizeof(double);
        grid = (int)std::max<size_t>(1, std::min<size_t>((size_t)grid, kBatchRowBytes / per));
    }
    return grid;
}
// bytes of the global working rows a batched factorization needs (0: none)
size_t numeric_wrow_bytes(tpilu_ctx ctx, tpilu_pattern pat, int32_t batch) {
    if (!batch_global_row(ctx, pat, batch)) return 0;
    return (size_t)batch_numeric_grid(ctx, pat, batch) * (size_t)std::max(pat->st.max_row, 1) * 64 *
           sizeof(double);
}

// wrow: numeric_wrow_bytes(ctx, pat, batch) bytes of device memory, or null
// when that is 0.  b, x (batches only, both or neither): the forward
// substitution x = L~^-1 b fused into the factorization.
tpilu_status enqueue_numeric(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val, int32_t batch,
                             double* f_val, Ctl* ctl, double* wrow, const double* b = nullptr,
                             double* x = nullptr) {
    if ((x || b) && (batch < 2 || !x || !b)) return fail(ctx, TPILU_E_INVAL, "fused forward: batches only");
    if (batch == 1 && (size_t)pat->st.max_row * 8 + 12 * 1024 > kBatchLdsLimit)
        return fail(ctx, TPILU_E_INVAL, "numeric factorization supports rows of at most 6600 entries");
    if (batch == 1 && ctx->numeric == 1 && !pat->flow)
        return fail(ctx, TPILU_E_INVAL, "the rows of this pattern do not fit the dataflow numeric kernel");
    // automatic choice: rows with very short L parts (a few pivots each) gain
    // nothing from spreading a row over lanes and pay for the extra staging;
    // long update chains per entry (a lane walks its entry's chain alone) are
    // faster pivot by pivot with the lanes over that pivot's updates.
    // Measured: random banded n=160,000 ILU(2) (1.7 updates per entry)
    // 6.0 ms dataflow vs 22.9 ms pivot-serial; 27-point 50^3 ILU(2) and ILU(3)
    // (16.5 and 26 per entry) 20.8 and 38.7 ms dataflow vs 4.7 and 8.6 ms.
    const bool auto_flow = (int64_t)pat->st.nnz_l >= kFlowMinL * pat->n &&
                           pat->n_updates < kFlowMaxChain * pat->nnz_f &&
                           pat->n < kFlowMaxWidth * std::max<int64_t>(pat->depth_l, 1);
    const bool flow = batch == 1 && pat->flow && (ctx->numeric == 1 || (ctx->numeric == 0 && auto_flow));
    // one XCD only when asked for: the factorization keeps many rows in flight
    // and needs the whole device (random banded n=160,000 ILU(2) ran 3x
    // slower on one XCD); there the grid is that XCD's resident maximum
    const bool one_xcd = ctx->placement == 2;
    const int grid = batch > 1 ? batch_numeric_grid(ctx, pat, batch)
                     : ctx->grid_override
                         ? ctx->grid_override
                         : std::max(1, numeric_grid(batch, pat->st.max_row, pat->st.max_lrow, flow, ctx->num_cu) /
                                           (one_xcd ? kXcds : 1));
    if (batch_global_row(ctx, pat, batch) && !wrow) return fail(ctx, TPILU_E_NOMEM, "batched working rows");
    {
        // the timed region holds the pending-marker fill of F too: the
        // elimination cannot run without it
        TimedLaunch tl(ctx, TPILU_KERNEL_NUMERIC);
        HIPCHK(ctx, launch_fill_pending_upper(f_val, (int32_t)pat->n, pat->rpF, pat->diagF, batch, ctl, true,
                                              ctx->stream));
        if (x) HIPCHK(ctx, launch_fill_pending(x, pat->n * batch, ctl, false, ctx->stream));
        HIPCHK(ctx, launch_numeric(pdev(ctx, pat, RowKernel::Numeric, true), a_val, batch, f_val, ctl,
                                   ctx->spin_limit, ctx->skip_row, grid, pat->st.max_row, pat->st.max_lrow, flow,
                                   one_xcd, batch_global_row(ctx, pat, batch) ? wrow : nullptr, b, x,
                                   ctx->fused, ctx->stream));
    }
    return TPILU_OK;
}

// Launch shape of the single-instance solves, per direction (the grid
// argument of launch_forward / launch_backward): > 0 wavefront per row with
// that many wavefronts (on one XCD when one_xcd), 0 one workgroup, < 0 lane
// per row with -grid wavefronts.  Automatic choice: lane per row when the rows are short and a
// dependency level is wide next to the row length (a lane runs a whole row
// alone, so it needs many rows per level to beat 64 lanes on one row),
// namely rows per level >= max(64, 16 x average entries per row half); else
// a wavefront per row; few rows per level want fewer wavefronts (hand-offs
// dominate), many rows more.  Measured on MI355X: 7-point 64^3 ILU(1) (692
// rows per level, 6 entries per half) 0.8 vs 2.1 ms by lane; 27-point 90^3
// ILU(1) (630 rows, 30 entries) 6.3 vs 8.2 ms by lane; 27-point 70^3 ILU(1)
// (382 rows, 30 entries) 3.9 vs 4.3 ms by wavefront; 27-point 30^3 ILU(1)
// (71 rows) 0.46 vs 1.6 ms by wavefront; random banded n=160,000 ILU(2) (82
// entries per half) 3x faster by wavefront.
constexpr int64_t kLaneMaxAvg = 40;    // average entries per row half at or below
constexpr int64_t kLaneMinWidth = 64;  // rows per dependency level at or above
constexpr int64_t kLaneWidthPerEntry = 16;  // ... and at or above this many per entry of a row half
constexpr int32_t kLaneWaves = 128;

struct SolveShape {
    int32_t grid;  // 0: one CU (launch_solve_cu)
    bool one_xcd;
};

// placement of a wavefront-per-row sweep over n rows of `depth` dependency
// levels whose row halves hold `half` entries in all (rule at kXcdMaxAvg)
bool solve_on_xcd(tpilu_ctx ctx, int64_t n, int64_t half, int64_t depth) {
    if (ctx->placement != 0) return ctx->placement == 2;
    const int64_t width = n / std::max<int64_t>(depth, 1);
    return (width < kNarrowWidth && half <= kXcdMaxAvg * n) || (width < 64 && half < 64 * n);
}

SolveShape solve_shape(tpilu_ctx ctx, tpilu_pattern pat, int32_t batch, bool backward) {
    if (batch > 1) {
        const bool x = batch_one_xcd(ctx, batch);
        return {ctx->grid_override ? ctx->grid_override : x ? kBatchSolveWavesXcd : kBatchSolveWaves, x};
    }
    const int64_t n = std::max<int64_t>(pat->n, 1);
    const int64_t half = backward ? pat->nnz_f - (int64_t)pat->st.nnz_l - pat->n : (int64_t)pat->st.nnz_l;
    const int64_t depth = std::max<int64_t>(1, backward ? pat->depth_u : pat->depth_l);
    int mode = ctx->solver;
    if (mode == 0) {
        const int64_t width = n / depth;
        const bool lanes = half <= kLaneMaxAvg * n && width >= kLaneMinWidth &&
                           width * n >= kLaneWidthPerEntry * half;
        mode = lanes ? 3 : 1;
    }
    if (mode == 2) return {0, false};
    if (mode == 3) return {-(ctx->grid_override ? ctx->grid_override : kLaneWaves), false};
    const int64_t width = n / depth;
    const bool one_xcd = solve_on_xcd(ctx, n, half, depth);
    if (ctx->grid_override) return {ctx->grid_override, one_xcd};
    if (width < kNarrowWidth) return {kSolveWavesNarrow, one_xcd};
    if (width < 64 && half < 64 * n) return {kSolveWavesMid, one_xcd};
    return {kSolveWavesWide, one_xcd};
}

// forward = false: x already holds L~^-1 b (the batched factorization with
// the forward substitution fused in); only the backward sweep runs
tpilu_status enqueue_apply(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val, int32_t batch,
                           const double* b, double* y, double* x, bool reset, Ctl* ctl, bool timed = true,
                           bool forward = true) {
    SolveShape gf = solve_shape(ctx, pat, batch, false), gb = solve_shape(ctx, pat, batch, true);
    // the one-CU shape needs the dependency positions; without them (never
    // built, and this call may not allocate) the wavefront-per-row shape runs
    if (!pat->dep_pos) {
        if (gf.grid == 0) gf = {kSolveWavesNarrow, true};
        if (gb.grid == 0) gb = {kSolveWavesNarrow, true};
    }
    const PatDev P = pdev(ctx, pat, RowKernel::Solve, true);
    // the one-CU kernel hands values over through LDS and needs no pending
    // marks in the output; the control block is reset all the same
    if (forward) {
        HIPCHK(ctx, launch_fill_pending(x, gf.grid == 0 ? 0 : pat->n * batch, ctl, reset, ctx->stream));
        TimedLaunch tl(ctx, TPILU_KERNEL_FORWARD, timed);
        if (gf.grid == 0)
            HIPCHK(ctx, launch_solve_cu(P, pat->dep_pos, f_val, b, x, false, ctl, ctx->spin_limit, ctx->stream));
        else
            HIPCHK(ctx, launch_forward(P, f_val, batch, b, x, ctl, ctx->spin_limit, gf.grid, gf.one_xcd,
                                       ctx->stream));
    }
    HIPCHK(ctx, launch_fill_pending(y, gb.grid == 0 ? 0 : pat->n * batch, ctl, false, ctx->stream));
    {
        TimedLaunch tl(ctx, TPILU_KERNEL_BACKWARD, timed);
        if (gb.grid == 0)
            HIPCHK(ctx, launch_solve_cu(P, pat->dep_pos, f_val, x, y, true, ctl, ctx->spin_limit, ctx->stream));
        else
            HIPCHK(ctx, launch_backward(P, f_val, batch, x, y, ctl, ctx->spin_limit, gb.grid, gb.one_xcd,
                                        ctx->stream));
    }
    return TPILU_OK;
}


// temporaries released when the enclosing call returns
struct TmpBufs {
    Alloc al;
    std::vector<void*> v;
    void* get(size_t b) {
        void* p = al.get(b);
        if (p) v.push_back(p);
        return p;
    }
    ~TmpBufs() { for (void* p : v) al.put(p); }
};

// Per F slot, the level-order position of the row its column names, for the
// one-CU solves.
tpilu_status build_dep_positions(tpilu_ctx ctx, tpilu_pattern pat) {
    if (pat->dep_pos || pat->n == 0) return TPILU_OK;
    const int32_t n = (int32_t)pat->n;
    TmpBufs T{pat->al, {}};
    int32_t* ipl = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);
    int32_t* ipu = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);
    int32_t* pq = (int32_t*)pat->take(sizeof(int32_t) * (size_t)pat->nnz_f);
    if (!ipl || !ipu || !pq) return fail(ctx, TPILU_E_NOMEM, "dependency positions");
    HIPCHK(ctx, launch_dep_positions(n, pat->rpF, pat->ciF, pat->diagF, pat->permL, pat->permU, ipl, ipu, pq,
                                     ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    pat->dep_pos = pq;
    return TPILU_OK;
}

// Levels of one or two dependency DAGs (computed in one launch, so their
// chains overlap) and their nodes sorted by level (the ticket order of the
// kernels that walk them).  deps = number of edges: with long dependency
// lists a wavefront per node in natural order, else a lane per node so that
// every node is in flight at once.
struct LevelSpec {
    DepGraph G;
    int desc;
    int64_t deps;
    int32_t* depth;
    int32_t* perm;
    int32_t* max_depth;
};

// Enqueue the level computation on stream s without waiting for it: the
// level-order sort is sized for the largest possible depth (n), so no host
// read-back is needed; the maxima land in dmax (16 ints apart).  Temporaries
// come from T and must outlive the work.
tpilu_status enqueue_levels(tpilu_ctx ctx, tpilu_pattern pat, const LevelSpec* js, int njobs, hipStream_t s,
                            TmpBufs& T, int32_t** dmax_out) {
    const int32_t n = (int32_t)pat->n;
    int32_t* dmax = (int32_t*)T.get(sizeof(int32_t) * 32);
    Ctl* ctl2 = (Ctl*)T.get(sizeof(Ctl));
    if (!dmax || !ctl2) return fail(ctx, TPILU_E_NOMEM, "levels");
    *dmax_out = dmax;
    int64_t deps = 0;
    for (int q = 0; q < njobs; ++q) deps = std::max(deps, js[q].deps);
    const int32_t lane_waves = (int32_t)std::min<int64_t>(((int64_t)n + 63) / 64, 8192);
    // Shape by dependencies per node: a lane per node for short lists (every
    // node in flight, a lane scans its few dependencies itself); a wavefront
    // per node otherwise, with a wide window of nodes in flight (natural
    // order hands out consecutive nodes, whose chains need many lines of the
    // grid in flight at once) unless the lists are long.  Measured (ms):
    // 64^3 7-point ILU(1) lanes 9.6 / waves 17.6; 27-point 90^3 ILU(1) 192
    // waves 152, 768 waves 71; 64^3 ILU(3) 72 lanes, 31 at 768 waves; random
    // banded n=160,000 ILU(2) 28.5 at 192 waves, 32 at 768.
    const int64_t avg = deps / std::max<int64_t>(n, 1);
    const int32_t grid = avg < kLevelLaneMax ? -lane_waves : (avg < kLevelWideMax ? kLevelWavesWide
                                                                                    : kLevelWavesNarrow);
    LevelJob jb[2];
    for (int q = 0; q < njobs; ++q) {
        HIPCHK(ctx, launch_fill_i32(js[q].depth, n, -1, s));
        jb[q] = LevelJob{js[q].G, js[q].desc, js[q].depth, q == 0 ? pat->ctl : ctl2};
    }
    HIPCHK(ctx, launch_fill_pending(nullptr, 0, pat->ctl, true, s));
    HIPCHK(ctx, launch_fill_pending(nullptr, 0, ctl2, false, s));
    // one XCD per DAG only when the placement setting asks for it: on its own
    // the level kernel gains there (random banded n=160,000 ILU(2): 14.9 ->
    // 9.6 ms), but it runs beside the update schedule, whose launches on the
    // same XCDs then slow down (6.2 -> 11 ms), and Phase I as a whole gains
    // nothing (27.2 vs 30.1 ms; 27-point 50^3 ILU(3) 50.1 vs 53.0 ms)
    const bool lv_xcd = grid > 0 && ctx->placement == 2;
    HIPCHK(ctx, launch_depth(n, jb[0], njobs > 1 ? &jb[1] : nullptr, pat->ctl, ctx->spin_limit, grid, lv_xcd, s));
    HIPCHK(ctx, launch_fill_i32(dmax, 32, 0, s));
    for (int q = 0; q < njobs; ++q) {
        HIPCHK(ctx, launch_max_i32(js[q].depth, n, dmax + 16 * q, s));
        int32_t* hist = (int32_t*)T.get(sizeof(int32_t) * 2 * (size_t)std::max(n, 1));
        int64_t* off = (int64_t*)T.get(sizeof(int64_t) * ((size_t)n + 1));
        int64_t* stmp = (int64_t*)T.get(sizeof(int64_t) * scan_tmp_elems(std::max(n, 1)));
        if (!hist || !off || !stmp) return fail(ctx, TPILU_E_NOMEM, "level order");
        HIPCHK(ctx, launch_level_order(n, js[q].depth, std::max(n, 1), hist, off, stmp, js[q].perm, s));
    }
    return TPILU_OK;
}

// After the level work has completed: the maxima to the host, and the
// watchdog / abort status of the level kernels.
tpilu_status finish_levels(tpilu_ctx ctx, tpilu_pattern pat, const LevelSpec* js, int njobs, const int32_t* dmax) {
    int32_t dm[32] = {0};
    HIPCHK(ctx, hipMemcpy(dm, dmax, sizeof(dm), hipMemcpyDeviceToHost));
    for (int q = 0; q < njobs; ++q) *js[q].max_depth = dm[16 * q];
    return read_ctl(ctx, pat, nullptr, false);
}

tpilu_status compute_levels(tpilu_ctx ctx, tpilu_pattern pat, const LevelSpec* js, int njobs) {
    TmpBufs T{pat->al, {}};
    int32_t* dmax = nullptr;
    tpilu_status st = enqueue_levels(ctx, pat, js, njobs, ctx->stream, T, &dmax);
    if (st != TPILU_OK) return st;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return finish_levels(ctx, pat, js, njobs, dmax);
}

// Shape of the two products (kProd*): as the solver mode asks (1 a wavefront
// per row, 3 a thread per row) or automatically: 64 rows per wavefront
// staged through LDS (each lane one row's in-order sum) when the rows are of
// even length (longest row at most 1.5 x the average) and not very long,
// else a wavefront per row.  Measured on MI355X (both products): 7-point
// 64^3 ILU(1), 13 entries per row: 0.042 ms tiled, 0.061 by thread, 0.165
// by wavefront; 27-point 50^3 ILU(3), 165 per row (longest 183): 0.147 vs
// 0.225 ms by wavefront; random banded n=160,000 ILU(2), 164 per row (longest
// 419): 0.29 ms by wavefront, 0.35 tiled; paper-scale ILU(1), 1,276 per row:
// 1.9 ms by wavefront, 2.8 tiled.
constexpr int64_t kInvTileMaxAvg = 512;
constexpr int64_t kInvShortAvg = 24;  // entries per row of F at or below: 8-entry tiles
int inverse_product_shape(tpilu_ctx ctx, tpilu_pattern pat) {
    if (ctx->solver == 1) return kProdWaveRows;
    if (ctx->solver == 3) return kProdThreadRows;
    const int64_t n = std::max<int64_t>(pat->n, 1);
    if (pat->nnz_f > kInvTileMaxAvg * n) return kProdWaveRows;
    return pat->nnz_f <= kInvShortAvg * n ? kProdTileShort : kProdTile;
}

tpilu_status build_inverse_sched(tpilu_ctx ctx, tpilu_pattern pat) {
    if (pat->have_inv) return TPILU_OK;
    if (isched_lds_bytes(pat->st.max_row) > kBatchLdsLimit)
        return fail(ctx, TPILU_E_INVAL, "incomplete inverses support rows of at most 4096 entries");
    const int32_t n = (int32_t)pat->n;
    const int64_t nnzf = pat->nnz_f;
    hipStream_t s = ctx->stream;
    TmpBufs T{pat->al, {}};
    int32_t* cnt = (int32_t*)T.get(sizeof(int32_t) * (size_t)nnzf);
    int64_t* stmp = (int64_t*)T.get(sizeof(int64_t) * scan_tmp_elems(nnzf));
    int64_t* iptr = (int64_t*)pat->take(sizeof(int64_t) * (size_t)(nnzf + 1));
    if (!cnt || !stmp || !iptr) return fail(ctx, TPILU_E_NOMEM, "inverse schedule");
    for (int up = 0; up < 2; ++up)
        HIPCHK(ctx, launch_isched(n, pat->rpF, pat->ciF, pat->diagF, up, 0, cnt, nullptr, nullptr, nullptr,
                                  pat->st.max_row, s));
    HIPCHK(ctx, launch_scan(cnt, nnzf, iptr, stmp, s));
    int64_t total = 0;
    HIPCHK(ctx, hipMemcpyAsync(&total, iptr + nnzf, sizeof(total), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    int32_t* ps = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
    int32_t* pq = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(total, 1));
    if (!ps || !pq) return fail(ctx, TPILU_E_NOMEM, "inverse schedule");
    for (int up = 0; up < 2; ++up)
        HIPCHK(ctx, launch_isched(n, pat->rpF, pat->ciF, pat->diagF, up, 1, nullptr, iptr, ps, pq,
                                  pat->st.max_row, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    pat->iptr = iptr;
    pat->is_s = ps;
    pat->is_q = pq;
    pat->n_inv_updates = total;
    pat->have_inv = true;
    return TPILU_OK;
}

// waits for the second stream when it goes out of scope (before the
// temporaries declared ahead of it are released)
struct AuxJoin {
    hipStream_t a = nullptr;
    ~AuxJoin() {
        if (a) (void)hipStreamSynchronize(a);
    }
};

hipError_t ctx_aux(tpilu_ctx ctx) {
    if (!ctx->aux) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ctx->aux = nullptr;
            return e;
        }
    }
    if (!ctx->fork_ev) {
        hipError_t e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            ctx->fork_ev = nullptr;
            return e;
        }
    }
    if (!ctx->join_ev) {
        hipError_t e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            ctx->join_ev = nullptr;
            return e;
        }
    }
    return hipSuccess;
}

tpilu_status build_transposes(tpilu_ctx ctx, tpilu_pattern pat) {
    if (pat->have_t) return TPILU_OK;
    const int32_t n = (int32_t)pat->n;
    hipStream_t s = ctx->stream;
    int32_t* cnt = (int32_t*)pat->take(sizeof(int32_t) * (size_t)(4 * n + 4));
    int64_t* tmp = (int64_t*)pat->take(sizeof(int64_t) * scan_tmp_elems(n));
    pat->tpL = (int64_t*)pat->take(sizeof(int64_t) * (size_t)(n + 1));
    pat->tpU = (int64_t*)pat->take(sizeof(int64_t) * (size_t)(n + 1));
    if (!cnt || !tmp || !pat->tpL || !pat->tpU) return fail(ctx, TPILU_E_NOMEM, "transpose");
    int32_t *cntL = cnt, *cntU = cnt + n, *curL = cnt + 2 * n, *curU = cnt + 3 * n;
    HIPCHK(ctx, launch_fill_i32(cnt, 4 * (int64_t)n, 0, s));
    HIPCHK(ctx, launch_transpose_count(n, pat->rpF, pat->ciF, pat->diagF, cntL, cntU, s));
    HIPCHK(ctx, launch_scan(cntL, n, pat->tpL, tmp, s));
    HIPCHK(ctx, launch_scan(cntU, n, pat->tpU, tmp, s));
    const int64_t nl = (int64_t)pat->st.nnz_l;
    const int64_t nu = pat->nnz_f - nl - pat->n;
    pat->tsL = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nl, 1));
    pat->trL = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nl, 1));
    pat->tsU = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nu, 1));
    pat->trU = (int32_t*)pat->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nu, 1));
    if (!pat->tsL || !pat->trL || !pat->tsU || !pat->trU) return fail(ctx, TPILU_E_NOMEM, "transpose");
    HIPCHK(ctx, launch_transpose_fill(n, pat->rpF, pat->ciF, pat->diagF, pat->tpL, pat->tsL, pat->trL,
                                      pat->tpU, pat->tsU, pat->trU, curL, curU, s));
    HIPCHK(ctx, launch_sort_columns(n, pat->tpL, pat->tsL, pat->trL, s));
    HIPCHK(ctx, launch_sort_columns(n, pat->tpU, pat->tsU, pat->trU, s));
    // level orders of the transposed sweeps: U~^T ascending (row i waits on
    // the rows of column i of U~), L~^T descending (on those of column i of L~)
    int32_t* depth = (int32_t*)pat->take(sizeof(int32_t) * (size_t)n);
    pat->permUT = (int32_t*)pat->take(sizeof(int32_t) * (size_t)n);
    pat->permLT = (int32_t*)pat->take(sizeof(int32_t) * (size_t)n);
    if (!depth || !pat->permUT || !pat->permLT) return fail(ctx, TPILU_E_NOMEM, "transpose levels");
    int32_t* depth2 = (int32_t*)pat->take(sizeof(int32_t) * (size_t)n);
    if (!depth2) return fail(ctx, TPILU_E_NOMEM, "transpose levels");
    int32_t dm0 = 0, dm1 = 0;
    const LevelSpec js[2] = {{DepGraph{pat->tpU, pat->trU, nullptr, 2}, 0, nu, depth, pat->permUT, &dm0},
                             {DepGraph{pat->tpL, pat->trL, nullptr, 2}, 1, nl, depth2, pat->permLT, &dm1}};
    tpilu_status st = compute_levels(ctx, pat, js, 2);
    if (st) return st;
    pat->have_t = true;
    return TPILU_OK;
}

}  // namespace

// =====================================================================================
// context
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_ctx_create(int device, void* hip_stream, tpilu_alloc_fn alloc,
                                                   tpilu_free_fn free_fn, void* user, tpilu_ctx* out) {
    if (!out) return TPILU_E_INVAL;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return TPILU_E_INVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TPILU_E_DEVICE;
    tpilu_ctx c = new (std::nothrow) tpilu_ctx_s;
    if (!c) return TPILU_E_NOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->alloc = alloc;
    c->free_fn = free_fn;
    c->user = user;
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
        c->num_cu = cu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        c->ticks_per_us = std::max<uint64_t>(1, (uint64_t)khz / 1000);
    c->spin_limit = kDefaultWaitUs * c->ticks_per_us;
    {
        // the no-alloc scratch's address on this device, with the device current
        DeviceGuard dg(device);
        c->scratch = scratch_on(device, &c->scratch_err);
    }
    *out = c;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_stream(tpilu_ctx ctx, void* hip_stream) {
    if (!ctx) return TPILU_E_INVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return TPILU_OK;
}

extern "C" TPILU_API void tpilu_ctx_destroy(tpilu_ctx ctx) { delete ctx; }

extern "C" TPILU_API tpilu_status tpilu_ctx_set_watchdog(tpilu_ctx ctx, uint32_t timeout_us,
                                                         int64_t skip_publish_row) {
    if (!ctx) return TPILU_E_INVAL;
    ctx->spin_limit = (timeout_us ? (uint64_t)timeout_us : kDefaultWaitUs) * ctx->ticks_per_us;
    ctx->skip_row = skip_publish_row;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_grid(tpilu_ctx ctx, int32_t waves) {
    if (!ctx) return TPILU_E_INVAL;
    if (waves < 0) return fail(ctx, TPILU_E_INVAL, "waves must be >= 0");
    ctx->grid_override = waves;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_group(tpilu_ctx ctx, int32_t rows) {
    if (!ctx) return TPILU_E_INVAL;
    if (rows < 0 || rows > 64) return fail(ctx, TPILU_E_INVAL, "rows per ticket must be in [0, 64]");
    ctx->group = rows;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_tickets(tpilu_ctx ctx, int32_t counters) {
    if (!ctx) return TPILU_E_INVAL;
    if (counters < 0 || counters > kTicketParts)
        return fail(ctx, TPILU_E_INVAL, "task counters must be in [0, 8]");
    ctx->tickets = counters;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_trace(tpilu_ctx ctx, uint64_t* rows4n) {
    if (!ctx) return TPILU_E_INVAL;
    ctx->trace = reinterpret_cast<unsigned long long*>(rows4n);
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_solver(tpilu_ctx ctx, int mode) {
    if (!ctx) return TPILU_E_INVAL;
    if (mode < 0 || mode > 3) return fail(ctx, TPILU_E_INVAL, "solver mode must be 0, 1, 2 or 3");
    ctx->solver = mode;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_numeric(tpilu_ctx ctx, int mode) {
    if (!ctx) return TPILU_E_INVAL;
    if (mode < 0 || mode > 2) return fail(ctx, TPILU_E_INVAL, "numeric mode must be 0, 1 or 2");
    ctx->numeric = mode;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_fused(tpilu_ctx ctx, int on) {
    if (!ctx) return TPILU_E_INVAL;
    if (on < 0 || on > 1) return fail(ctx, TPILU_E_INVAL, "fused must be 0 or 1");
    ctx->fused = on == 1;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_placement(tpilu_ctx ctx, int where) {
    if (!ctx) return TPILU_E_INVAL;
    if (where < 0 || where > 2) return fail(ctx, TPILU_E_INVAL, "placement must be 0, 1 or 2");
    ctx->placement = where;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_set_timing(tpilu_ctx ctx, int on) {
    if (!ctx) return TPILU_E_INVAL;
    ctx->timing = on != 0;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_ctx_read_timing(tpilu_ctx ctx, int kernel, double* total_ms,
                                                       int64_t* launches) {
    if (!ctx) return TPILU_E_INVAL;
    if (kernel < 0 || kernel > 2 || !total_ms || !launches) return fail(ctx, TPILU_E_INVAL, "bad argument");
    DeviceGuard dg(ctx->device);
    double sum = 0.0;
    int64_t cnt = 0;
    tpilu_status st = TPILU_OK;
    for (auto& p : ctx->ev[kernel]) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) != hipSuccess || hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess)
            st = fail(ctx, TPILU_E_DEVICE, "event timing failed");
        sum += ms;
        ++cnt;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    ctx->ev[kernel].clear();
    *total_ms = sum;
    *launches = cnt;
    return st;
}

extern "C" TPILU_API const char* tpilu_status_string(tpilu_status st) {
    switch (st) {
        case TPILU_OK: return "ok";
        case TPILU_E_INVAL: return "invalid argument";
        case TPILU_E_NOMEM: return "out of device memory";
        case TPILU_E_ZEROPIVOT: return "zero pivot";
        case TPILU_E_DEVICE: return "HIP runtime error";
        case TPILU_E_NOTCONV: return "not converged";
        case TPILU_E_TIMEOUT: return "dependency wait timed out";
    }
    return "unknown status";
}

extern "C" TPILU_API const char* tpilu_last_error(tpilu_ctx ctx) {
    return ctx ? ctx->err.c_str() : "null context";
}

// =====================================================================================
// Phase I
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_symbolic(tpilu_ctx ctx, int64_t n, int64_t nnz,
                                                 const int64_t* rowptr, const int32_t* col, int32_t k,
                                                 tpilu_pattern* out) {
    if (!ctx) return TPILU_E_INVAL;
    if (!out) return fail(ctx, TPILU_E_INVAL, "null output");
    *out = nullptr;
    if (n < 0 || n >= (1ll << 31) - 1 || nnz < 0 || nnz >= (1ll << 31) || k < 0)
        return fail(ctx, TPILU_E_INVAL, "n, nnz or k out of range");
    if (n > 0 && (!rowptr || (nnz > 0 && !col))) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    tpilu_pattern P = new (std::nothrow) tpilu_pattern_s;
    if (!P) return fail(ctx, TPILU_E_NOMEM, "pattern");
    P->al = ctx_alloc(ctx);
    P->device = ctx->device;
    P->n = n;
    P->nnz_a = nnz;
    P->k = k;
    bool forked = false;  // work on the second stream may still use P's arrays
    auto bail = [&](tpilu_status st) {
        if (forked) (void)hipStreamSynchronize(ctx->aux);
        delete P;
        return st;
    };
    P->ctl = (Ctl*)P->take(sizeof(Ctl));
    uint32_t* vstat = (uint32_t*)P->take(64);
    P->rpA = (int64_t*)P->take(sizeof(int64_t) * (size_t)(n + 1));
    P->ciA = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    if (!P->ctl || !vstat || !P->rpA || !P->ciA) return bail(fail(ctx, TPILU_E_NOMEM, "pattern arrays"));
    {
        Ctl z{};
        z.bad_row = ~0ull;
        HIPCHK(ctx, hipMemcpyAsync(P->ctl, &z, sizeof(Ctl), hipMemcpyHostToDevice, s));
    }
    if (n == 0) {
        int64_t zero = 0;
        HIPCHK(ctx, hipMemcpyAsync(P->rpA, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        P->rpF = P->rpA;
        HIPCHK(ctx, hipStreamSynchronize(s));
        *out = P;
        return TPILU_OK;
    }
    HIPCHK(ctx, hipMemcpyAsync(P->rpA, rowptr, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToDevice, s));
    if (nnz > 0)
        HIPCHK(ctx, hipMemcpyAsync(P->ciA, col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    // ---- a1: validation
    trace("symbolic: validate", n, nnz);
    HIPCHK(ctx, launch_fill_i32((int32_t*)vstat, 16, 0, s));
    HIPCHK(ctx, launch_validate((int32_t)n, nnz, P->rpA, P->ciA, vstat, s));
    uint32_t vs = 0;
    HIPCHK(ctx, hipMemcpyAsync(&vs, vstat, sizeof(vs), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (vs) {
        std::string m = "invalid CSR:";
        if (vs & kValBadRowptr) m += " rowptr not monotone or not [0, nnz];";
        if (vs & kValBadCol) m += " column index out of range;";
        if (vs & kValUnsorted) m += " columns not strictly ascending;";
        if (vs & kValNoDiag) m += " diagonal entry missing;";
        return bail(fail(ctx, TPILU_E_INVAL, m));
    }
    const int32_t ni = (int32_t)n;
    // ---- a2: level-of-fill pattern, count pass
    TmpBufs T{P->al, {}};
    int32_t* cnt = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);
    int32_t* list0 = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);      // rows tier 0 builds first
    int32_t* over_list = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);  // rows for tier 1
    int32_t* over2_list = (int32_t*)T.get(sizeof(int32_t) * (size_t)n);  // rows past tier 1
    int32_t* over_n = (int32_t*)T.get(64);
    uint8_t* tier_of = (uint8_t*)T.get((size_t)n + 4);
    int64_t* scan_tmp = (int64_t*)T.get(sizeof(int64_t) * scan_tmp_elems(n));
    if (!cnt || !list0 || !over_list || !over2_list || !over_n || !tier_of || !scan_tmp)
        return bail(fail(ctx, TPILU_E_NOMEM, "symbolic scratch"));
    HIPCHK(ctx, launch_fill_i32((int32_t*)tier_of, (n + 4) / 4, 0, s));
    HIPCHK(ctx, launch_fill_i32(over_n, 4, 0, s));
    const int sym_grid = std::min<int64_t>(n, (int64_t)ctx->num_cu * 4);
    // rows whose one-step bound already passes tier 0's capacity start in
    // tier 1 (over_list[0, n_pred)); the rest (list0) start in tier 0
    int32_t n0 = ni;
    if (k >= 1) {
        HIPCHK(ctx, launch_route_rows(ni, P->rpA, P->ciA, cnt, sym_route_limit(), list0, over_list, over_n + 2,
                                      tier_of, s));
        int32_t rc[2] = {0, 0};
        HIPCHK(ctx, hipMemcpyAsync(rc, over_n + 2, sizeof(rc), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        n0 = rc[0];
        HIPCHK(ctx, hipMemcpyAsync(over_n, over_n + 3, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    const int32_t* l0 = k >= 1 ? list0 : nullptr;
    trace("symbolic: count pass, rows starting in tier 0", n, n0);
    HIPCHK(ctx, launch_sym_rows(0, ni, P->rpA, P->ciA, k, l0, n0, 0, cnt, nullptr, nullptr,
                                nullptr, nullptr, nullptr, nullptr, 0, std::min(std::max(n0, 1), sym_grid), s));
    HIPCHK(ctx, launch_collect_overflow(n0, l0, cnt, over_list, over_n, tier_of, 1, s));
    int32_t n_over = 0, n_over2 = 0;
    HIPCHK(ctx, hipMemcpyAsync(&n_over, over_n, sizeof(n_over), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (n_over > 0) {
        // long rows: the same construction with four times the map capacity
        HIPCHK(ctx, launch_sym_rows(1, ni, P->rpA, P->ciA, k, over_list, n_over, 0, cnt, nullptr, nullptr,
                                    nullptr, nullptr, nullptr, nullptr, 0, std::min(n_over, sym_grid), s));
        HIPCHK(ctx, launch_collect_overflow(n_over, over_list, cnt, over2_list, over_n + 1, tier_of, 2, s));
        HIPCHK(ctx, hipMemcpyAsync(&n_over2, over_n + 1, sizeof(n_over2), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
    }
    P->long_rows = n_over - n_over2;
    P->overflow_rows = n_over2;
    trace("symbolic: long rows, overflow rows", n_over - n_over2, n_over2);
    int32_t* gscr = nullptr;
    uint32_t gcap = 0;
    int ggrid = 0;
    if (n_over2 > 0) {
        gcap = next_pow2(2 * (uint64_t)n + 2);
        ggrid = std::min(n_over2, 32);
        gscr = (int32_t*)T.get(sizeof(int32_t) * sym_global_scratch_ints(ni, gcap) * (size_t)ggrid);
        if (!gscr) return bail(fail(ctx, TPILU_E_NOMEM, "symbolic global scratch"));
        HIPCHK(ctx, launch_sym_rows(2, ni, P->rpA, P->ciA, k, over2_list, n_over2, 0, cnt, nullptr, nullptr,
                                    nullptr, nullptr, nullptr, gscr, gcap, ggrid, s));
    }
    P->rpF = (int64_t*)P->take(sizeof(int64_t) * (size_t)(n + 1));
    if (!P->rpF) return bail(fail(ctx, TPILU_E_NOMEM, "rowptr"));
    HIPCHK(ctx, launch_scan(cnt, n, P->rpF, scan_tmp, s));
    int64_t nnzf = 0;
    HIPCHK(ctx, hipMemcpyAsync(&nnzf, P->rpF + n, sizeof(nnzf), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (nnzf >= (1ll << 31) - 1) return bail(fail(ctx, TPILU_E_INVAL, "nnz(F) exceeds 2^31"));
    P->nnz_f = nnzf;
    trace("symbolic: fill pass, nnz(F)", nnzf);
    P->ciF = (int32_t*)P->take(sizeof(int32_t) * (size_t)nnzf);
    P->lvF = (uint8_t*)P->take((size_t)nnzf);
    P->diagF = (int32_t*)P->take(sizeof(int32_t) * (size_t)n);
    P->a2f = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
    P->lsd = (int32_t*)P->take(sizeof(int32_t) * (size_t)nnzf);
    P->sptr = (int64_t*)P->take(sizeof(int64_t) * (size_t)(nnzf + 1));
    if (!P->ciF || !P->lvF || !P->diagF || !P->a2f || !P->lsd || !P->sptr)
        return bail(fail(ctx, TPILU_E_NOMEM, "pattern arrays"));
    // fill pass
    HIPCHK(ctx, launch_sym_rows(0, ni, P->rpA, P->ciA, k, l0, n0, 1, cnt, P->rpF, P->ciF, P->lvF,
                                P->diagF, tier_of, nullptr, 0, std::min(std::max(n0, 1), sym_grid), s));
    if (n_over > 0)
        HIPCHK(ctx, launch_sym_rows(1, ni, P->rpA, P->ciA, k, over_list, n_over, 1, cnt, P->rpF, P->ciF,
                                    P->lvF, P->diagF, tier_of, nullptr, 0, std::min(n_over, sym_grid), s));
    if (n_over2 > 0)
        HIPCHK(ctx, launch_sym_rows(2, ni, P->rpA, P->ciA, k, over2_list, n_over2, 1, cnt, P->rpF, P->ciF,
                                    P->lvF, P->diagF, tier_of, gscr, gcap, ggrid, s));
    // A -> F map
    HIPCHK(ctx, launch_fill_i32((int32_t*)vstat, 16, 0, s));
    HIPCHK(ctx, launch_a2f(ni, P->rpA, P->ciA, P->rpF, P->ciF, P->a2f, vstat, s));
    // statistics
    PatStats* dst = (PatStats*)T.get(sizeof(PatStats));
    if (!dst) return bail(fail(ctx, TPILU_E_NOMEM, "stats"));
    {
        PatStats z{};
        HIPCHK(ctx, hipMemcpyAsync(dst, &z, sizeof(z), hipMemcpyHostToDevice, s));
    }
    HIPCHK(ctx, launch_stats(ni, P->rpF, P->diagF, dst, s));
    HIPCHK(ctx, hipMemcpyAsync(&P->st, dst, sizeof(PatStats), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(&vs, vstat, sizeof(vs), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (vs) return bail(fail(ctx, TPILU_E_INVAL, "internal: an entry of A is missing from F"));
    // ---- dependency levels and the level-ordered schedules, on the second
    // stream: a latency-bound chain on a few wavefronts, overlapped with the
    // throughput-bound update schedules below
    P->depthL = (int32_t*)P->take(sizeof(int32_t) * (size_t)n);
    P->depthU = (int32_t*)P->take(sizeof(int32_t) * (size_t)n);
    P->permL = (int32_t*)P->take(sizeof(int32_t) * (size_t)n);
    P->permU = (int32_t*)P->take(sizeof(int32_t) * (size_t)n);
    if (!P->depthL || !P->depthU || !P->permL || !P->permU) return bail(fail(ctx, TPILU_E_NOMEM, "levels"));
    const int64_t nl_ = (int64_t)P->st.nnz_l, nu_ = nnzf - nl_ - n;
    const LevelSpec ljobs[2] = {{DepGraph{P->rpF, P->ciF, P->diagF, 0}, 0, nl_, P->depthL, P->permL, &P->depth_l},
                                {DepGraph{P->rpF, P->ciF, P->diagF, 1}, 1, nu_, P->depthU, P->permU, &P->depth_u}};
    AuxJoin aux_join;
    int32_t* ldmax = nullptr;
    {
        trace("symbolic: forward and backward levels (second stream)");
        HIPCHK(ctx, ctx_aux(ctx));
        HIPCHK(ctx, hipEventRecord(ctx->fork_ev, s));
        HIPCHK(ctx, hipStreamWaitEvent(ctx->aux, ctx->fork_ev, 0));
        aux_join.a = ctx->aux;
        forked = true;
        tpilu_status ls = enqueue_levels(ctx, P, ljobs, 2, ctx->aux, T, &ldmax);
        if (ls != TPILU_OK) return bail(ls);
    }
    // ---- update schedule for Phase II: one search pass that counts and
    // stages the pairs in a pool (sized from a sample of the rows), a scan,
    // and a copy into place; the two-pass form (count, then search again and
    // write) when the pool cannot be had or turns out too small
    trace("symbolic: schedule", P->st.max_row, P->st.max_lrow);
    int32_t* scount = (int32_t*)T.get(sizeof(int32_t) * (size_t)nnzf);
    int64_t* scan2 = (int64_t*)T.get(sizeof(int64_t) * scan_tmp_elems(nnzf));
    unsigned long long* sctr = (unsigned long long*)T.get(64);
    if (!scount || !scan2 || !sctr) return bail(fail(ctx, TPILU_E_NOMEM, "schedule scratch"));
    HIPCHK(ctx, launch_fill_i32((int32_t*)sctr, 16, 0, s));
    SchedPool pool{};
    pool.ctr = sctr;
    pool.sample = sctr + 2;  // [0] pairs, [2] candidates
    pool.overflow = (uint32_t*)(sctr + 3);
    HIPCHK(ctx, launch_sched(ni, P->rpF, P->ciF, P->diagF, 3, nullptr, nullptr, nullptr, nullptr, nullptr,
                             P->st.max_row, s, &pool, kSchedSampleStride));
    unsigned long long sample[3] = {0, 0, 0};  // pairs, (unused), candidates of the sampled rows
    HIPCHK(ctx, hipMemcpyAsync(sample, pool.sample, sizeof(sample), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    // One pass saves a second search (about one probe per candidate) and
    // costs a copy of the pairs and the sample; taken when candidates
    // outnumber pairs kSchedOnePassRatio to 1 (measured on MI355X: random
    // n=160,000 ILU(1), 55 candidates per pair, 697 -> 434 ms; 27-point 50^3
    // ILU(3), few candidates per pair, 53 ms with two passes, 57 with one)
    {
        const int64_t est = (int64_t)sample[0] * kSchedSampleStride;
        const bool worth = (int64_t)sample[2] > kSchedOnePassRatio * (int64_t)sample[0];
        // chunks of about a quarter of a wavefront's expected share (64 to
        // 4096 pairs): few atomics, and little left unused in the chunks
        // the wavefronts hold when they finish
        const int64_t waves = std::min<int64_t>(n, 65536);
        pool.chunk = (int32_t)std::min<int64_t>(4096, std::max<int64_t>(64, (est / waves / 4 + 63) / 64 * 64));
        pool.cap = est + est / 2 + waves * pool.chunk + (1 << 20);
        pool.seg_cap = pool.cap / pool.chunk + n + 1;
        size_t free_b = 0, total_b = 0;
        const bool fits = worth && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                          (size_t)pool.cap * 8 + (size_t)pool.seg_cap * 32 <= free_b / 3;
        if (fits) {
            pool.q = (int32_t*)T.get(sizeof(int32_t) * (size_t)pool.cap);
            pool.p = (int32_t*)T.get(sizeof(int32_t) * (size_t)pool.cap);
            pool.seg = (longlong4*)T.get(sizeof(longlong4) * (size_t)pool.seg_cap);
        }
        if (!pool.q || !pool.p || !pool.seg) {
            pool.cap = 0;
            pool.seg_cap = 0;
        }
    }
    const bool one_pass = pool.cap > 0;
    trace("symbolic: schedule pool (pairs), one pass", pool.cap, one_pass);
    if (one_pass)
        HIPCHK(ctx, launch_sched(ni, P->rpF, P->ciF, P->diagF, 2, scount, P->lsd, nullptr, nullptr, nullptr,
                                 P->st.max_row, s, &pool));
    else
        HIPCHK(ctx, launch_sched(ni, P->rpF, P->ciF, P->diagF, 0, scount, P->lsd, nullptr, nullptr, nullptr,
                                 P->st.max_row, s));
    HIPCHK(ctx, launch_scan(scount, nnzf, P->sptr, scan2, s));
    int64_t nupd = 0;
    unsigned long long pc[4] = {0, 0, 0, 0};
    HIPCHK(ctx, hipMemcpyAsync(&nupd, P->sptr + nnzf, sizeof(nupd), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(pc, sctr, sizeof(pc), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    P->n_updates = nupd;
    const bool pooled = one_pass && (pc[3] & 0xffffffffull) == 0;
    trace("symbolic: schedule updates, taken from the pool", nupd, pooled);
    P->sq = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nupd, 1));
    P->sp = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nupd, 1));
    if (!P->sq || !P->sp) return bail(fail(ctx, TPILU_E_NOMEM, "schedule"));
    if (pooled)
        HIPCHK(ctx, launch_sched_copy(pool, (int64_t)pc[1], P->rpF, P->sptr, P->sq, P->sp, s));
    else
        HIPCHK(ctx, launch_sched(ni, P->rpF, P->ciF, P->diagF, 1, nullptr, nullptr, P->sptr, P->sq, P->sp,
                                 P->st.max_row, s));
    // ---- the same schedule by target, for the dataflow numeric kernel
    if (numeric_flow_fits(P->st.max_row, P->st.max_lrow, kBatchLdsLimit) &&
        tsched_lds_bytes(P->st.max_row, P->st.max_lrow) <= kBatchLdsLimit) {
        trace("symbolic: target-major schedule");
        P->tptr = (int64_t*)P->take(sizeof(int64_t) * (size_t)(nnzf + 1));
        P->tsl = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nupd, 1));
        P->tq = (int32_t*)P->take(sizeof(int32_t) * (size_t)std::max<int64_t>(nupd, 1));
        if (!P->tptr || !P->tsl || !P->tq) return bail(fail(ctx, TPILU_E_NOMEM, "target-major schedule"));
        HIPCHK(ctx, launch_tsched(ni, P->rpF, P->diagF, P->sptr, P->sq, P->sp, 0, scount, nullptr, nullptr, nullptr,
                                  P->st.max_row, P->st.max_lrow, s));
        HIPCHK(ctx, launch_scan(scount, nnzf, P->tptr, scan2, s));
        HIPCHK(ctx, launch_tsched(ni, P->rpF, P->diagF, P->sptr, P->sq, P->sp, 1, nullptr, P->tptr, P->tsl, P->tq,
                                  P->st.max_row, P->st.max_lrow, s));
        P->flow = true;
    }
    // ---- join the level work
    HIPCHK(ctx, hipEventRecord(ctx->join_ev, ctx->aux));
    HIPCHK(ctx, hipStreamWaitEvent(s, ctx->join_ev, 0));
    HIPCHK(ctx, hipStreamSynchronize(s));
    {
        tpilu_status ls = finish_levels(ctx, P, ljobs, 2, ldmax);
        if (ls != TPILU_OK) return bail(ls);
    }
    tpilu_status st = read_ctl(ctx, P, nullptr, true);
    if (st != TPILU_OK) return bail(st);
    *out = P;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_pattern_info(tpilu_pattern pat, tpilu_pattern_info_t* info) {
    if (!pat || !info) return TPILU_E_INVAL;
    info->n = pat->n;
    info->nnz_a = pat->nnz_a;
    info->nnz_f = pat->nnz_f;
    info->nnz_l = (int64_t)pat->st.nnz_l;
    info->nnz_u = pat->nnz_f - (int64_t)pat->st.nnz_l;
    info->n_updates = pat->n_updates;
    info->k = pat->k;
    info->max_row = pat->st.max_row;
    info->max_lrow = pat->st.max_lrow;
    info->depth_l = pat->depth_l;
    info->depth_u = pat->depth_u;
    info->overflow_rows = pat->overflow_rows;
    info->long_rows = pat->long_rows;
    info->flow_ready = pat->flow ? 1 : 0;
    return TPILU_OK;
}

__global__ void k_u8_copy(uint8_t* dst, const uint8_t* src, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

extern "C" TPILU_API tpilu_status tpilu_pattern_export(tpilu_ctx ctx, tpilu_pattern pat, int64_t* rowptr,
                                                       int32_t* col, int32_t* diag, uint8_t* level,
                                                       int32_t* a2f) {
    if (!ctx) return TPILU_E_INVAL;
    if (!pat) return fail(ctx, TPILU_E_INVAL, "null pattern");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    const size_t n = (size_t)pat->n, nf = (size_t)pat->nnz_f, na = (size_t)pat->nnz_a;
    if (rowptr) HIPCHK(ctx, hipMemcpyAsync(rowptr, pat->rpF, 8 * (n + 1), hipMemcpyDeviceToDevice, s));
    if (n == 0) {
        HIPCHK(ctx, hipStreamSynchronize(s));
        return TPILU_OK;
    }
    if (col && nf) HIPCHK(ctx, hipMemcpyAsync(col, pat->ciF, 4 * nf, hipMemcpyDeviceToDevice, s));
    if (diag) HIPCHK(ctx, hipMemcpyAsync(diag, pat->diagF, 4 * n, hipMemcpyDeviceToDevice, s));
    if (level && nf) {
        hipLaunchKernelGGL(k_u8_copy, dim3(1024), dim3(256), 0, s, level, pat->lvF, (int64_t)nf);
        HIPCHK(ctx, hipGetLastError());
    }
    if (a2f && na) HIPCHK(ctx, hipMemcpyAsync(a2f, pat->a2f, 4 * na, hipMemcpyDeviceToDevice, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return TPILU_OK;
}

extern "C" TPILU_API void tpilu_pattern_destroy(tpilu_pattern pat) {
    if (!pat) return;
    DeviceGuard dg(pat->device);
    delete pat;
}

// =====================================================================================
// Phase II and the solves
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_numeric(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val,
                                                int32_t batch, double* f_val, int64_t* bad_row) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (pat->n == 0) {
        if (bad_row) *bad_row = -1;
        return TPILU_OK;
    }
    if (!a_val || !f_val) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    trace("numeric", pat->n, batch);
    double* wrow = nullptr;
    if (const size_t wb = numeric_wrow_bytes(ctx, pat, batch)) {
        wrow = pat->grow(pat->ws_wrow, wb);
        if (!wrow) return fail(ctx, TPILU_E_NOMEM, "batched working rows");
    }
    st = enqueue_numeric(ctx, pat, a_val, batch, f_val, pat->ctl, wrow);
    if (st) return st;
    if (bad_row) return read_ctl(ctx, pat, bad_row, false);
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_pattern_check(tpilu_ctx ctx, tpilu_pattern pat, int64_t* bad_row) {
    if (!ctx) return TPILU_E_INVAL;
    if (!pat) return fail(ctx, TPILU_E_INVAL, "null pattern");
    DeviceGuard dg(ctx->device);
    return read_ctl(ctx, pat, bad_row, true);
}

extern "C" TPILU_API tpilu_status tpilu_apply(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val,
                                              int32_t batch, const double* b, double* y, double* x_out) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (pat->n == 0) return TPILU_OK;
    if (!f_val || !b || !y) return fail(ctx, TPILU_E_INVAL, "null array");
    if (b == y) return fail(ctx, TPILU_E_INVAL, "b and y alias");
    DeviceGuard dg(ctx->device);
    double* x = x_out;
    if (!x) {
        x = pat->grow(pat->ws_x, sizeof(double) * (size_t)pat->n * batch);
        if (!x) return fail(ctx, TPILU_E_NOMEM, "apply workspace");
    }
    trace("apply", pat->n, batch);
    if (batch == 1 && ctx->solver == 2) {
        st = build_dep_positions(ctx, pat);
        if (st) return st;
    }
    return enqueue_apply(ctx, pat, f_val, batch, b, y, x, true, pat->ctl);
}

extern "C" TPILU_API tpilu_status tpilu_apply_noalloc(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val,
                                                      int32_t batch, const double* b, double* y) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (pat->n == 0) return TPILU_OK;
    if (!f_val || !b || !y) return fail(ctx, TPILU_E_INVAL, "null array");
    if (b == y) return fail(ctx, TPILU_E_INVAL, "b and y alias");
    if (pat->n * (int64_t)batch > kScratchDoubles)
        return fail(ctx, TPILU_E_INVAL,
                    "apply_noalloc: n * batch = " + std::to_string(pat->n * (int64_t)batch) +
                        " exceeds the fixed scratch of " + std::to_string(kScratchDoubles) + " values");
    if (!ctx->scratch)
        return fail(ctx, TPILU_E_DEVICE,
                    std::string("apply_noalloc: no scratch address on this device: ") +
                        hipGetErrorString(ctx->scratch_err));
    DeviceGuard dg(ctx->device);
    trace("apply_noalloc", pat->n, batch);
    // x lives in the scratch; the first kernel overwrites the part used with
    // the pending marker, so nothing left by an earlier call is read
    // (no timing events either: creating them is not allowed here)
    return enqueue_apply(ctx, pat, f_val, batch, b, y, ctx->scratch, true, pat->ctl, false);
}

extern "C" TPILU_API tpilu_status tpilu_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val,
                                                int32_t batch, double* g_val) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (batch != 1) return fail(ctx, TPILU_E_INVAL, "incomplete inverses: batch must be 1");
    if (pat->n == 0) return TPILU_OK;
    if (!f_val || !g_val) return fail(ctx, TPILU_E_INVAL, "null array");
    if (f_val == g_val) return fail(ctx, TPILU_E_INVAL, "f_val and g_val alias");
    DeviceGuard dg(ctx->device);
    trace("inverse", pat->n);
    st = build_inverse_sched(ctx, pat);
    if (st) return st;
    hipStream_t s = ctx->stream;
    const InvSched S{pat->iptr, pat->is_s, pat->is_q};
    const int grid = ctx->grid_override ? ctx->grid_override : kInverseWaves;
    const PatDev P = pdev(ctx, pat, RowKernel::Inverse);
    HIPCHK(ctx, launch_fill_pending(g_val, pat->nnz_f, pat->ctl, true, s));
    HIPCHK(ctx, launch_inverse(P, S, f_val, g_val, false, pat->ctl, ctx->spin_limit, grid, s));
    HIPCHK(ctx, launch_fill_pending(nullptr, 0, pat->ctl, false, s));
    HIPCHK(ctx, launch_inverse(P, S, f_val, g_val, true, pat->ctl, ctx->spin_limit, grid, s));
    return read_ctl(ctx, pat, nullptr, false);
}

extern "C" TPILU_API tpilu_status tpilu_apply_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double* g_val,
                                                      int32_t batch, const double* b, double* y, double* x_out) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (batch != 1) return fail(ctx, TPILU_E_INVAL, "incomplete inverses: batch must be 1");
    if (pat->n == 0) return TPILU_OK;
    if (!g_val || !b || !y) return fail(ctx, TPILU_E_INVAL, "null array");
    if (b == y || (x_out && (x_out == b || x_out == y))) return fail(ctx, TPILU_E_INVAL, "vectors alias");
    DeviceGuard dg(ctx->device);
    double* x = x_out;
    if (!x) {
        x = pat->grow(pat->ws_x, sizeof(double) * (size_t)pat->n);
        if (!x) return fail(ctx, TPILU_E_NOMEM, "apply workspace");
    }
    HIPCHK(ctx, launch_apply_inverse(pdev(ctx, pat), g_val, b, x, y, inverse_product_shape(ctx, pat),
                                     ctx->stream));
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_spmv(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val,
                                             const double* x, double* y) {
    tpilu_status st = check_common(ctx, pat, 1);
    if (st) return st;
    DeviceGuard dg(ctx->device);
    HIPCHK(ctx, launch_spmv((int32_t)pat->n, pat->rpA, pat->ciA, a_val, x, nullptr, y, ctx->stream));
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_dot(tpilu_ctx ctx, int64_t n, const double* x, const double* y,
                                            double* result) {
    if (!ctx) return TPILU_E_INVAL;
    if (n < 0 || !result || (n > 0 && (!x || !y))) return fail(ctx, TPILU_E_INVAL, "bad argument");
    DeviceGuard dg(ctx->device);
    Alloc al = ctx_alloc(ctx);
    double* buf = (double*)al.get(sizeof(double) * (kDotBlocks + 1));
    if (!buf) return fail(ctx, TPILU_E_NOMEM, "dot");
    hipError_t e = launch_dot_partial(n, x, y, buf, ctx->stream);
    if (e == hipSuccess) e = launch_dot_final(buf, buf + kDotBlocks, 0, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(result, buf + kDotBlocks, sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    al.put(buf);
    if (e != hipSuccess) return fail(ctx, TPILU_E_DEVICE, hipGetErrorString(e));
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_numeric_critical_path(tpilu_ctx ctx, tpilu_pattern pat, double w_hop,
                                                              double w_step, double* length) {
    tpilu_status st = check_common(ctx, pat, 1);
    if (st) return st;
    if (!length) return fail(ctx, TPILU_E_INVAL, "null output");
    *length = 0.0;
    if (!(w_hop >= 0.0) || !(w_step >= 0.0) || w_hop > 1e12 || w_step > 1e12)
        return fail(ctx, TPILU_E_INVAL, "weights must be finite and >= 0");
    if (pat->n == 0) return TPILU_OK;
    if (!pat->flow)
        return fail(ctx, TPILU_E_INVAL, "critical path: the rows of this pattern do not fit the dataflow kernel");
    DeviceGuard dg(ctx->device);
    TmpBufs T{pat->al, {}};
    double* h = (double*)T.get(sizeof(double) * (size_t)pat->nnz_f);
    unsigned long long* mx = (unsigned long long*)T.get(64);
    if (!h || !mx) return fail(ctx, TPILU_E_NOMEM, "critical path workspace");
    hipStream_t s = ctx->stream;
    const int grid = ctx->grid_override ? ctx->grid_override
                                        : numeric_grid(1, pat->st.max_row, pat->st.max_lrow, true, ctx->num_cu);
    HIPCHK(ctx, launch_fill_pending(h, pat->nnz_f, pat->ctl, true, s));
    HIPCHK(ctx, launch_numeric_hops(pdev(ctx, pat), h, pat->ctl, ctx->spin_limit, grid, pat->st.max_row,
                                    pat->st.max_lrow, w_hop, w_step, s));
    HIPCHK(ctx, launch_fill_i32((int32_t*)mx, 2, 0, s));
    HIPCHK(ctx, launch_max_nonneg(h, pat->nnz_f, mx, s));
    unsigned long long bits = 0ull;
    HIPCHK(ctx, hipMemcpyAsync(&bits, mx, sizeof(bits), hipMemcpyDeviceToHost, s));
    st = read_ctl(ctx, pat, nullptr, false);
    double v = 0.0;
    std::memcpy(&v, &bits, sizeof(v));
    *length = v;
    return st;
}

extern "C" TPILU_API tpilu_status tpilu_handoff_probe(tpilu_ctx ctx, int32_t same_xcd, int32_t rounds,
                                                      double* ns_round_trip) {
    if (!ctx) return TPILU_E_INVAL;
    if (!ns_round_trip || rounds < 1 || rounds > (1 << 24)) return fail(ctx, TPILU_E_INVAL, "bad argument");
    *ns_round_trip = 0.0;
    DeviceGuard dg(ctx->device);
    Alloc al = ctx_alloc(ctx);
    const size_t bytes = probe_buf_bytes();
    void* buf = al.get(bytes);
    if (!buf) return fail(ctx, TPILU_E_NOMEM, "probe buffer");
    std::vector<unsigned char> host(bytes, 0);
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(buf, host.data(), bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_handoff(buf, rounds, same_xcd != 0, ctx->spin_limit, s);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), buf, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    al.put(buf);
    if (e != hipSuccess) return fail(ctx, TPILU_E_DEVICE, std::string("handoff probe: ") + hipGetErrorString(e));
    unsigned long long ticks = 0;
    uint32_t status = 0;
    probe_read(host.data(), &ticks, &status);
    if (status) return fail(ctx, TPILU_E_TIMEOUT, "handoff probe: a wait ran out (no partner on the XCD?)");
    *ns_round_trip = (double)ticks * 1000.0 / (double)ctx->ticks_per_us / (double)rounds;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_givens(tpilu_ctx ctx, int64_t count, const double* a, const double* b,
                                               double* rho, double* c, double* s) {
    if (!ctx) return TPILU_E_INVAL;
    if (count < 0 || (count > 0 && (!a || !b || !rho || !c || !s)))
        return fail(ctx, TPILU_E_INVAL, "bad argument");
    DeviceGuard dg(ctx->device);
    HIPCHK(ctx, launch_givens_batch(count, a, b, rho, c, s, ctx->stream));
    return TPILU_OK;
}

// =====================================================================================
// GMRES
// =====================================================================================
__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

namespace {
// z = M^-1 v: the two substitutions with F, or the two products with G
tpilu_status enqueue_precond(tpilu_ctx ctx, tpilu_pattern pat, const double* m_val, bool inverse,
                             const double* v, double* z, double* t, bool reset) {
    if (!inverse) return enqueue_apply(ctx, pat, m_val, 1, v, z, t, reset, pat->ctl);
    if (reset) HIPCHK(ctx, launch_fill_pending(nullptr, 0, pat->ctl, true, ctx->stream));
    HIPCHK(ctx, launch_apply_inverse(pdev(ctx, pat), m_val, v, t, z, inverse_product_shape(ctx, pat),
                                     ctx->stream));
    return TPILU_OK;
}

tpilu_status gmres_impl(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val, const double* f_val, bool inverse,
                        const double* b, double* x, int32_t restart, int32_t maxit, double rtol, int32_t* iters,
                        double* relres, double* hist) {
    tpilu_status st = check_common(ctx, pat, 1);
    if (st) return st;
    if (!iters || !relres) return fail(ctx, TPILU_E_INVAL, "null host output");
    *iters = 0;
    *relres = 0.0;
    if (restart < 1 || maxit < 0) return fail(ctx, TPILU_E_INVAL, "restart >= 1 and maxit >= 0 required");
    const int64_t n = pat->n;
    if (n == 0) return TPILU_OK;
    if (!a_val || !f_val || !b || !x) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    const int32_t m = restart;
    // workspace (doubles): V (m+1)n | w, z, t, u (n each) | partial 64 | H (m+1)m |
    // cs m | sn m | g m+1 | yv m | scal 8 | hist max(maxit,1) | flags (2 int32)
    const size_t nn = (size_t)n;
    const size_t mh = (size_t)std::max(maxit, 1);
    const size_t o_w = (size_t)(m + 1) * nn;
    const size_t o_partial = o_w + 4 * nn;
    const size_t o_H = o_partial + kDotBlocks;
    const size_t o_cs = o_H + (size_t)(m + 1) * m;
    const size_t o_sn = o_cs + m;
    const size_t o_g = o_sn + m;
    const size_t o_yv = o_g + m + 1;
    const size_t o_scal = o_yv + m;
    const size_t o_hist = o_scal + 8;
    const size_t o_flags = o_hist + mh;
    const size_t doubles = o_flags + 1;
    double* wsd = pat->grow(pat->ws_gm, sizeof(double) * doubles);
    if (!wsd) return fail(ctx, TPILU_E_NOMEM, "gmres workspace");
    double* V = wsd;
    double* w = wsd + o_w;
    double* z = w + nn;
    double* t = z + nn;
    double* u = t + nn;
    double* partial = wsd + o_partial;
    double* H = wsd + o_H;
    double* cs = wsd + o_cs;
    double* sn = wsd + o_sn;
    double* g = wsd + o_g;
    double* yv = wsd + o_yv;
    double* scal = wsd + o_scal;  // [0] bnorm [1] beta [2] final residual norm
    double* dhist = wsd + o_hist;
    int32_t* iflags = reinterpret_cast<int32_t*>(wsd + o_flags);  // [0] iters [1] stop
    const int32_t ni = (int32_t)n;

    HIPCHK(ctx, launch_dot_partial(n, b, b, partial, s));
    HIPCHK(ctx, launch_dot_final(partial, scal + 0, 1, s));
    HIPCHK(ctx, launch_fill_i32(iflags, 2, 0, s));
    double bnorm = 0.0;
    HIPCHK(ctx, hipMemcpyAsync(&bnorm, scal + 0, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, x, n, 0.0);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipStreamSynchronize(s));
        return TPILU_OK;
    }
    const double tol = rtol * bnorm;
    int32_t it_host = 0;
    bool reset = true;
    for (;;) {
        HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, x, b, w, s));
        HIPCHK(ctx, launch_dot_partial(n, w, w, partial, s));
        HIPCHK(ctx, launch_dot_final(partial, scal + 1, 1, s));
        double beta = 0.0;
        HIPCHK(ctx, hipMemcpyAsync(&beta, scal + 1, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (beta <= tol || it_host >= maxit) break;
        HIPCHK(ctx, launch_gm_start(n, partial, scal + 1, g, w, V, s));
        int32_t jj = 0;
        for (int32_t j = 0; j < m; ++j) {
            double* vj = V + (size_t)j * nn;
            st = enqueue_precond(ctx, pat, f_val, inverse, vj, z, t, reset);
            reset = false;
            if (st) return st;
            HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, z, nullptr, w, s));
            for (int32_t i = 0; i <= j; ++i) {
                HIPCHK(ctx, launch_dot_partial(n, w, V + (size_t)i * nn, partial, s));
                HIPCHK(ctx, launch_gm_axpy_h(n, partial, H + (size_t)i * m + j, w, V + (size_t)i * nn, s));
            }
            HIPCHK(ctx, launch_dot_partial(n, w, w, partial, s));
            HIPCHK(ctx, launch_gm_norm_scale(n, partial, H + (size_t)(j + 1) * m + j, w,
                                             V + (size_t)(j + 1) * nn, s));
            HIPCHK(ctx, launch_gm_givens(H, cs, sn, g, m, j, tol, iflags, maxit, dhist, iflags + 1, s));
            int32_t hf[2] = {0, 0};
            uint32_t cst = 0;
            HIPCHK(ctx, hipMemcpyAsync(hf, iflags, sizeof(hf), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipMemcpyAsync(&cst, &pat->ctl->status, sizeof(cst), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            it_host = hf[0];
            jj = j + 1;
            // a preconditioner wait that ran out leaves NaN iterates behind,
            // which no stopping test catches: end the solve at once
            if (cst & kStTimeout) {
                *iters = it_host;
                *relres = NAN;
                return read_ctl(ctx, pat, nullptr, false);
            }
            if (hf[1]) break;
        }
        HIPCHK(ctx, launch_gm_backsub(H, g, yv, m, jj, s));
        HIPCHK(ctx, launch_gm_combine(n, V, yv, jj, u, s));
        st = enqueue_precond(ctx, pat, f_val, inverse, u, z, t, false);
        if (st) return st;
        HIPCHK(ctx, launch_axpy1(n, x, z, s));
    }
    HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, x, b, w, s));
    HIPCHK(ctx, launch_dot_partial(n, w, w, partial, s));
    HIPCHK(ctx, launch_dot_final(partial, scal + 2, 1, s));
    double rn = 0.0;
    HIPCHK(ctx, hipMemcpyAsync(&rn, scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    if (hist && it_host > 0)
        HIPCHK(ctx, hipMemcpyAsync(hist, dhist, sizeof(double) * (size_t)it_host, hipMemcpyDeviceToHost, s));
    st = read_ctl(ctx, pat, nullptr, false);
    *iters = it_host;
    *relres = rn / bnorm;
    if (st) return st;
    if (!(*relres <= rtol)) return fail(ctx, TPILU_E_NOTCONV, "GMRES reached maxit");
    return TPILU_OK;
}
}  // namespace

extern "C" TPILU_API tpilu_status tpilu_gmres(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val,
                                              const double* f_val, const double* b, double* x,
                                              int32_t restart, int32_t maxit, double rtol, int32_t* iters,
                                              double* relres, double* hist) {
    return gmres_impl(ctx, pat, a_val, f_val, false, b, x, restart, maxit, rtol, iters, relres, hist);
}

extern "C" TPILU_API tpilu_status tpilu_gmres_inverse(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val,
                                                      const double* g_val, const double* b, double* x,
                                                      int32_t restart, int32_t maxit, double rtol,
                                                      int32_t* iters, double* relres, double* hist) {
    return gmres_impl(ctx, pat, a_val, g_val, true, b, x, restart, maxit, rtol, iters, relres, hist);
}

// =====================================================================================
// BiCGSTAB
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_bicgstab(tpilu_ctx ctx, tpilu_pattern pat, const double* a_val,
                                                 const double* m_val, int32_t inverse, const double* b, double* x,
                                                 int32_t maxit, double rtol, int32_t* iters, double* relres,
                                                 double* hist) {
    tpilu_status st = check_common(ctx, pat, 1);
    if (st) return st;
    if (!iters || !relres) return fail(ctx, TPILU_E_INVAL, "null host output");
    *iters = 0;
    *relres = 0.0;
    if (maxit < 0) return fail(ctx, TPILU_E_INVAL, "maxit >= 0 required");
    const int64_t n = pat->n;
    if (n == 0) return TPILU_OK;
    if (!a_val || !m_val || !b || !x) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    hipStream_t s = ctx->stream;
    const bool inv = inverse != 0;
    // workspace: r rs p v ph sv sh t tmp (n each) | 3 partial blocks | scalars
    const size_t nn = (size_t)n;
    double* wsd = pat->grow(pat->ws_bi, sizeof(double) * (9 * nn + 3 * kDotBlocks + 16));
    if (!wsd) return fail(ctx, TPILU_E_NOMEM, "bicgstab workspace");
    double *r = wsd, *rs = r + nn, *p = rs + nn, *v = p + nn, *ph = v + nn, *sv = ph + nn, *sh = sv + nn,
           *t = sh + nn, *tmp = t + nn;
    double *pa = tmp + nn, *pb = pa + kDotBlocks, *pc = pb + kDotBlocks, *sc = pc + kDotBlocks;
    const int32_t ni = (int32_t)n;
    auto nrm = [&](const double* vec, double* out_host) -> tpilu_status {
        HIPCHK(ctx, launch_dot_partial(n, vec, vec, pc, s));
        HIPCHK(ctx, launch_dot_final(pc, sc + 8, 1, s));
        HIPCHK(ctx, hipMemcpyAsync(out_host, sc + 8, sizeof(double), hipMemcpyDeviceToHost, s));
        return TPILU_OK;
    };
    double bnorm = 0.0;
    st = nrm(b, &bnorm);
    if (st) return st;
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, x, n, 0.0);
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipStreamSynchronize(s));
        return TPILU_OK;
    }
    const double tol = rtol * bnorm;
    // r = b - A x, rs = r, p = v = 0, rho = alpha = omega = 1
    HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, x, b, r, s));
    HIPCHK(ctx, launch_copy(rs, r, n, s));
    {
        const double init[8] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.0, 0.0};
        HIPCHK(ctx, hipMemcpyAsync(sc, init, sizeof(init), hipMemcpyHostToDevice, s));
    }
    double r0 = 0.0;
    st = nrm(r, &r0);
    if (st) return st;
    HIPCHK(ctx, hipStreamSynchronize(s));
    int32_t it = 0;
    bool breakdown = false, first = true, reset = true;
    if (!(r0 <= tol)) {
        // rho for the first step
        HIPCHK(ctx, launch_dot_partial(n, rs, r, pa, s));
        HIPCHK(ctx, launch_bi(kBiOpRho, n, 0, pa, nullptr, sc, nullptr, nullptr, nullptr, nullptr, nullptr,
                              nullptr, s));
        while (it < maxit) {
            double hs[2] = {0, 0};
            HIPCHK(ctx, hipMemcpyAsync(hs, sc + kBiRho, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            if (hs[0] == 0.0) { breakdown = true; break; }
            HIPCHK(ctx, launch_bi(kBiOpP, n, first ? 1 : 0, nullptr, nullptr, sc, p, nullptr, r, v, nullptr,
                                  nullptr, s));
            first = false;
            st = enqueue_precond(ctx, pat, m_val, inv, p, ph, tmp, reset);
            reset = false;
            if (st) return st;
            HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, ph, nullptr, v, s));
            HIPCHK(ctx, launch_dot_partial(n, rs, v, pa, s));
            HIPCHK(ctx, launch_bi(kBiOpAlpha, n, 0, pa, nullptr, sc, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, s));
            HIPCHK(ctx, launch_bi(kBiOpS, n, 0, nullptr, nullptr, sc, sv, nullptr, r, v, nullptr, nullptr, s));
            double snorm = 0.0, rv = 0.0;
            st = nrm(sv, &snorm);
            if (st) return st;
            uint32_t cst = 0;
            HIPCHK(ctx, hipMemcpyAsync(&rv, sc + kBiRv, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipMemcpyAsync(&cst, &pat->ctl->status, sizeof(cst), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            if (cst & kStTimeout) {  // NaN iterates from here on: stop (see GMRES)
                *iters = it;
                *relres = NAN;
                return read_ctl(ctx, pat, nullptr, false);
            }
            if (rv == 0.0) { breakdown = true; break; }
            if (hist) hist[it] = snorm;
            ++it;
            if (snorm <= tol || it >= maxit) {
                HIPCHK(ctx, launch_bi(kBiOpXHalf, n, 0, nullptr, nullptr, sc, x, nullptr, ph, nullptr, nullptr,
                                      nullptr, s));
                break;
            }
            st = enqueue_precond(ctx, pat, m_val, inv, sv, sh, tmp, false);
            if (st) return st;
            HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, sh, nullptr, t, s));
            HIPCHK(ctx, launch_dot_partial(n, t, sv, pa, s));
            HIPCHK(ctx, launch_dot_partial(n, t, t, pb, s));
            HIPCHK(ctx, launch_bi(kBiOpOmega, n, 0, pa, pb, sc, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, s));
            HIPCHK(ctx, launch_bi(kBiOpXR, n, 0, nullptr, nullptr, sc, x, r, ph, sh, sv, t, s));
            double rnorm = 0.0;
            st = nrm(r, &rnorm);
            if (st) return st;
            // rho for the next step, read with the residual (rho_old <- rho inside)
            HIPCHK(ctx, launch_dot_partial(n, rs, r, pa, s));
            HIPCHK(ctx, launch_bi(kBiOpRho, n, 0, pa, nullptr, sc, nullptr, nullptr, nullptr, nullptr, nullptr,
                                  nullptr, s));
            double so[2] = {0, 0};  // tt, omega
            HIPCHK(ctx, hipMemcpyAsync(&so[0], sc + kBiTt, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipMemcpyAsync(&so[1], sc + kBiOmega, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipMemcpyAsync(&cst, &pat->ctl->status, sizeof(cst), hipMemcpyDeviceToHost, s));
            HIPCHK(ctx, hipStreamSynchronize(s));
            if (cst & kStTimeout) {
                *iters = it;
                *relres = NAN;
                return read_ctl(ctx, pat, nullptr, false);
            }
            if (so[0] == 0.0) { breakdown = true; break; }
            if (hist) hist[it] = rnorm;
            ++it;
            if (rnorm <= tol) break;
            if (so[1] == 0.0) { breakdown = true; break; }
        }
    }
    // true residual
    HIPCHK(ctx, launch_spmv(ni, pat->rpA, pat->ciA, a_val, x, b, tmp, s));
    double rn = 0.0;
    st = nrm(tmp, &rn);
    if (st) return st;
    st = read_ctl(ctx, pat, nullptr, false);
    *iters = it;
    *relres = rn / bnorm;
    if (st) return st;
    if (breakdown) return fail(ctx, TPILU_E_NOTCONV, "BiCGSTAB breakdown");
    if (!(*relres <= rtol)) return fail(ctx, TPILU_E_NOTCONV, "BiCGSTAB reached maxit");
    return TPILU_OK;
}

// =====================================================================================
// adjoints
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_apply_adjoint(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val,
                                                      int32_t batch, const double* x, const double* y,
                                                      const double* ybar, double* bbar, double* fbar) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (pat->n == 0) return TPILU_OK;
    if (!f_val || !x || !y || !ybar || !bbar || !fbar) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    st = build_transposes(ctx, pat);
    if (st) return st;
    hipStream_t s = ctx->stream;
    double* z = pat->grow(pat->ws_z, sizeof(double) * (size_t)pat->n * batch);
    if (!z) return fail(ctx, TPILU_E_NOMEM, "adjoint workspace");
    AdjPat T{pat->tpL, pat->tsL, pat->trL, pat->tpU, pat->tsU, pat->trU, pat->permUT, pat->permLT};
    // transposed sweeps: the DAGs of U~ and L~ reversed, of the same depths
    const int64_t n = pat->n, half_u = pat->nnz_f - (int64_t)pat->st.nnz_l - n, half_l = pat->st.nnz_l;
    const bool xu = batch == 1 && solve_on_xcd(ctx, n, half_u, pat->depth_u);
    const bool xl = batch == 1 && solve_on_xcd(ctx, n, half_l, pat->depth_l);
    auto waves = [&](bool x, int64_t depth) {
        if (ctx->grid_override) return (int)ctx->grid_override;
        if (batch > 1) return (int)kBatchSolveWaves;
        if (!x) return (int)kAdjointWaves;
        return n / std::max<int64_t>(depth, 1) < kNarrowWidth ? (int)kSolveWavesNarrow : (int)kSolveWavesMid;
    };
    HIPCHK(ctx, launch_fill_pending(z, pat->n * batch, pat->ctl, true, s));
    HIPCHK(ctx, launch_adj_solve_u(pdev(ctx, pat), T, f_val, batch, ybar, z, pat->ctl, ctx->spin_limit,
                                   waves(xu, pat->depth_u), xu, s));
    HIPCHK(ctx, launch_fill_pending(bbar, pat->n * batch, pat->ctl, false, s));
    HIPCHK(ctx, launch_adj_solve_l(pdev(ctx, pat), T, f_val, batch, z, bbar, pat->ctl, ctx->spin_limit,
                                   waves(xl, pat->depth_l), xl, s));
    HIPCHK(ctx, launch_adj_fbar(pdev(ctx, pat), batch, x, y, z, bbar, fbar, s));
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_numeric_adjoint(tpilu_ctx ctx, tpilu_pattern pat, const double* f_val,
                                                        int32_t batch, double* fbar, double* abar) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (pat->n == 0) return TPILU_OK;
    if (!f_val || !fbar || !abar) return fail(ctx, TPILU_E_INVAL, "null array");
    DeviceGuard dg(ctx->device);
    st = build_transposes(ctx, pat);
    if (st) return st;
    hipStream_t s = ctx->stream;
    const int64_t nfb = pat->nnz_f * batch;
    double* fin = pat->grow(pat->ws_fin, sizeof(double) * (size_t)nfb);
    double* lbar = pat->grow(pat->ws_lbar, sizeof(double) * (size_t)nfb);
    if (!fin || !lbar) return fail(ctx, TPILU_E_NOMEM, "adjoint workspace");
    if ((size_t)pat->st.max_row * 8 > kBatchLdsLimit)
        return fail(ctx, TPILU_E_INVAL, "adjoint supports rows of at most 8192 entries");
    AdjPat T{pat->tpL, pat->tsL, pat->trL, pat->tpU, pat->tsU, pat->trU, pat->permUT, pat->permLT};
    HIPCHK(ctx, launch_copy(fin, fbar, nfb, s));
    HIPCHK(ctx, launch_fill_pending(fbar, nfb, pat->ctl, true, s));
    HIPCHK(ctx, launch_fill_pending(lbar, nfb, pat->ctl, false, s));
    const int grid = ctx->grid_override ? ctx->grid_override : batch > 1 ? kAdjointBatchWaves : kAdjointWaves;
    HIPCHK(ctx, launch_adj_numeric(pdev(ctx, pat), T, f_val, batch, fin, fbar, lbar, abar, pat->ctl,
                                   ctx->spin_limit, grid, pat->st.max_row, s));
    return TPILU_OK;
}

// =====================================================================================
// batched graph
// =====================================================================================
extern "C" TPILU_API tpilu_status tpilu_batched_graph_create(tpilu_ctx ctx, tpilu_pattern pat,
                                                             const double* a_val, int32_t batch,
                                                             double* f_val, const double* b, double* y,
                                                             tpilu_graph* out) {
    tpilu_status st = check_common(ctx, pat, batch);
    if (st) return st;
    if (!out) return fail(ctx, TPILU_E_INVAL, "null output");
    *out = nullptr;
    if (!a_val || !f_val || !b || !y) return fail(ctx, TPILU_E_INVAL, "null array");
    if (b == y) return fail(ctx, TPILU_E_INVAL, "b and y alias");
    if (pat->n == 0) return fail(ctx, TPILU_E_INVAL, "empty pattern");
    DeviceGuard dg(ctx->device);
    tpilu_graph g = new (std::nothrow) tpilu_graph_s;
    if (!g) return fail(ctx, TPILU_E_NOMEM, "graph handle");
    g->device = ctx->device;
    g->al = ctx_alloc(ctx);
    g->x = (double*)g->al.get(sizeof(double) * (size_t)pat->n * batch);
    g->ctl = (Ctl*)g->al.get(sizeof(Ctl));
    const size_t wb = numeric_wrow_bytes(ctx, pat, batch);
    if (wb) g->wrow = (double*)g->al.get(wb);
    if (!g->x || !g->ctl || (wb && !g->wrow)) {
        delete g;
        return fail(ctx, TPILU_E_NOMEM, "graph workspace");
    }
    {
        Ctl z{};
        z.bad_row = ~0ull;
        hipError_t e = hipMemcpy(g->ctl, &z, sizeof(Ctl), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            delete g;
            return fail(ctx, TPILU_E_DEVICE, std::string("graph control block: ") + hipGetErrorString(e));
        }
    }
    hipStream_t cap = nullptr;
    {
        hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete g;
            return fail(ctx, TPILU_E_DEVICE, std::string("capture stream: ") + hipGetErrorString(e));
        }
    }
    hipStream_t saved = ctx->stream;
    ctx->stream = cap;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // batches: the forward substitution runs inside the factorization
        const bool fused = batch > 1;
        st = enqueue_numeric(ctx, pat, a_val, batch, f_val, g->ctl, g->wrow, fused ? b : nullptr,
                             fused ? g->x : nullptr);
        if (st == TPILU_OK) st = enqueue_apply(ctx, pat, f_val, batch, b, y, g->x, false, g->ctl, true, !fused);
        e = hipStreamEndCapture(cap, &graph);
    }
    ctx->stream = saved;
    (void)hipStreamDestroy(cap);
    g->graph = graph;
    if (st) {
        delete g;
        return st;
    }
    if (e != hipSuccess) {
        delete g;
        return fail(ctx, TPILU_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        g->exec = nullptr;
        delete g;
        return fail(ctx, TPILU_E_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
    }
    *out = g;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_batched_graph_launch(tpilu_graph g, void* hip_stream) {
    if (!g) return TPILU_E_INVAL;
    DeviceGuard dg(g->device);
    if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(hip_stream)) != hipSuccess) return TPILU_E_DEVICE;
    return TPILU_OK;
}

extern "C" TPILU_API tpilu_status tpilu_batched_graph_check(tpilu_graph g, void* hip_stream, int64_t* bad_row) {
    if (!g) return TPILU_E_INVAL;
    DeviceGuard dg(g->device);
    if (hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) != hipSuccess) return TPILU_E_DEVICE;
    Ctl h{};
    if (hipMemcpy(&h, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost) != hipSuccess) return TPILU_E_DEVICE;
    // the status words are reset by the graph's first kernel on every launch
    const int64_t bad = h.bad_row == ~0ull ? -1 : (int64_t)h.bad_row;
    if (bad_row) *bad_row = bad;
    if (h.status & kStTimeout) return TPILU_E_TIMEOUT;
    if (h.status & kStReservedNaN) return TPILU_E_INVAL;
    if (bad >= 0) return TPILU_E_ZEROPIVOT;
    return TPILU_OK;
}

extern "C" TPILU_API void tpilu_batched_graph_destroy(tpilu_graph g) {
    if (!g) return;
    DeviceGuard dg(g->device);
    delete g;
}
