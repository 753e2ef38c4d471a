// Host-side sanitizer run of the library (test infrastructure).  Built by
// tests/host_sanitizer_build.py together with a copy of the library whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer (the GPU
// code is the normal build), and linked with the oracle.  It calls every
// entry point of include/tpilu.h through the C ABI on a small 2-D
// convection-diffusion problem, checks the results against the oracle bit
// for bit where the oracle defines them, drives the error paths (null and
// malformed arguments, oversize requests, a failing allocator, the
// watchdog), and checks that every device allocation made through the
// allocator callback is released.  A memory error or undefined behaviour in
// the host code stops the run; exit status 0 means every check passed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "tpilu.h"

extern "C" {
typedef struct {
    int64_t n, nnz;
    int64_t* rowptr;
    int32_t* col;
    int32_t* lev;
} orc_pattern;
int orc_symbolic(int64_t n, const int64_t* rp, const int32_t* ci, int32_t k, orc_pattern* out);
void orc_pattern_free(orc_pattern* p);
int orc_numeric(int64_t n, const int64_t* rpA, const int32_t* ciA, const double* vA, const int64_t* rpF,
                const int32_t* ciF, double* vF, int64_t* bad_row);
int orc_apply(int64_t n, const int64_t* rpF, const int32_t* ciF, const double* vF, const double* p, double* x,
              double* y);
int orc_gmres(int64_t n, const int64_t* rpA, const int32_t* ciA, const double* vA, const int64_t* rpF,
              const int32_t* ciF, const double* vF, const double* b, double* x, int32_t m, int32_t maxit,
              double rtol, int32_t* iters_out, double* relres_out, double* hist);
int orc_inverse(int64_t n, const int64_t* rpF, const int32_t* ciF, const double* vF, double* vG);
}

static int failures = 0;
#define CHECK(cond, ...)                                                          \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "driver: check failed (line %d): ", __LINE__);   \
            std::fprintf(stderr, __VA_ARGS__);                                    \
            std::fprintf(stderr, "\n");                                           \
            ++failures;                                                           \
        }                                                                         \
    } while (0)

// allocator callback that records every live allocation; `fail_after` >= 0
// makes the allocation after that many succeed return NULL
struct Tracker {
    std::map<void*, size_t> live;
    long calls = 0;
    long fail_after = -1;
};
static void* t_alloc(size_t bytes, void* user) {
    Tracker* t = static_cast<Tracker*>(user);
    if (t->fail_after >= 0 && t->calls++ >= t->fail_after) return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    t->live[p] = bytes;
    return p;
}
static void t_free(void* p, void* user) {
    Tracker* t = static_cast<Tracker*>(user);
    auto it = t->live.find(p);
    if (it == t->live.end()) {
        std::fprintf(stderr, "driver: free of a pointer the allocator never gave out\n");
        ++failures;
        return;
    }
    t->live.erase(it);
    (void)hipFree(p);
}

template <typename T>
struct Dev {
    T* p = nullptr;
    size_t n = 0;
    explicit Dev(size_t count) : n(count) {
        if (hipMalloc(&p, sizeof(T) * (count ? count : 1)) != hipSuccess) std::abort();
    }
    Dev(const std::vector<T>& h) : Dev(h.size()) { up(h); }
    ~Dev() { (void)hipFree(p); }
    void up(const std::vector<T>& h) { (void)hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice); }
    std::vector<T> down() const {
        std::vector<T> h(n);
        (void)hipMemcpy(h.data(), p, sizeof(T) * n, hipMemcpyDeviceToHost);
        return h;
    }
};

static bool same_bits(const std::vector<double>& a, const std::vector<double>& b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i) {
        if (std::isnan(a[i]) && std::isnan(b[i])) continue;
        if (std::memcmp(&a[i], &b[i], sizeof(double)) != 0) return false;
    }
    return true;
}

// 2-D convection-diffusion, 5-point, m x m, natural order
static void conv_diff(int m, double bx, double by, std::vector<int64_t>& rp, std::vector<int32_t>& ci,
                      std::vector<double>& v) {
    const int n = m * m;
    const double h = 1.0 / (m + 1);
    rp.assign(1, 0);
    ci.clear();
    v.clear();
    for (int i = 0; i < n; ++i) {
        const int x = i % m, y = i / m;
        auto put = [&](int j, double a) {
            ci.push_back(j);
            v.push_back(a);
        };
        if (y > 0) put(i - m, -1.0 - by * h / 2);
        if (x > 0) put(i - 1, -1.0 - bx * h / 2);
        put(i, 4.0);
        if (x < m - 1) put(i + 1, -1.0 + bx * h / 2);
        if (y < m - 1) put(i + m, -1.0 + by * h / 2);
        rp.push_back((int64_t)ci.size());
    }
}

static void run(Tracker& tr) {
    tpilu_ctx ctx = nullptr;
    CHECK(tpilu_ctx_create(0, nullptr, t_alloc, t_free, &tr, &ctx) == TPILU_OK, "ctx_create");
    if (!ctx) return;
    const int m = 40, n = m * m;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> va;
    conv_diff(m, 30.0, -20.0, rp, ci, va);
    const int64_t nnz = (int64_t)ci.size();
    Dev<int64_t> drp(rp);
    Dev<int32_t> dci(ci);
    Dev<double> dva(va);
    std::vector<double> b(n);
    for (int i = 0; i < n; ++i) b[i] = std::sin(0.37 * i) + 0.5;
    Dev<double> db(b);
    for (int k = 0; k <= 3; ++k) {
        tpilu_pattern pat = nullptr;
        CHECK(tpilu_symbolic(ctx, n, nnz, drp.p, dci.p, k, &pat) == TPILU_OK, "symbolic k=%d: %s", k,
              tpilu_last_error(ctx));
        if (!pat) continue;
        tpilu_pattern_info_t info;
        CHECK(tpilu_pattern_info(pat, &info) == TPILU_OK, "pattern_info");
        orc_pattern op;
        CHECK(orc_symbolic(n, rp.data(), ci.data(), k, &op) == 0, "oracle symbolic");
        CHECK(info.nnz_f == op.nnz, "nnz_f %lld vs %lld", (long long)info.nnz_f, (long long)op.nnz);
        Dev<int64_t> erp(n + 1);
        Dev<int32_t> eci(info.nnz_f), edg(n), ea2f(nnz);
        Dev<uint8_t> elv(info.nnz_f);
        CHECK(tpilu_pattern_export(ctx, pat, erp.p, eci.p, edg.p, elv.p, ea2f.p) == TPILU_OK, "export");
        const std::vector<int64_t> hrp = erp.down();
        const std::vector<int32_t> hci = eci.down();
        CHECK(std::memcmp(hrp.data(), op.rowptr, sizeof(int64_t) * (n + 1)) == 0, "rowptr k=%d", k);
        CHECK(std::memcmp(hci.data(), op.col, sizeof(int32_t) * op.nnz) == 0, "col k=%d", k);
        // factor, solves, inverses, Krylov, against the oracle
        std::vector<double> fref(op.nnz), xr(n), yr(n), gref(op.nnz);
        int64_t bad = 0;
        CHECK(orc_numeric(n, rp.data(), ci.data(), va.data(), op.rowptr, op.col, fref.data(), &bad) == 0, "orc");
        CHECK(orc_apply(n, op.rowptr, op.col, fref.data(), b.data(), xr.data(), yr.data()) == 0, "orc apply");
        CHECK(orc_inverse(n, op.rowptr, op.col, fref.data(), gref.data()) == 0, "orc inverse");
        Dev<double> df(op.nnz), dy(n), dx(n), dg(op.nnz);
        int64_t badg = 7;
        CHECK(tpilu_numeric(ctx, pat, dva.p, 1, df.p, &badg) == TPILU_OK && badg == -1, "numeric");
        CHECK(same_bits(df.down(), fref), "F bits k=%d", k);
        CHECK(tpilu_apply(ctx, pat, df.p, 1, db.p, dy.p, dx.p) == TPILU_OK, "apply");
        CHECK(same_bits(dy.down(), yr) && same_bits(dx.down(), xr), "y bits k=%d", k);
        CHECK(tpilu_apply_noalloc(ctx, pat, df.p, 1, db.p, dy.p) == TPILU_OK, "apply_noalloc");
        CHECK(same_bits(dy.down(), yr), "noalloc y bits k=%d", k);
        CHECK(tpilu_inverse(ctx, pat, df.p, 1, dg.p) == TPILU_OK, "inverse");
        CHECK(same_bits(dg.down(), gref), "inverse bits k=%d", k);
        CHECK(tpilu_apply_inverse(ctx, pat, dg.p, 1, db.p, dy.p, nullptr) == TPILU_OK, "apply_inverse");
        for (int mode = 1; mode <= 3; ++mode) {
            CHECK(tpilu_ctx_set_solver(ctx, mode) == TPILU_OK, "set_solver");
            CHECK(tpilu_apply(ctx, pat, df.p, 1, db.p, dy.p, nullptr) == TPILU_OK, "apply mode %d", mode);
            CHECK(same_bits(dy.down(), yr), "y bits mode %d k=%d", mode, k);
        }
        CHECK(tpilu_ctx_set_solver(ctx, 0) == TPILU_OK, "set_solver");
        {
            std::vector<double> xo(n, 0.0), ho(200);
            int32_t it = 0, itg = 0;
            double rr = 0, rrg = 0;
            const int so = orc_gmres(n, rp.data(), ci.data(), va.data(), op.rowptr, op.col, fref.data(),
                                     b.data(), xo.data(), 30, 200, 1e-8, &it, &rr, ho.data());
            Dev<double> xg(std::vector<double>(n, 0.0));
            std::vector<double> hg(200);
            const tpilu_status sg = tpilu_gmres(ctx, pat, dva.p, df.p, db.p, xg.p, 30, 200, 1e-8, &itg, &rrg,
                                                hg.data());
            CHECK(so == 0 && sg == TPILU_OK && it == itg, "gmres %d %d iters %d %d", so, (int)sg, it, itg);
            CHECK(same_bits(xg.down(), xo), "gmres x bits k=%d", k);
            Dev<double> xb(std::vector<double>(n, 0.0));
            const tpilu_status sb = tpilu_bicgstab(ctx, pat, dva.p, df.p, 0, db.p, xb.p, 200, 1e-8, &itg, &rrg,
                                                   hg.data());
            CHECK(sb == TPILU_OK || sb == TPILU_E_NOTCONV, "bicgstab %d", (int)sb);
            Dev<double> xi(std::vector<double>(n, 0.0));
            const tpilu_status si = tpilu_gmres_inverse(ctx, pat, dva.p, dg.p, db.p, xi.p, 30, 200, 1e-8, &itg,
                                                        &rrg, hg.data());
            CHECK(si == TPILU_OK || si == TPILU_E_NOTCONV, "gmres_inverse %d", (int)si);
        }
        // building blocks
        {
            double d = 0;
            CHECK(tpilu_spmv(ctx, pat, dva.p, db.p, dy.p) == TPILU_OK, "spmv");
            CHECK(tpilu_dot(ctx, n, db.p, db.p, &d) == TPILU_OK && d > 0, "dot");
            double len = 0;
            CHECK(tpilu_numeric_critical_path(ctx, pat, 1.0, 0.0, &len) == TPILU_OK && len >= 0, "critical path");
        }
        // batches: three instances, eager and in a graph, and reverse mode
        {
            const int B = 3;
            std::vector<double> vb((size_t)nnz * B), bb((size_t)n * B);
            for (int64_t p = 0; p < nnz; ++p)
                for (int i = 0; i < B; ++i) vb[(size_t)p * B + i] = va[p] * (1.0 + 0.25 * i);
            for (int r = 0; r < n; ++r)
                for (int i = 0; i < B; ++i) bb[(size_t)r * B + i] = b[r] - i;
            Dev<double> dvb(vb), dbb(bb), dfb((size_t)op.nnz * B), dyb((size_t)n * B), dxb((size_t)n * B);
            CHECK(tpilu_numeric(ctx, pat, dvb.p, B, dfb.p, &badg) == TPILU_OK, "batched numeric");
            CHECK(tpilu_apply(ctx, pat, dfb.p, B, dbb.p, dyb.p, dxb.p) == TPILU_OK, "batched apply");
            const std::vector<double> fb = dfb.down(), yb = dyb.down();
            for (int i = 0; i < B; ++i) {
                std::vector<double> vi(nnz), fi(op.nnz), fr(op.nnz), bi(n), xi(n), yi(n), yg(n);
                for (int64_t p = 0; p < nnz; ++p) vi[p] = vb[(size_t)p * B + i];
                for (int64_t p = 0; p < op.nnz; ++p) fi[p] = fb[(size_t)p * B + i];
                for (int r = 0; r < n; ++r) {
                    bi[r] = bb[(size_t)r * B + i];
                    yg[r] = yb[(size_t)r * B + i];
                }
                orc_numeric(n, rp.data(), ci.data(), vi.data(), op.rowptr, op.col, fr.data(), &bad);
                orc_apply(n, op.rowptr, op.col, fr.data(), bi.data(), xi.data(), yi.data());
                CHECK(same_bits(fi, fr) && same_bits(yg, yi), "batched instance %d k=%d", i, k);
            }
            tpilu_graph gr = nullptr;
            Dev<double> gf((size_t)op.nnz * B), gy((size_t)n * B);
            CHECK(tpilu_batched_graph_create(ctx, pat, dvb.p, B, gf.p, dbb.p, gy.p, &gr) == TPILU_OK, "graph");
            if (gr) {
                CHECK(tpilu_batched_graph_launch(gr, nullptr) == TPILU_OK, "graph launch");
                int64_t gb = 0;
                CHECK(tpilu_batched_graph_check(gr, nullptr, &gb) == TPILU_OK && gb == -1, "graph check");
                CHECK(same_bits(gf.down(), fb) && same_bits(gy.down(), yb), "graph bits k=%d", k);
                tpilu_batched_graph_destroy(gr);
            }
            Dev<double> ybar(bb), bbar((size_t)n * B), fbar((size_t)op.nnz * B), abar((size_t)nnz * B);
            CHECK(tpilu_apply_adjoint(ctx, pat, dfb.p, B, dxb.p, dyb.p, ybar.p, bbar.p, fbar.p) == TPILU_OK,
                  "apply_adjoint");
            CHECK(tpilu_numeric_adjoint(ctx, pat, dfb.p, B, fbar.p, abar.p) == TPILU_OK, "numeric_adjoint");
        }
        // error paths on this pattern
        CHECK(tpilu_numeric(ctx, pat, nullptr, 1, df.p, nullptr) == TPILU_E_INVAL, "null a_val accepted");
        CHECK(tpilu_numeric(ctx, pat, dva.p, 0, df.p, nullptr) == TPILU_E_INVAL, "batch 0 accepted");
        CHECK(tpilu_apply(ctx, pat, df.p, 1, db.p, nullptr, nullptr) == TPILU_E_INVAL, "null y accepted");
        CHECK(tpilu_apply_noalloc(ctx, pat, df.p, 1 << 20, db.p, dy.p) == TPILU_E_INVAL, "oversize noalloc");
        orc_pattern_free(&op);
        tpilu_pattern_destroy(pat);
    }
    // the watchdog, forced from the host: a row never published
    {
        tpilu_pattern pat = nullptr;
        CHECK(tpilu_symbolic(ctx, n, nnz, drp.p, dci.p, 1, &pat) == TPILU_OK, "symbolic");
        tpilu_pattern_info_t info;
        tpilu_pattern_info(pat, &info);
        Dev<double> df(info.nnz_f);
        CHECK(tpilu_ctx_set_watchdog(ctx, 20000, 100) == TPILU_OK, "set_watchdog");
        int64_t badg = 0;
        CHECK(tpilu_numeric(ctx, pat, dva.p, 1, df.p, &badg) == TPILU_E_TIMEOUT, "watchdog did not fire");
        CHECK(tpilu_ctx_set_watchdog(ctx, 0, -1) == TPILU_OK, "set_watchdog");
        CHECK(tpilu_numeric(ctx, pat, dva.p, 1, df.p, &badg) == TPILU_OK, "no recovery after the watchdog");
        tpilu_pattern_destroy(pat);
    }
    // malformed structure and argument errors
    {
        std::vector<int64_t> brp = {0, 2, 3};
        std::vector<int32_t> bci = {1, 0, 1};  // unsorted row 0
        Dev<int64_t> dbrp(brp);
        Dev<int32_t> dbci(bci);
        tpilu_pattern pat = nullptr;
        CHECK(tpilu_symbolic(ctx, 2, 3, dbrp.p, dbci.p, 1, &pat) == TPILU_E_INVAL && !pat, "bad CSR accepted");
        CHECK(tpilu_symbolic(ctx, n, nnz, drp.p, dci.p, -1, &pat) == TPILU_E_INVAL, "k < 0 accepted");
        CHECK(tpilu_ctx_set_grid(ctx, -1) == TPILU_E_INVAL, "grid < 0 accepted");
        CHECK(tpilu_ctx_set_group(ctx, 65) == TPILU_E_INVAL, "group 65 accepted");
        CHECK(tpilu_numeric(nullptr, nullptr, nullptr, 1, nullptr, nullptr) == TPILU_E_INVAL, "null ctx");
        CHECK(std::strlen(tpilu_status_string(TPILU_E_TIMEOUT)) > 0, "status string");
        double rho = 0, c = 0, s = 0;
        Dev<double> ga(std::vector<double>{3.0}), gb(std::vector<double>{4.0}), gr(1), gc(1), gs(1);
        CHECK(tpilu_givens(ctx, 1, ga.p, gb.p, gr.p, gc.p, gs.p) == TPILU_OK, "givens");
        rho = gr.down()[0];
        c = gc.down()[0];
        s = gs.down()[0];
        CHECK(rho == 5.0 && c == 0.6 && s == 0.8, "givens 3,4 -> %g %g %g", rho, c, s);
    }
    tpilu_ctx_destroy(ctx);
}

int main() {
    Tracker tr;
    run(tr);
    CHECK(tr.live.empty(), "%zu device allocations not released", tr.live.size());
    // a failing allocator: every call reports E_NOMEM, nothing leaks
    for (long fail_after = 0; fail_after < 6; ++fail_after) {
        Tracker t2;
        t2.fail_after = fail_after;
        tpilu_ctx ctx = nullptr;
        if (tpilu_ctx_create(0, nullptr, t_alloc, t_free, &t2, &ctx) != TPILU_OK) {
            ++failures;
            continue;
        }
        std::vector<int64_t> rp;
        std::vector<int32_t> ci;
        std::vector<double> va;
        conv_diff(16, 1.0, 1.0, rp, ci, va);
        Dev<int64_t> drp(rp);
        Dev<int32_t> dci(ci);
        tpilu_pattern pat = nullptr;
        const tpilu_status st = tpilu_symbolic(ctx, 256, (int64_t)ci.size(), drp.p, dci.p, 1, &pat);
        CHECK(st == TPILU_E_NOMEM || st == TPILU_OK, "symbolic under a failing allocator: %d", (int)st);
        if (pat) tpilu_pattern_destroy(pat);
        tpilu_ctx_destroy(ctx);
        CHECK(t2.live.empty(), "failing allocator (after %ld): %zu allocations not released", fail_after,
              t2.live.size());
    }
    if (failures) {
        std::fprintf(stderr, "driver: %d checks failed\n", failures);
        return 1;
    }
    std::printf("host sanitizer driver: all checks passed\n");
    return 0;
}
