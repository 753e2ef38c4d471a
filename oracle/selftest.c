/* Self-test driver of the oracle, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py (test
 * infrastructure, like the oracle itself).  It compiles the oracle into the
 * same unit and runs every exported routine over seeded random patterns of
 * 0 to 60 rows and every level limit from 0 to complete fill, so that an out
 * of bounds access, a use after free, a leak or undefined arithmetic
 * anywhere in the oracle stops the run.  It also checks results that hold
 * whatever the rounding, with tolerances where rounding enters:
 *   - the pattern holds A and every diagonal, rows are sorted, levels are
 *     within [0, k], and with k = n it is the fill of dense boolean
 *     elimination (the complete LU pattern, Def. 2.3 with no limit);
 *   - with complete fill the factor is the exact LU: L U reproduces A and
 *     the substitutions solve A y = b (Eq. 1);
 *   - when the complete fill is the whole matrix, the incomplete inverses are
 *     the exact inverses of L and U, so their products give the same y
 *     (Sec. 3.5; a sparser complete fill does not hold those inverses);
 *   - GMRES and BiCGSTAB report convergence with a residual at the tolerance;
 *   - single rows of the elimination equal the whole one bit for bit;
 *   - the reverse sweeps satisfy the dot-product identity of the adjoint.
 * Exit status 0 when every check passes. */
#include "ilu_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void)
{
    /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double urand(void) { return (double)(rnd() >> 11) * (1.0 / 9007199254740992.0); }

static int failures = 0;
static int exact_inverse_checks = 0;
#define CHECK(cond, ...)                                                        \
    do {                                                                        \
        if (!(cond)) {                                                          \
            fprintf(stderr, "selftest: check failed (%s:%d): ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                                       \
            fprintf(stderr, "\n");                                              \
            ++failures;                                                         \
        }                                                                       \
    } while (0)

/* random pattern with every diagonal, diagonally dominant values */
static void random_matrix(int64_t n, double density, int64_t **rp_out, int32_t **ci_out, double **v_out)
{
    int64_t *rp = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *ci = (int32_t *)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(int32_t));
    double *v = (double *)malloc((size_t)(n * n > 0 ? n * n : 1) * sizeof(double));
    rp[0] = 0;
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i) {
        double rowsum = 0.0;
        int64_t dpos = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i || urand() < density) {
                ci[e] = (int32_t)j;
                v[e] = 2.0 * urand() - 1.0;
                if (j == i) dpos = e;
                else rowsum += fabs(v[e]);
                ++e;
            }
        }
        v[dpos] = rowsum + 1.0 + urand();
        rp[i + 1] = e;
    }
    *rp_out = rp;
    *ci_out = ci;
    *v_out = v;
}

static double *dense_of(int64_t n, const int64_t *rp, const int32_t *ci, const double *v)
{
    double *d = (double *)calloc((size_t)(n * n > 0 ? n * n : 1), sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) d[i * n + ci[e]] = v ? v[e] : 1.0;
    return d;
}

static void check_pattern(int64_t n, const int64_t *rp, const int32_t *ci, int32_t k, const orc_pattern *P)
{
    CHECK(P->n == n, "pattern size");
    for (int64_t i = 0; i < n; ++i) {
        int have_diag = 0;
        for (int64_t e = P->rowptr[i]; e < P->rowptr[i + 1]; ++e) {
            if (e > P->rowptr[i]) CHECK(P->col[e - 1] < P->col[e], "row %lld not sorted", (long long)i);
            CHECK(P->lev[e] >= 0 && P->lev[e] <= k, "level out of range");
            have_diag |= P->col[e] == i;
        }
        CHECK(have_diag, "row %lld has no diagonal", (long long)i);
        /* A's entries are in, at level 0 */
        for (int64_t a = rp[i]; a < rp[i + 1]; ++a) {
            int found = 0;
            for (int64_t e = P->rowptr[i]; e < P->rowptr[i + 1]; ++e)
                if (P->col[e] == ci[a]) found = P->lev[e] == 0;
            CHECK(found, "entry of A missing or not at level 0");
        }
    }
    if (k >= n) {
        /* complete fill: the structure of dense boolean elimination */
        char *s = (char *)calloc((size_t)(n * n > 0 ? n * n : 1), 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s[i * n + ci[e]] = 1;
        for (int64_t h = 0; h < n; ++h)
            for (int64_t i = h + 1; i < n; ++i)
                if (s[i * n + h])
                    for (int64_t t = h + 1; t < n; ++t)
                        if (s[h * n + t]) s[i * n + t] = 1;
        int64_t cnt = 0;
        for (int64_t i = 0; i < n * n; ++i) cnt += s[i];
        CHECK(cnt == (n > 0 ? P->rowptr[n] : 0), "complete fill count %lld vs %lld", (long long)cnt,
              (long long)(n > 0 ? P->rowptr[n] : 0));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = P->rowptr[i]; e < P->rowptr[i + 1]; ++e)
                CHECK(s[i * n + P->col[e]], "position outside the complete fill");
        free(s);
    }
}

static void run_case(int64_t n, double density, int32_t k)
{
    int64_t *rp;
    int32_t *ci;
    double *v;
    random_matrix(n, density, &rp, &ci, &v);
    CHECK(orc_validate(n, rp, ci) == ORC_OK, "valid CSR refused");
    orc_pattern P;
    int st = orc_symbolic(n, rp, ci, k, &P);
    CHECK(st == ORC_OK, "symbolic status %d", st);
    if (st != ORC_OK) goto done_a;
    check_pattern(n, rp, ci, k, &P);
    const int64_t nnzf = n > 0 ? P.rowptr[n] : 0;
    double *f = (double *)malloc((size_t)(nnzf > 0 ? nnzf : 1) * sizeof(double));
    int64_t bad = 0;
    st = orc_numeric(n, rp, ci, v, P.rowptr, P.col, f, &bad);
    CHECK(st == ORC_OK && bad == -1, "numeric status %d bad %lld", st, (long long)bad);
    /* the fused update: the same pattern, finite values, within rounding of
       the default rounding's factor */
    {
        double *ff = (double *)malloc((size_t)(nnzf > 0 ? nnzf : 1) * sizeof(double));
        int64_t badf = 0;
        st = orc_numeric_fused(n, rp, ci, v, P.rowptr, P.col, ff, &badf);
        CHECK(st == ORC_OK && badf == -1, "fused numeric status %d bad %lld", st, (long long)badf);
        for (int64_t e = 0; e < nnzf; ++e)
            CHECK(isfinite(ff[e]) && fabs(ff[e] - f[e]) <= 1e-9 * (1.0 + fabs(f[e])), "fused entry %lld", (long long)e);
        free(ff);
    }
    double *b = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *x = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *y = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *r = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) b[i] = 2.0 * urand() - 1.0;
    CHECK(orc_apply(n, P.rowptr, P.col, f, b, x, y) == ORC_OK, "apply");
    /* single rows of the elimination */
    if (n > 0) {
        int64_t rows[3] = {0, n / 2, n - 1};
        int64_t tot = 0;
        for (int q = 0; q < 3; ++q) tot += P.rowptr[rows[q] + 1] - P.rowptr[rows[q]];
        double *out = (double *)malloc((size_t)tot * sizeof(double));
        CHECK(orc_numeric_rows(n, rp, ci, v, P.rowptr, P.col, f, 3, rows, out) == ORC_OK, "numeric_rows");
        int64_t o = 0;
        for (int q = 0; q < 3; ++q)
            for (int64_t e = P.rowptr[rows[q]]; e < P.rowptr[rows[q] + 1]; ++e, ++o)
                CHECK(memcmp(&out[o], &f[e], sizeof(double)) == 0, "row %lld differs", (long long)rows[q]);
        free(out);
    }
    /* incomplete inverses and their products */
    double *gv = (double *)malloc((size_t)(nnzf > 0 ? nnzf : 1) * sizeof(double));
    double *x2 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *y2 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    CHECK(orc_inverse(n, P.rowptr, P.col, f, gv) == ORC_OK, "inverse");
    CHECK(orc_apply_inverse(n, P.rowptr, P.col, gv, b, x2, y2) == ORC_OK, "apply_inverse");
    if (k >= n && n > 0) {
        /* exact LU: A y = b, and the inverses give the same y */
        orc_spmv(n, rp, ci, v, y, r);
        double err = 0.0, scale = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            err = fmax(err, fabs(r[i] - b[i]));
            scale = fmax(scale, fabs(b[i]));
        }
        CHECK(err <= 1e-10 * scale, "complete LU does not solve A y = b: %g", err);
        if (nnzf == n * n) {
            ++exact_inverse_checks;
            double d = 0.0, s = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                d = fmax(d, fabs(y2[i] - y[i]));
                s = fmax(s, fabs(y[i]));
            }
            CHECK(d <= 1e-10 * s, "inverse products differ from the substitutions: %g", d);
        }
        /* L U = A on every stored position */
        double *L = (double *)calloc((size_t)(n * n), sizeof(double));
        double *U = (double *)calloc((size_t)(n * n), sizeof(double));
        for (int64_t i = 0; i < n; ++i) {
            L[i * n + i] = 1.0;
            for (int64_t e = P.rowptr[i]; e < P.rowptr[i + 1]; ++e) {
                if (P.col[e] < i) L[i * n + P.col[e]] = f[e];
                else U[i * n + P.col[e]] = f[e];
            }
        }
        double *Ad = dense_of(n, rp, ci, v);
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) {
                double s2 = 0.0;
                for (int64_t h = 0; h < n; ++h) s2 += L[i * n + h] * U[h * n + j];
                worst = fmax(worst, fabs(s2 - Ad[i * n + j]));
            }
        CHECK(worst <= 1e-10 * (double)n, "L U differs from A by %g", worst);
        free(L);
        free(U);
        free(Ad);
    }
    /* Krylov drivers */
    if (n > 0) {
        const int32_t maxit = (int32_t)(10 * n + 10);
        double *hist = (double *)malloc((size_t)maxit * sizeof(double));
        int32_t it = 0;
        double rr = 0.0;
        memset(x, 0, (size_t)n * sizeof(double));
        st = orc_gmres(n, rp, ci, v, P.rowptr, P.col, f, b, x, 5, maxit, 1e-10, &it, &rr, hist);
        CHECK(st == ORC_OK && rr <= 1e-10, "gmres status %d relres %g", st, rr);
        memset(x, 0, (size_t)n * sizeof(double));
        st = orc_gmres_inverse(n, rp, ci, v, P.rowptr, P.col, gv, b, x, 5, maxit, 1e-10, &it, &rr, hist);
        CHECK(st == ORC_OK && rr <= 1e-10, "gmres (inverses) status %d relres %g", st, rr);
        for (int inv = 0; inv < 2; ++inv) {
            memset(x, 0, (size_t)n * sizeof(double));
            st = orc_bicgstab(n, rp, ci, v, P.rowptr, P.col, inv ? gv : f, inv, b, x, maxit, 1e-10, &it, &rr,
                              hist);
            /* a breakdown (reported as not converged) is a legitimate outcome
               of BiCGSTAB; a converged run must meet the tolerance */
            CHECK(st == ORC_OK || st == ORC_ENOTCONV, "bicgstab status %d", st);
            if (st == ORC_OK) CHECK(rr <= 1e-10, "bicgstab relres %g", rr);
        }
        free(hist);
        /* reverse sweeps: for y = M^-1 b, <ybar, dy> = <bbar, db> for any db */
        double *ybar = (double *)malloc((size_t)n * sizeof(double));
        double *bbar = (double *)malloc((size_t)n * sizeof(double));
        double *Fbar = (double *)malloc((size_t)(nnzf > 0 ? nnzf : 1) * sizeof(double));
        double *abar = (double *)malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(double));
        for (int64_t i = 0; i < n; ++i) ybar[i] = 2.0 * urand() - 1.0;
        CHECK(orc_apply(n, P.rowptr, P.col, f, b, x, y) == ORC_OK, "apply");
        CHECK(orc_apply_adjoint(n, P.rowptr, P.col, f, x, y, ybar, bbar, Fbar) == ORC_OK, "apply_adjoint");
        CHECK(orc_numeric_adjoint(n, rp, ci, P.rowptr, P.col, f, Fbar, abar) == ORC_OK, "numeric_adjoint");
        double *db = (double *)malloc((size_t)n * sizeof(double));
        for (int64_t i = 0; i < n; ++i) db[i] = 2.0 * urand() - 1.0;
        CHECK(orc_apply(n, P.rowptr, P.col, f, db, x2, y2) == ORC_OK, "apply");
        double lhs = 0.0, rhs = 0.0, mag = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            lhs += ybar[i] * y2[i];
            rhs += bbar[i] * db[i];
            mag += fabs(ybar[i] * y2[i]) + fabs(bbar[i] * db[i]);
        }
        CHECK(fabs(lhs - rhs) <= 1e-12 * mag + 1e-300, "adjoint identity %g vs %g", lhs, rhs);
        for (int64_t e = 0; e < rp[n]; ++e) CHECK(isfinite(abar[e]), "abar not finite");
        free(ybar);
        free(bbar);
        free(Fbar);
        free(abar);
        free(db);
        /* dot, norm and product against plain loops */
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += fabs(b[i] * y[i]);
        double dd = orc_dot(n, b, y), naive = 0.0;
        for (int64_t i = 0; i < n; ++i) naive += b[i] * y[i];
        CHECK(fabs(dd - naive) <= 1e-13 * s + 1e-300, "dot %g vs %g", dd, naive);
        CHECK(orc_nrm2(n, b) >= 0.0, "norm");
    }
    free(gv);
    free(x2);
    free(y2);
    free(f);
    free(b);
    free(x);
    free(y);
    free(r);
    orc_pattern_free(&P);
done_a:
    free(rp);
    free(ci);
    free(v);
}

int main(void)
{
    int cases = 0;
    for (int64_t n = 0; n <= 60; n += (n < 8 ? 1 : 7)) {
        const double dens[3] = {0.03, 0.1, 0.3};
        for (int d = 0; d < 3; ++d) {
            const int32_t ks[5] = {0, 1, 2, 3, (int32_t)(n > 0 ? n : 1)};
            for (int q = 0; q < 5; ++q) {
                run_case(n, dens[d], ks[q]);
                ++cases;
            }
        }
    }
    /* malformed structures are refused */
    {
        int64_t rp[3] = {0, 2, 3};
        int32_t ci[3] = {1, 0, 1};  /* unsorted row 0 */
        CHECK(orc_validate(2, rp, ci) == ORC_EINVAL, "unsorted row accepted");
        int32_t ci2[3] = {0, 5, 1};  /* column out of range */
        CHECK(orc_validate(2, rp, ci2) == ORC_EINVAL, "column out of range accepted");
        orc_pattern P;
        CHECK(orc_symbolic(2, rp, ci, 1, &P) == ORC_EINVAL, "symbolic accepted an unsorted row");
        orc_pattern_free(&P);
    }
    if (failures) {
        fprintf(stderr, "selftest: %d checks failed over %d cases\n", failures, cases);
        return 1;
    }
    if (exact_inverse_checks == 0) {
        fprintf(stderr, "selftest: no case reached a dense complete fill\n");
        return 1;
    }
    printf("selftest: %d cases passed (%d with exact inverses)\n", cases, exact_inverse_checks);
    return 0;
}
