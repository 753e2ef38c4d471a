/*
 * Sequential CPU oracle for level-of-fill ILU(k) preconditioning.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg do.  It shares no code, header, table or
 * helper with the GPU library; both sides only consume the same seeded input
 * arrays.
 *
 * Every routine is the plain sequential definition written out, in the order
 * of operations the paper fixes (Dong & Cooperman, "A Bit-Compatible Shared
 * Memory Parallelization for ILU(k) Preconditioning ...").  Floating point is
 * IEEE-754 binary64 with round-to-nearest-even; every product and every sum
 * is rounded on its own (the file is compiled with -ffp-contract=off, no
 * -ffast-math, SSE2 arithmetic as on any x86-64 target).
 *
 * Conventions: 0-based indices, CSR with columns strictly ascending in each
 * row; F holds L~ strictly below the diagonal (unit diagonal implicit) and U~
 * on and above it (Sec. 2, "filled matrix").
 *
 * Status codes: 0 ok, 1 invalid input, 2 out of memory, 3 zero pivot,
 * 5 not converged.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2
#define ORC_EZEROPIVOT 3
#define ORC_ENOTCONV 5

/* ------------------------------------------------------------------------ */
/* Input validation: strictly ascending in-range columns, diagonal stored.   */
/* Every stored entry counts as a nonzero of A (structural reading of        */
/* Def. 2.3), so explicit zeros take part in the pattern.                    */
/* ------------------------------------------------------------------------ */
int orc_validate(int64_t n, const int64_t *rp, const int32_t *ci)
{
    if (n < 0 || rp[0] != 0) return ORC_EINVAL;
    for (int64_t j = 0; j < n; ++j) {
        if (rp[j + 1] < rp[j]) return ORC_EINVAL;
        int has_diag = 0;
        for (int64_t p = rp[j]; p < rp[j + 1]; ++p) {
            if (ci[p] < 0 || ci[p] >= n) return ORC_EINVAL;
            if (p > rp[j] && ci[p] <= ci[p - 1]) return ORC_EINVAL;
            if (ci[p] == j) has_diag = 1;
        }
        if (!has_diag) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase I: the level-k pattern of F (Def. 2.3; Sec. 2.2 computes it as     */
/* Phase I of ILU(k)).                                                       */
/*                                                                           */
/* Def. 2.3 gives every position (j,t) a level: 0 where A stores an entry    */
/* (every stored entry, explicit zeros included), otherwise the minimum over */
/* h < min(j,t) of level(j,h) + level(h,t) + 1.  The pattern is the set of   */
/* positions whose level is at most k.                                       */
/*                                                                           */
/* This routine evaluates that recurrence directly.  Rows go in ascending    */
/* order: the terms of row j only use positions (j,h) with h < j and rows h  */
/* < j, which are complete by then.  Inside row j the positions are found in */
/* rounds of increasing level value L = 0, 1, ..., k: round 0 takes A's      */
/* row; round L takes every position not found yet for which some h of row j */
/* with h < j and level a < L has (h,t), t > h, at level L-1-a.  A position  */
/* found in round L has no term below L (a smaller term would have been seen */
/* in an earlier round, whose parts were all known by then), so L is its     */
/* level.  Pruning: a term is larger than each of its two parts, so a        */
/* position of level <= k only ever takes its minimum over parts of level    */
/* <= k; rows h are therefore kept only up to level k.                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n, nnz;
    int64_t *rowptr; /* n+1 */
    int32_t *col;    /* nnz */
    int32_t *lev;    /* nnz */
} orc_pattern;

void orc_pattern_free(orc_pattern *p)
{
    free(p->rowptr);
    free(p->col);
    free(p->lev);
    p->rowptr = NULL;
    p->col = NULL;
    p->lev = NULL;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* (level, column) pairs of a row's strict upper part, ordered by level and
 * then column, so that the positions of one level are one contiguous run */
typedef struct {
    int32_t lev, col;
} lev_col;

static int cmp_lev_col(const void *a, const void *b)
{
    const lev_col *x = (const lev_col *)a, *y = (const lev_col *)b;
    if (x->lev != y->lev) return (x->lev > y->lev) - (x->lev < y->lev);
    return (x->col > y->col) - (x->col < y->col);
}

/* grow two parallel int32 arrays of capacity *cap to hold `need` entries;
 * returns 0 when out of memory (both arrays stay valid and owned) */
static int grow_pair(int32_t **a, int32_t **b, int64_t *cap, int64_t need)
{
    if (need <= *cap) return 1;
    int64_t c = *cap;
    while (c < need) c *= 2;
    int32_t *a2 = (int32_t *)realloc(*a, (size_t)c * sizeof(int32_t));
    if (!a2) return 0;
    *a = a2;
    int32_t *b2 = (int32_t *)realloc(*b, (size_t)c * sizeof(int32_t));
    if (!b2) return 0;
    *b = b2;
    *cap = c;
    return 1;
}

int orc_symbolic(int64_t n, const int64_t *rp, const int32_t *ci, int32_t k, orc_pattern *out)
{
    memset(out, 0, sizeof(*out));
    if (k < 0) return ORC_EINVAL;
    int st = orc_validate(n, rp, ci);
    if (st) return st;

    const size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t cap = rp[n] > 16 ? rp[n] : 16, ucap = cap;
    int64_t *rowptr = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    int32_t *lev = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
    /* strict upper part of every finished row, by level then column */
    int64_t *uptr = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *ucol = (int32_t *)malloc((size_t)ucap * sizeof(int32_t));
    int32_t *ulev = (int32_t *)malloc((size_t)ucap * sizeof(int32_t));
    int32_t *lev_of = (int32_t *)malloc(nn * sizeof(int32_t)); /* level of (j,t) in row j, -1 if absent */
    int32_t *found = (int32_t *)malloc(nn * sizeof(int32_t));  /* columns of row j, in order found */
    int32_t *lower = (int32_t *)malloc(nn * sizeof(int32_t));  /* its columns h < j, in order found */
    lev_col *upper = (lev_col *)malloc(nn * sizeof(lev_col));
    int ok = rowptr && col && lev && uptr && ucol && ulev && lev_of && found && lower && upper;
    if (ok)
        for (int64_t t = 0; t < n; ++t) lev_of[t] = -1;

    int64_t nnz = 0, unnz = 0;
    int64_t max_up = -1; /* highest level in the strict upper part of any finished row */
    if (ok) {
        rowptr[0] = 0;
        uptr[0] = 0;
    }
    for (int64_t j = 0; ok && j < n; ++j) {
        int64_t nf = 0, nl = 0, max_low = -1;
        /* level 0: the entries A stores in row j */
        for (int64_t p = rp[j]; p < rp[j + 1]; ++p) {
            int32_t t = ci[p];
            lev_of[t] = 0;
            found[nf++] = t;
            if (t < j) {
                lower[nl++] = t;
                max_low = 0;
            }
        }
        /* levels 1, 2, ...: a round can only produce levels up to
         * max_low + max_up + 1, and never more than k */
        for (int64_t L = 1; L <= (int64_t)k && L <= max_low + max_up + 1; ++L) {
            const int64_t nl_start = nl; /* positions found in this round have level L */
            for (int64_t a_i = 0; a_i < nl_start; ++a_i) {
                const int32_t h = lower[a_i];
                const int64_t a = lev_of[h];
                if (a > L - 1) continue;
                const int64_t b = L - 1 - a;
                /* the run of row h's strict upper part at level b */
                int64_t lo = uptr[h], hi = uptr[h + 1];
                while (lo < hi) {
                    int64_t mid = lo + (hi - lo) / 2;
                    if (ulev[mid] < b) lo = mid + 1;
                    else hi = mid;
                }
                for (int64_t q = lo; q < uptr[h + 1] && ulev[q] == b; ++q) {
                    const int32_t t = ucol[q];
                    if (lev_of[t] >= 0) continue; /* already at a level <= L */
                    lev_of[t] = (int32_t)L;
                    found[nf++] = t;
                    if (t < j) {
                        lower[nl++] = t;
                        max_low = L;
                    }
                }
            }
        }
        qsort(found, (size_t)nf, sizeof(int32_t), cmp_i32);
        int64_t nu = 0;
        for (int64_t a = 0; a < nf; ++a)
            if (found[a] > j) {
                upper[nu].lev = lev_of[found[a]];
                upper[nu].col = found[a];
                ++nu;
            }
        qsort(upper, (size_t)nu, sizeof(lev_col), cmp_lev_col);
        if (!grow_pair(&col, &lev, &cap, nnz + nf) || !grow_pair(&ucol, &ulev, &ucap, unnz + nu)) ok = 0;
        if (!ok) break;
        for (int64_t a = 0; a < nf; ++a) {
            col[nnz + a] = found[a];
            lev[nnz + a] = lev_of[found[a]];
            lev_of[found[a]] = -1;
        }
        for (int64_t a = 0; a < nu; ++a) {
            ucol[unnz + a] = upper[a].col;
            ulev[unnz + a] = upper[a].lev;
            if (upper[a].lev > max_up) max_up = upper[a].lev;
        }
        nnz += nf;
        unnz += nu;
        rowptr[j + 1] = nnz;
        uptr[j + 1] = unnz;
    }
    free(uptr);
    free(ucol);
    free(ulev);
    free(lev_of);
    free(found);
    free(lower);
    free(upper);
    if (!ok) {
        free(rowptr);
        free(col);
        free(lev);
        return ORC_ENOMEM;
    }
    out->n = n;
    out->nnz = nnz;
    out->rowptr = rowptr;
    out->col = col;
    out->lev = lev;
    return ORC_OK;
}

/* diagonal slot of every row of a pattern; -1 if absent */
static int find_diag(int64_t n, const int64_t *rpF, const int32_t *ciF, int64_t *diag)
{
    for (int64_t i = 0; i < n; ++i) {
        diag[i] = -1;
        for (int64_t s = rpF[i]; s < rpF[i + 1]; ++s)
            if (ciF[s] == i) { diag[i] = s; break; }
        if (diag[i] < 0) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Phase II: numeric factorization, row-wise IKJ (Eq. 2 read as running      */
/* updates, Eqs. 6a/6b).  F starts as A scattered into the pattern, fill     */
/* entries +0.0.  Row j in ascending order; for each pivot h < j of row j in */
/* ascending order:  f_jh <- f_jh / f_hh, then for every t > h stored in     */
/* both row h and row j:  f_jt <- f_jt - f_jh * f_ht.                        */
/* A zero pivot does not stop the elimination (IEEE division yields +-inf or */
/* NaN); *bad_row receives the smallest row whose final pivot f_jj is +-0,   */
/* or -1.                                                                    */
/* The update is rounded in one of two ways: product and difference each     */
/* rounded (orc_numeric), or the exact f_jt - f_jh * f_ht rounded once, a    */
/* fused multiply-add (orc_numeric_fused).                                   */
/* ------------------------------------------------------------------------ */
/* Row j of the factor (Eq. 2 restricted to the pattern, IKJ order): A's row
 * scattered into F's pattern, then for every pivot h < j of the row in
 * ascending column order l = f_jh / u_hh and f_jt -= l * u_ht for the t of
 * U~'s row h that lie in row j's pattern.  `row` receives row j's values
 * (its slots rpF[j]..rpF[j+1]-1); pivot rows are read from `vpiv` at their
 * own slots.  slot_of must be all -1 on entry and is left so. */
static int eliminate_row(int64_t j, const int64_t *rpA, const int32_t *ciA, const double *vA,
                         const int64_t *rpF, const int32_t *ciF, const int64_t *diag,
                         int64_t *slot_of, const double *vpiv, double *row, int fused)
{
    const int64_t r0 = rpF[j];
    int st = ORC_OK;
    for (int64_t s = r0; s < rpF[j + 1]; ++s) {
        slot_of[ciF[s]] = s - r0;
        row[s - r0] = 0.0;
    }
    for (int64_t p = rpA[j]; p < rpA[j + 1]; ++p) {
        int64_t s = slot_of[ciA[p]];
        if (s < 0) { st = ORC_EINVAL; break; }
        row[s] = vA[p];
    }
    if (st == ORC_OK) {
        for (int64_t s = r0; s < diag[j]; ++s) {
            int64_t h = ciF[s];
            row[s - r0] = row[s - r0] / vpiv[diag[h]];
            double l = row[s - r0];
            for (int64_t q = diag[h] + 1; q < rpF[h + 1]; ++q) {
                int64_t p = slot_of[ciF[q]];
                if (p >= 0) row[p] = fused ? fma(-l, vpiv[q], row[p]) : row[p] - l * vpiv[q];
            }
        }
    }
    for (int64_t s = r0; s < rpF[j + 1]; ++s) slot_of[ciF[s]] = -1;
    return st;
}

static int numeric_impl(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                        const int64_t *rpF, const int32_t *ciF, double *vF, int64_t *bad_row, int fused)
{
    *bad_row = -1;
    int64_t *slot_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!slot_of || !diag) { free(slot_of); free(diag); return ORC_ENOMEM; }
    int st = find_diag(n, rpF, ciF, diag);
    if (st) { free(slot_of); free(diag); return st; }
    for (int64_t t = 0; t < n; ++t) slot_of[t] = -1;

    for (int64_t j = 0; j < n; ++j) {
        /* rows are produced in order, so every pivot row is final in vF */
        st = eliminate_row(j, rpA, ciA, vA, rpF, ciF, diag, slot_of, vF, vF + rpF[j], fused);
        if (st) break;
        if (vF[diag[j]] == 0.0 && *bad_row < 0) *bad_row = j;
    }
    free(slot_of);
    free(diag);
    if (st) return st;
    return *bad_row >= 0 ? ORC_EZEROPIVOT : ORC_OK;
}

int orc_numeric(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                const int64_t *rpF, const int32_t *ciF, double *vF, int64_t *bad_row)
{
    return numeric_impl(n, rpA, ciA, vA, rpF, ciF, vF, bad_row, 0);
}

int orc_numeric_fused(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                      const int64_t *rpF, const int32_t *ciF, double *vF, int64_t *bad_row)
{
    return numeric_impl(n, rpA, ciA, vA, rpF, ciF, vF, bad_row, 1);
}

/* The listed rows alone, each eliminated against the pivot rows given in
 * vF (for instance a factor computed elsewhere): row rows[r] goes to
 * out[off[r] .. off[r+1]), off[r] = sum of the lengths of the rows before. */
int orc_numeric_rows(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                     const int64_t *rpF, const int32_t *ciF, const double *vF, int64_t nrows,
                     const int64_t *rows, double *out)
{
    int64_t *slot_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!slot_of || !diag) { free(slot_of); free(diag); return ORC_ENOMEM; }
    int st = find_diag(n, rpF, ciF, diag);
    for (int64_t t = 0; t < n; ++t) slot_of[t] = -1;
    int64_t o = 0;
    for (int64_t r = 0; r < nrows && st == ORC_OK; ++r) {
        const int64_t j = rows[r];
        if (j < 0 || j >= n) { st = ORC_EINVAL; break; }
        st = eliminate_row(j, rpA, ciA, vA, rpF, ciF, diag, slot_of, vF, out + o, 0);
        o += rpF[j + 1] - rpF[j];
    }
    free(slot_of);
    free(diag);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Applying M^-1 = U~^-1 L~^-1 (Eq. 1): forward substitution (Eq. 3b) with   */
/* a running subtraction in ascending column order; then the backward        */
/* substitution from the last row to the first, each row a running           */
/* subtraction in descending column order (right to left) followed by the   */
/* division by the pivot.  The paper does not fix the order inside the      */
/* backward substitution; right to left is the reading taken (the nearest   */
/* row's value, the last one to be known in a parallel sweep, is then the   */
/* last term).                                                              */
/* ------------------------------------------------------------------------ */
int orc_apply(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vF,
              const double *p, double *x, double *y)
{
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!diag) return ORC_ENOMEM;
    int st = find_diag(n, rpF, ciF, diag);
    if (st) { free(diag); return st; }
    for (int64_t i = 0; i < n; ++i) {
        double s = p[i];
        for (int64_t q = rpF[i]; q < diag[i]; ++q) s = s - vF[q] * x[ciF[q]];
        x[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t q = rpF[i + 1] - 1; q > diag[i]; --q) s = s - vF[q] * y[ciF[q]];
        y[i] = s / vF[diag[i]];
    }
    free(diag);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Krylov building blocks.  The paper keeps inner products sequential so     */
/* their result does not depend on the thread count (Sec. 3.5); here every   */
/* reduction has one fixed shape that depends only on the vector length.    */
/* ------------------------------------------------------------------------ */

/* y = A x, each row summed from +0.0 in ascending column order */
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
              const double *x, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s = s + v[p] * x[ci[p]];
        y[i] = s;
    }
}

#define ORC_DOT_LANES 16384

/* Fixed-shape inner product: 16384 strided partial sums (lane l sums the    */
/* products of elements l, l+16384, ... in ascending order from +0.0), then  */
/* a pairwise tree: at stride w = 1, 2, 4, ..., lane l (l a multiple of 2w)  */
/* becomes lane l + lane l+w.  The result is lane 0.                         */
double orc_dot(int64_t n, const double *x, const double *y)
{
    static double s[ORC_DOT_LANES];
    for (int64_t l = 0; l < ORC_DOT_LANES; ++l) {
        double a = 0.0;
        for (int64_t e = l; e < n; e += ORC_DOT_LANES) a = a + x[e] * y[e];
        s[l] = a;
    }
    for (int64_t w = 1; w < ORC_DOT_LANES; w *= 2)
        for (int64_t l = 0; l < ORC_DOT_LANES; l += 2 * w) s[l] = s[l] + s[l + w];
    return s[0];
}

double orc_nrm2(int64_t n, const double *x) { return sqrt(orc_dot(n, x, x)); }

/* ------------------------------------------------------------------------ */
/* Restarted GMRES(m), right preconditioned: the solver works on A M^-1,     */
/* M = L~ U~ (Sec. 2: the iterative solver implicitly solves A U~^-1 L~^-1). */
/* Modified Gram-Schmidt Arnoldi, Givens rotations (rho computed as          */
/* sqrt(a*a + b*b), no hypot), inner loop stopped on the implicit residual   */
/* |g_{j+1}|, outer loop on the true residual.  maxit counts inner           */
/* iterations over all cycles.  x holds x0 on entry.  hist (nullable, maxit  */
/* entries) receives |g_{j+1}| after every inner iteration.                  */
/* ------------------------------------------------------------------------ */
int orc_apply_inverse(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vG,
                      const double *p, double *x, double *y);

/* z = M^-1 v: the two substitutions (vM = F), or the two products with the
   incomplete inverses (vM = G) */
static void apply_m(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vM, int inverse,
                    const double *v, double *t, double *z)
{
    if (inverse) orc_apply_inverse(n, rpF, ciF, vM, v, t, z);
    else orc_apply(n, rpF, ciF, vM, v, t, z);
}

static int gmres_impl(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                      const int64_t *rpF, const int32_t *ciF, const double *vF, int inverse,
                      const double *b, double *x, int32_t m, int32_t maxit, double rtol,
                      int32_t *iters_out, double *relres_out, double *hist)
{
    *iters_out = 0;
    *relres_out = 0.0;
    if (m < 1 || maxit < 0) return ORC_EINVAL;
    size_t N = (size_t)(n > 0 ? n : 1);
    double *V = (double *)malloc((size_t)(m + 1) * N * sizeof(double));
    double *w = (double *)malloc(N * sizeof(double));
    double *z = (double *)malloc(N * sizeof(double));
    double *t = (double *)malloc(N * sizeof(double));
    double *H = (double *)malloc((size_t)(m + 1) * (size_t)m * sizeof(double));
    double *cs = (double *)malloc((size_t)m * sizeof(double));
    double *sn = (double *)malloc((size_t)m * sizeof(double));
    double *g = (double *)malloc((size_t)(m + 1) * sizeof(double));
    double *yv = (double *)malloc((size_t)m * sizeof(double));
    if (!V || !w || !z || !t || !H || !cs || !sn || !g || !yv) {
        free(V); free(w); free(z); free(t); free(H); free(cs); free(sn); free(g); free(yv);
        return ORC_ENOMEM;
    }
#define HH(i, j) H[(size_t)(i) * (size_t)m + (size_t)(j)]
    int st = ORC_OK;
    int32_t iters = 0;
    double bnorm = orc_nrm2(n, b);
    if (bnorm == 0.0) {
        for (int64_t e = 0; e < n; ++e) x[e] = 0.0;
        goto done;
    }
    double tol = rtol * bnorm;
    for (;;) {
        /* true residual */
        orc_spmv(n, rpA, ciA, vA, x, w);
        for (int64_t e = 0; e < n; ++e) w[e] = b[e] - w[e];
        double beta = orc_nrm2(n, w);
        if (beta <= tol || iters >= maxit) break;
        for (int64_t e = 0; e < n; ++e) V[e] = w[e] / beta;
        g[0] = beta;
        int32_t jj = 0;
        for (int32_t j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * N;
            apply_m(n, rpF, ciF, vF, inverse, vj, t, z);
            orc_spmv(n, rpA, ciA, vA, z, w);
            for (int32_t i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * N;
                double hij = orc_dot(n, w, vi);
                HH(i, j) = hij;
                for (int64_t e = 0; e < n; ++e) w[e] = w[e] - hij * vi[e];
            }
            double hn = orc_nrm2(n, w);
            HH(j + 1, j) = hn;
            if (hn != 0.0) {
                double *vn = V + (size_t)(j + 1) * N;
                for (int64_t e = 0; e < n; ++e) vn[e] = w[e] / hn;
            }
            for (int32_t i = 0; i < j; ++i) {
                double a = HH(i, j), c = HH(i + 1, j);
                double tau = cs[i] * a + sn[i] * c;
                HH(i + 1, j) = cs[i] * c - sn[i] * a;
                HH(i, j) = tau;
            }
            double a = HH(j, j), c = HH(j + 1, j);
            double rho = sqrt(a * a + c * c);
            cs[j] = a / rho;
            sn[j] = c / rho;
            HH(j, j) = rho;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            if (hist) hist[iters] = fabs(g[j + 1]);
            ++iters;
            jj = j + 1;
            if (fabs(g[j + 1]) <= tol || iters >= maxit || hn == 0.0) break;
        }
        /* back substitution H(0:jj,0:jj) y = g, then x += M^-1 (V y) */
        for (int32_t i = jj - 1; i >= 0; --i) {
            double s = g[i];
            for (int32_t l = i + 1; l < jj; ++l) s = s - HH(i, l) * yv[l];
            yv[i] = s / HH(i, i);
        }
        for (int64_t e = 0; e < n; ++e) {
            double s = 0.0;
            for (int32_t i = 0; i < jj; ++i) s = s + yv[i] * V[(size_t)i * N + (size_t)e];
            w[e] = s;
        }
        apply_m(n, rpF, ciF, vF, inverse, w, t, z);
        for (int64_t e = 0; e < n; ++e) x[e] = x[e] + z[e];
    }
    orc_spmv(n, rpA, ciA, vA, x, w);
    for (int64_t e = 0; e < n; ++e) w[e] = b[e] - w[e];
    *relres_out = orc_nrm2(n, w) / bnorm;
    if (!(*relres_out <= rtol)) st = ORC_ENOTCONV;
done:
    *iters_out = iters;
#undef HH
    free(V); free(w); free(z); free(t); free(H); free(cs); free(sn); free(g); free(yv);
    return st;
}

int orc_gmres(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
              const int64_t *rpF, const int32_t *ciF, const double *vF,
              const double *b, double *x, int32_t m, int32_t maxit, double rtol,
              int32_t *iters_out, double *relres_out, double *hist)
{
    return gmres_impl(n, rpA, ciA, vA, rpF, ciF, vF, 0, b, x, m, maxit, rtol, iters_out, relres_out, hist);
}

/* ------------------------------------------------------------------------ */
/* BiCGSTAB, the Krylov method the paper runs (through Hypre, Sec. 4), right */
/* preconditioned (the solver works on A M^-1, Sec. 2), in the textbook form */
/* of van der Vorst with the shadow residual fixed to the first residual.   */
/* Every scalar and vector step is one fixed expression, rounded step by    */
/* step as written:                                                          */
/*   r = b - A x, rs = r, rho_old = alpha = omega = 1, v = p = 0             */
/*   loop: rho = (rs, r); stop on rho == 0 (breakdown)                        */
/*     first pass p = r, else beta = (rho / rho_old) * (alpha / omega) and    */
/*       p_e = r_e + beta * (p_e - omega * v_e)                               */
/*     ph = M^-1 p; v = A ph; alpha = rho / (rs, v) (breakdown on 0)          */
/*     s_e = r_e - alpha * v_e; iters++; hist = ||s||                         */
/*     if ||s|| <= rtol ||b||: x_e = x_e + alpha * ph_e, stop                 */
/*     sh = M^-1 s; t = A sh; omega = (t, s) / (t, t) (breakdown on 0)        */
/*     x_e = (x_e + alpha * ph_e) + omega * sh_e; r_e = s_e - omega * t_e     */
/*     hist = ||r||; stop if ||r|| <= rtol ||b|| or iters >= maxit            */
/*     rho_old = rho                                                          */
/* iters counts half steps (each ph and each sh), so hist has one entry per */
/* preconditioner application.  Returns the true relative residual.         */
/* ------------------------------------------------------------------------ */
static int bicgstab_impl(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                         const int64_t *rpF, const int32_t *ciF, const double *vM, int inverse,
                         const double *b, double *x, int32_t maxit, double rtol,
                         int32_t *iters_out, double *relres_out, double *hist)
{
    *iters_out = 0;
    *relres_out = 0.0;
    if (maxit < 0) return ORC_EINVAL;
    size_t N = (size_t)(n > 0 ? n : 1);
    double *r = (double *)malloc(N * sizeof(double));
    double *rs = (double *)malloc(N * sizeof(double));
    double *p = (double *)malloc(N * sizeof(double));
    double *v = (double *)malloc(N * sizeof(double));
    double *ph = (double *)malloc(N * sizeof(double));
    double *sv = (double *)malloc(N * sizeof(double));
    double *sh = (double *)malloc(N * sizeof(double));
    double *t = (double *)malloc(N * sizeof(double));
    double *tmp = (double *)malloc(N * sizeof(double));
    if (!r || !rs || !p || !v || !ph || !sv || !sh || !t || !tmp) {
        free(r); free(rs); free(p); free(v); free(ph); free(sv); free(sh); free(t); free(tmp);
        return ORC_ENOMEM;
    }
    int st = ORC_OK;
    int32_t iters = 0;
    double bnorm = orc_nrm2(n, b);
    if (bnorm == 0.0) {
        for (int64_t e = 0; e < n; ++e) x[e] = 0.0;
        goto done;
    }
    double tol = rtol * bnorm;
    orc_spmv(n, rpA, ciA, vA, x, r);
    for (int64_t e = 0; e < n; ++e) {
        r[e] = b[e] - r[e];
        rs[e] = r[e];
        p[e] = 0.0;
        v[e] = 0.0;
    }
    if (orc_nrm2(n, r) <= tol) goto finish;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    int first = 1;
    while (iters < maxit) {
        double rho = orc_dot(n, rs, r);
        if (rho == 0.0) { st = ORC_ENOTCONV; break; }
        if (first) {
            for (int64_t e = 0; e < n; ++e) p[e] = r[e];
            first = 0;
        } else {
            double beta = (rho / rho_old) * (alpha / omega);
            for (int64_t e = 0; e < n; ++e) p[e] = r[e] + beta * (p[e] - omega * v[e]);
        }
        apply_m(n, rpF, ciF, vM, inverse, p, tmp, ph);
        orc_spmv(n, rpA, ciA, vA, ph, v);
        double rv = orc_dot(n, rs, v);
        if (rv == 0.0) { st = ORC_ENOTCONV; break; }
        alpha = rho / rv;
        for (int64_t e = 0; e < n; ++e) sv[e] = r[e] - alpha * v[e];
        double snorm = orc_nrm2(n, sv);
        if (hist) hist[iters] = snorm;
        ++iters;
        if (snorm <= tol) {
            for (int64_t e = 0; e < n; ++e) x[e] = x[e] + alpha * ph[e];
            break;
        }
        if (iters >= maxit) {
            for (int64_t e = 0; e < n; ++e) x[e] = x[e] + alpha * ph[e];
            break;
        }
        apply_m(n, rpF, ciF, vM, inverse, sv, tmp, sh);
        orc_spmv(n, rpA, ciA, vA, sh, t);
        double ts = orc_dot(n, t, sv);
        double tt = orc_dot(n, t, t);
        if (tt == 0.0) { st = ORC_ENOTCONV; break; }
        omega = ts / tt;
        for (int64_t e = 0; e < n; ++e) {
            x[e] = (x[e] + alpha * ph[e]) + omega * sh[e];
            r[e] = sv[e] - omega * t[e];
        }
        double rnorm = orc_nrm2(n, r);
        if (hist) hist[iters] = rnorm;
        ++iters;
        if (rnorm <= tol) break;
        if (omega == 0.0) { st = ORC_ENOTCONV; break; }
        rho_old = rho;
    }
finish:
    orc_spmv(n, rpA, ciA, vA, x, tmp);
    for (int64_t e = 0; e < n; ++e) tmp[e] = b[e] - tmp[e];
    *relres_out = orc_nrm2(n, tmp) / bnorm;
    if (!(*relres_out <= rtol)) st = ORC_ENOTCONV;
done:
    *iters_out = iters;
    free(r); free(rs); free(p); free(v); free(ph); free(sv); free(sh); free(t); free(tmp);
    return st;
}

int orc_bicgstab(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                 const int64_t *rpF, const int32_t *ciF, const double *vM, int32_t inverse,
                 const double *b, double *x, int32_t maxit, double rtol,
                 int32_t *iters_out, double *relres_out, double *hist)
{
    return bicgstab_impl(n, rpA, ciA, vA, rpF, ciF, vM, inverse != 0, b, x, maxit, rtol, iters_out,
                         relres_out, hist);
}

/* the same GMRES(m) with M^-1 applied through the incomplete inverses vG */
int orc_gmres_inverse(int64_t n, const int64_t *rpA, const int32_t *ciA, const double *vA,
                      const int64_t *rpF, const int32_t *ciF, const double *vG,
                      const double *b, double *x, int32_t m, int32_t maxit, double rtol,
                      int32_t *iters_out, double *relres_out, double *hist)
{
    return gmres_impl(n, rpA, ciA, vA, rpF, ciF, vG, 1, b, x, m, maxit, rtol, iters_out, relres_out, hist);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of y = U~^-1 L~^-1 b (reverse mode).  With x = L~^-1 b:           */
/*   z = U~^-T ybar  (i ascending, z_i = (ybar_i - sum_{j<i} f_ji z_j)/f_ii, */
/*                    running subtraction in ascending j)                    */
/*   w = L~^-T z     (i descending, w_i = z_i - sum_{j>i} f_ji w_j,          */
/*                    running subtraction in descending j)                   */
/*   bbar = w;  Fbar_ij = -(z_i y_j) on U (j >= i);  Fbar_ih = -(w_i x_h)    */
/*   on the strict lower part.                                               */
/* ------------------------------------------------------------------------ */
static int transpose_pattern(int64_t n, const int64_t *rp, const int32_t *ci, int64_t **tp_out,
                             int64_t **tslot_out)
{
    int64_t nnz = rp[n];
    int64_t *tp = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *ts = (int64_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int64_t));
    int64_t *fillp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!tp || !ts || !fillp) { free(tp); free(ts); free(fillp); return ORC_ENOMEM; }
    for (int64_t s = 0; s < nnz; ++s) tp[ci[s] + 1]++;
    for (int64_t c = 0; c < n; ++c) tp[c + 1] += tp[c];
    for (int64_t c = 0; c < n; ++c) fillp[c] = tp[c];
    for (int64_t r = 0; r < n; ++r) /* rows ascending: each column lists rows ascending */
        for (int64_t s = rp[r]; s < rp[r + 1]; ++s) ts[fillp[ci[s]]++] = s;
    free(fillp);
    *tp_out = tp;
    *tslot_out = ts;
    return ORC_OK;
}

/* row index of slot s, by binary search in rp */
static int64_t row_of(int64_t n, const int64_t *rp, int64_t s)
{
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (rp[mid] <= s) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int orc_apply_adjoint(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vF,
                      const double *x, const double *y, const double *ybar, double *bbar,
                      double *Fbar)
{
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    double *z = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!diag || !z) { free(diag); free(z); return ORC_ENOMEM; }
    int st = find_diag(n, rpF, ciF, diag);
    int64_t *tp = NULL, *ts = NULL;
    if (!st) st = transpose_pattern(n, rpF, ciF, &tp, &ts);
    if (st) { free(diag); free(z); return st; }
    /* z = U^-T ybar: column i of U above the diagonal = rows j < i */
    for (int64_t i = 0; i < n; ++i) {
        double s = ybar[i];
        for (int64_t a = tp[i]; a < tp[i + 1]; ++a) {
            int64_t q = ts[a];
            int64_t j = row_of(n, rpF, q);
            if (j >= i) break; /* rows ascending: the rest are on/below the diagonal */
            s = s - vF[q] * z[j];
        }
        z[i] = s / vF[diag[i]];
    }
    /* w = L^-T z: column i of L = rows j > i, taken in descending j */
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int64_t a = tp[i + 1] - 1; a >= tp[i]; --a) {
            int64_t q = ts[a];
            int64_t j = row_of(n, rpF, q);
            if (j <= i) break; /* rows descending: the rest are on/above the diagonal */
            s = s - vF[q] * bbar[j];
        }
        bbar[i] = s;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t q = rpF[i]; q < diag[i]; ++q) Fbar[q] = -(bbar[i] * x[ciF[q]]);
        for (int64_t q = diag[i]; q < rpF[i + 1]; ++q) Fbar[q] = -(z[i] * y[ciF[q]]);
    }
    free(diag); free(z); free(tp); free(ts);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the numeric factorization (reverse sweep of Eqs. 6a/6b).       */
/* Fbar holds dL/dF on entry (final factor values); rows are undone in       */
/* descending order, pivots of a row in descending order.  For pivot h of    */
/* row j with l = f_jh:                                                      */
/*   lbar = Fbar_jh - sum_t Fbar_jt f_ht      (t ascending, t in U(h)∩P(j))  */
/*   Fbar_ht <- Fbar_ht - Fbar_jt * l         (each such t)                  */
/*   Fbar_jh <- lbar / f_hh                                                  */
/*   Fbar_hh <- Fbar_hh - (lbar * l) / f_hh                                  */
/* Afterwards Fbar_j* is the gradient with respect to row j's initial        */
/* values; abar[p] picks A's entries (fill entries were constants).  Every   */
/* entry of row h therefore receives its contributions in descending j.      */
/* ------------------------------------------------------------------------ */
int orc_numeric_adjoint(int64_t n, const int64_t *rpA, const int32_t *ciA, const int64_t *rpF,
                        const int32_t *ciF, const double *vF, double *Fbar, double *abar)
{
    int64_t *slot_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!slot_of || !diag) { free(slot_of); free(diag); return ORC_ENOMEM; }
    int st = find_diag(n, rpF, ciF, diag);
    if (st) { free(slot_of); free(diag); return st; }
    for (int64_t t = 0; t < n; ++t) slot_of[t] = -1;
    for (int64_t j = n - 1; j >= 0; --j) {
        for (int64_t s = rpF[j]; s < rpF[j + 1]; ++s) slot_of[ciF[s]] = s;
        for (int64_t s = diag[j] - 1; s >= rpF[j]; --s) {
            int64_t h = ciF[s];
            double l = vF[s];
            double lbar = Fbar[s];
            for (int64_t q = diag[h] + 1; q < rpF[h + 1]; ++q) {
                int64_t p = slot_of[ciF[q]];
                if (p >= 0) lbar = lbar - Fbar[p] * vF[q];
            }
            for (int64_t q = diag[h] + 1; q < rpF[h + 1]; ++q) {
                int64_t p = slot_of[ciF[q]];
                if (p >= 0) Fbar[q] = Fbar[q] - Fbar[p] * l;
            }
            Fbar[s] = lbar / vF[diag[h]];
            double tmp = lbar * l;
            tmp = tmp / vF[diag[h]];
            Fbar[diag[h]] = Fbar[diag[h]] - tmp;
        }
        for (int64_t p = rpA[j]; p < rpA[j + 1]; ++p) {
            int64_t s = slot_of[ciA[p]];
            if (s < 0) { st = ORC_EINVAL; break; }
            abar[p] = Fbar[s];
        }
        for (int64_t s = rpF[j]; s < rpF[j + 1]; ++s) slot_of[ciF[s]] = -1;
        if (st) break;
    }
    free(slot_of);
    free(diag);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Level-based incomplete inverses (Sec. 3.5).                               */
/*                                                                           */
/* L~^-1 has a unit diagonal and the entries -beta_it below it (Eq. 3a),     */
/* where beta_it = f_it - sum over t < h < i of f_ih beta_ht (Eq. 5).  Rows  */
/* in ascending order, each after the ILU rows it needs; row i starts from   */
/* beta_it = f_it and, for its pivots h in ascending order and every column  */
/* t < h stored in both row h and row i, takes beta_it <- beta_it - f_ih     */
/* beta_ht (Eq. 6c); the stored inverse entries are -beta_it (Eq. 6d).       */
/* Level-based: only the pattern of L~ is kept, contributions to positions   */
/* outside it are dropped.                                                   */
/*                                                                           */
/* U~^-1 (the paper omits the details and names only the order: rows from    */
/* the last to the first, right to left within a row).  Row i of the inverse */
/* is (e_i - sum over pivots j > i of row i of u_ij (row j of the inverse))  */
/* / u_ii: the working row starts as e_i on row i's upper pattern, the       */
/* pivots j are taken from right to left, each subtracting u_ij g_jt at      */
/* every column t stored in both row j's inverse and row i, and finally      */
/* every entry is divided by u_ii.  Kept: the pattern of U~.                 */
/*                                                                           */
/* vG receives both, in F's slots: inverse of L~ in the strict lower slots,  */
/* inverse of U~ in the upper slots (diagonal included).                     */
/* ------------------------------------------------------------------------ */
int orc_inverse(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vF, double *vG)
{
    const int64_t nnz = n > 0 ? rpF[n] : 0;
    int64_t *slot_of = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    double *beta = (double *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    if (!slot_of || !diag || !beta) { free(slot_of); free(diag); free(beta); return ORC_ENOMEM; }
    int st = find_diag(n, rpF, ciF, diag);
    if (st) { free(slot_of); free(diag); free(beta); return st; }
    for (int64_t t = 0; t < n; ++t) slot_of[t] = -1;

    /* L~: rows ascending, beta kept unflipped until every row is done */
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t s = rpF[i]; s < diag[i]; ++s) {
            slot_of[ciF[s]] = s;
            beta[s] = vF[s];
        }
        for (int64_t s = rpF[i]; s < diag[i]; ++s) {
            const int64_t h = ciF[s];
            const double fih = vF[s];
            for (int64_t q = rpF[h]; q < diag[h]; ++q) {
                const int64_t p = slot_of[ciF[q]];
                if (p >= 0) beta[p] = beta[p] - fih * beta[q];
            }
        }
        for (int64_t s = rpF[i]; s < diag[i]; ++s) slot_of[ciF[s]] = -1;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t s = rpF[i]; s < diag[i]; ++s) vG[s] = -beta[s];

    /* U~: rows descending, pivots right to left, then the division */
    for (int64_t i = n - 1; i >= 0; --i) {
        for (int64_t s = diag[i]; s < rpF[i + 1]; ++s) {
            slot_of[ciF[s]] = s;
            vG[s] = 0.0;
        }
        vG[diag[i]] = 1.0;
        for (int64_t s = rpF[i + 1] - 1; s > diag[i]; --s) {
            const int64_t j = ciF[s];
            const double uij = vF[s];
            for (int64_t q = diag[j]; q < rpF[j + 1]; ++q) {
                const int64_t p = slot_of[ciF[q]];
                if (p >= 0) vG[p] = vG[p] - uij * vG[q];
            }
        }
        for (int64_t s = diag[i]; s < rpF[i + 1]; ++s) {
            vG[s] = vG[s] / vF[diag[i]];
            slot_of[ciF[s]] = -1;
        }
    }
    free(slot_of);
    free(diag);
    free(beta);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Applying the incomplete inverses (Sec. 3.5: the triangular solve stage    */
/* becomes two matrix-vector products).  x = L~~^-1 p as Eq. 3a writes it:   */
/* the sum over t < i of (L~~^-1)_it p_t, from +0.0 in ascending t, then     */
/* + p_i.  y = U~~^-1 x: the sum over t >= i, from +0.0 in ascending t (the  */
/* SpMV order).                                                              */
/* ------------------------------------------------------------------------ */
int orc_apply_inverse(int64_t n, const int64_t *rpF, const int32_t *ciF, const double *vG,
                      const double *p, double *x, double *y)
{
    int64_t *diag = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!diag) return ORC_ENOMEM;
    int st = find_diag(n, rpF, ciF, diag);
    if (st) { free(diag); return st; }
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = rpF[i]; q < diag[i]; ++q) s = s + vG[q] * p[ciF[q]];
        x[i] = s + p[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = diag[i]; q < rpF[i + 1]; ++q) s = s + vG[q] * x[ciF[q]];
        y[i] = s;
    }
    free(diag);
    return ORC_OK;
}
