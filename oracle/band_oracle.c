/*
 * Oracle for banded linear solves: TEST INFRASTRUCTURE ONLY.
 *
 * This file is a plain, slow, single-threaded FP64 reference for what the
 * recursive SPIKE solver computes.  SPIKE reaches exactly (up to rounding
 * order) X = A^{-1} F for the non-transpose solve and X = A^{-T} F for the
 * transpose solve, for any partition count, leaf factorisation (LU or UL,
 * pivoting or not) and reduced-system organisation (the DS factorisation
 * A = DS and the reduced-system derivation of the SPIKE background section,
 * and the transpose derivation S^T D^T X = F of the transpose section).  So
 * the oracle is that plain definition, computed by textbook banded Gaussian
 * elimination without any partitioning:
 *
 *   - non-pivoting LU on LAPACK band storage;
 *   - partial-pivoting LU with row interchanges restricted to the kl rows
 *     below the diagonal and U widened to kl+ku superdiagonals (the pivoting
 *     section: a pivot row moves at most k places);
 *   - forward/backward substitution for A X = F, and U^T then L^T (undoing
 *     the interchanges in reverse order) for A^T X = F;
 *   - banded matrix-vector products, residual metrics with compensated
 *     summation, the 1-norm condition estimate in the role the paper gives
 *     to DGBCON (Hager 1984 / Higham 1988), and the load-balancing ratio of
 *     the load-balancing section (eq. R13_calculation, R12 = R13/2).
 *
 * Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
 * load this code.  It shares no code, header, table or helper with the GPU
 * library; the GPU library never loads it.
 *
 * Band storage (the LAPACK convention): A(i,j), 0-based, is held at
 * ab[(ku + i - j) + j*ldab] for max(0, j-ku) <= i <= min(n-1, j+kl).
 *
 * Compile with: gcc -O2 -ffp-contract=off -shared -fPIC (no FMA contraction,
 * so every product and sum rounds as written).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

static int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Working band copy: U part may need kl extra superdiagonals (pivoting).    */
/* Element (i,j) of the working matrix lives at w[(uw + i - j) + j*ldw],     */
/* where uw is the number of stored superdiagonals.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int kl, uw;      /* subdiagonals of L, superdiagonals of U */
    int64_t ldw;     /* = kl + uw + 1 */
    double *w;
} work_band;

static double *wref(const work_band *b, int64_t i, int64_t j) {
    return &b->w[(b->uw + i - j) + j * b->ldw];
}

static int make_work_band(work_band *b, int64_t n, int kl, int ku,
                          const double *ab, int64_t ldab, int pivot) {
    b->n = n;
    b->kl = kl;
    b->uw = pivot ? kl + ku : ku;
    b->ldw = (int64_t)kl + b->uw + 1;
    b->w = (double *)calloc((size_t)(b->ldw * (n > 0 ? n : 1)), sizeof(double));
    if (!b->w) return -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = imax64(0, j - ku); i <= imin64(n - 1, j + kl); ++i)
            *wref(b, i, j) = ab[(ku + i - j) + j * ldab];
    return 0;
}

/* Non-pivoting LU (Doolittle, column by column).  L is unit lower with kl
 * subdiagonals, U upper with ku superdiagonals, both in place.  Returns 0 or
 * the 1-based index of the first exactly-zero pivot (elimination stops). */
static int64_t lu_nopiv(work_band *b) {
    const int64_t n = b->n;
    for (int64_t j = 0; j < n; ++j) {
        double piv = *wref(b, j, j);
        if (piv == 0.0) return j + 1;
        int64_t last_row = imin64(n - 1, j + b->kl);
        int64_t last_col = imin64(n - 1, j + b->uw);
        for (int64_t i = j + 1; i <= last_row; ++i) {
            double l = *wref(b, i, j) / piv;
            *wref(b, i, j) = l;
            for (int64_t c = j + 1; c <= last_col; ++c)
                *wref(b, i, c) -= l * *wref(b, j, c);
        }
    }
    return 0;
}

/* Partial-pivoting LU with the interchanges of LAPACK's unblocked banded LU:
 * at column j the pivot is the first row of maximal magnitude among rows
 * j..j+kl; rows j and the pivot row are exchanged over columns j..j+kl+ku;
 * the multipliers of column j are stored below the diagonal and are not
 * permuted by later interchanges.  A zero pivot column records info and is
 * skipped, as LAPACK does. */
static int64_t lu_piv(work_band *b, int64_t *ipiv) {
    const int64_t n = b->n;
    int64_t info = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t last_row = imin64(n - 1, j + b->kl);
        int64_t last_col = imin64(n - 1, j + b->uw);
        int64_t r = j;
        double best = fabs(*wref(b, j, j));
        for (int64_t i = j + 1; i <= last_row; ++i) {
            double v = fabs(*wref(b, i, j));
            if (v > best) { best = v; r = i; }
        }
        ipiv[j] = r;
        if (*wref(b, r, j) == 0.0) {
            if (info == 0) info = j + 1;
            continue;
        }
        if (r != j)
            for (int64_t c = j; c <= last_col; ++c) {
                double t = *wref(b, j, c);
                *wref(b, j, c) = *wref(b, r, c);
                *wref(b, r, c) = t;
            }
        double piv = *wref(b, j, j);
        for (int64_t i = j + 1; i <= last_row; ++i) {
            double l = *wref(b, i, j) / piv;
            *wref(b, i, j) = l;
            for (int64_t c = j + 1; c <= last_col; ++c)
                *wref(b, i, c) -= l * *wref(b, j, c);
        }
    }
    return info;
}

/* x <- A^{-1} x for one column, given the factors. */
static void solve_n(const work_band *b, const int64_t *ipiv, double *x) {
    const int64_t n = b->n;
    for (int64_t j = 0; j < n; ++j) {           /* L^{-1} P, interleaved */
        if (ipiv && ipiv[j] != j) {
            double t = x[j]; x[j] = x[ipiv[j]]; x[ipiv[j]] = t;
        }
        for (int64_t i = j + 1; i <= imin64(n - 1, j + b->kl); ++i)
            x[i] -= *wref(b, i, j) * x[j];
    }
    for (int64_t j = n - 1; j >= 0; --j) {      /* U^{-1}, column oriented */
        x[j] /= *wref(b, j, j);
        for (int64_t i = imax64(0, j - b->uw); i < j; ++i)
            x[i] -= *wref(b, i, j) * x[j];
    }
}

/* x <- A^{-T} x for one column: U^T w = x forward, then L^T backward with the
 * interchanges undone in reverse order. */
static void solve_t(const work_band *b, const int64_t *ipiv, double *x) {
    const int64_t n = b->n;
    for (int64_t j = 0; j < n; ++j) {
        double s = x[j];
        for (int64_t i = imax64(0, j - b->uw); i < j; ++i)
            s -= *wref(b, i, j) * x[i];
        x[j] = s / *wref(b, j, j);
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        double s = x[j];
        for (int64_t i = j + 1; i <= imin64(n - 1, j + b->kl); ++i)
            s -= *wref(b, i, j) * x[i];
        x[j] = s;
        if (ipiv && ipiv[j] != j) {
            double t = x[j]; x[j] = x[ipiv[j]]; x[ipiv[j]] = t;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                      */
/* ------------------------------------------------------------------------ */

/* Solve op(A) X = F in place on B (n x nrhs, column-major, ldb >= n).
 * pivot: 0 = non-pivoting LU, 1 = partial pivoting.  trans: 0 = A, 1 = A^T.
 * Returns 0, a negative argument error, or the 1-based index of the first
 * zero pivot (B is then left untouched). */
ORC_EXPORT int64_t orc_gbsv(int64_t n, int kl, int ku, const double *ab,
                            int64_t ldab, int pivot, int trans, int nrhs,
                            double *B, int64_t ldb) {
    if (n < 0) return -1;
    if (kl < 0) return -2;
    if (ku < 0) return -3;
    if (ldab < (int64_t)kl + ku + 1) return -5;
    if (nrhs < 0) return -8;
    if (ldb < (n > 1 ? n : 1)) return -10;
    if (n == 0) return 0;
    work_band b;
    if (make_work_band(&b, n, kl, ku, ab, ldab, pivot)) return -100;
    int64_t *ipiv = NULL;
    int64_t info;
    if (pivot) {
        ipiv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        info = lu_piv(&b, ipiv);
    } else {
        info = lu_nopiv(&b);
    }
    if (info == 0)
        for (int c = 0; c < nrhs; ++c) {
            if (trans) solve_t(&b, ipiv, B + (int64_t)c * ldb);
            else       solve_n(&b, ipiv, B + (int64_t)c * ldb);
        }
    free(ipiv);
    free(b.w);
    return info;
}

/* One factorisation, then A X = F on B and A^T X = F on Bt (both n x nrhs,
 * leading dimension ldb).  Returns as orc_gbsv. */
ORC_EXPORT int64_t orc_gbsv_nt(int64_t n, int kl, int ku, const double *ab,
                               int64_t ldab, int pivot, int nrhs, double *B,
                               double *Bt, int64_t ldb) {
    if (n <= 0) return n < 0 ? -1 : 0;
    work_band b;
    if (make_work_band(&b, n, kl, ku, ab, ldab, pivot)) return -100;
    int64_t *ipiv = NULL;
    int64_t info;
    if (pivot) {
        ipiv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        info = lu_piv(&b, ipiv);
    } else {
        info = lu_nopiv(&b);
    }
    if (info == 0)
        for (int c = 0; c < nrhs; ++c) {
            solve_n(&b, ipiv, B + (int64_t)c * ldb);
            solve_t(&b, ipiv, Bt + (int64_t)c * ldb);
        }
    free(ipiv);
    free(b.w);
    return info;
}

/* Factor only, returning the working band (ld = 2kl+ku+1 when pivoting,
 * kl+ku+1 otherwise, U superdiagonals first) and the pivots; used by tests
 * that check the pivot invariants and reconstruct P A = L U. */
ORC_EXPORT int64_t orc_gbtrf(int64_t n, int kl, int ku, const double *ab,
                             int64_t ldab, int pivot, double *w_out,
                             int64_t *ipiv_out) {
    work_band b;
    if (make_work_band(&b, n, kl, ku, ab, ldab, pivot)) return -100;
    int64_t info = pivot ? lu_piv(&b, ipiv_out) : lu_nopiv(&b);
    if (!pivot && ipiv_out)
        for (int64_t j = 0; j < n; ++j) ipiv_out[j] = j;
    memcpy(w_out, b.w, (size_t)(b.ldw * n) * sizeof(double));
    free(b.w);
    return info;
}

/* Solve op(A) X = F in place on B with the factors orc_gbtrf returned (w:
 * working band of ld 2kl+ku+1 when pivoting, else kl+ku+1; ipiv: its
 * pivots), the same substitutions as orc_gbsv.  Lets a caller time the
 * factorisation and the solves apart. */
ORC_EXPORT void orc_gbtrs(int64_t n, int kl, int ku, const double *w,
                          const int64_t *ipiv, int pivot, int trans, int nrhs,
                          double *B, int64_t ldb) {
    work_band b;
    b.n = n;
    b.kl = kl;
    b.uw = pivot ? kl + ku : ku;
    b.ldw = (int64_t)kl + b.uw + 1;
    b.w = (double *)w;
    for (int c = 0; c < nrhs; ++c) {
        if (trans) solve_t(&b, pivot ? ipiv : NULL, B + (int64_t)c * ldb);
        else       solve_n(&b, pivot ? ipiv : NULL, B + (int64_t)c * ldb);
    }
}

/* Y = op(A) X (trans 0: A, 1: A^T), plain summation in index order. */
ORC_EXPORT void orc_gbmv(int64_t n, int kl, int ku, const double *ab,
                         int64_t ldab, int trans, int nrhs, const double *X,
                         int64_t ldx, double *Y, int64_t ldy) {
    for (int c = 0; c < nrhs; ++c) {
        const double *x = X + (int64_t)c * ldx;
        double *y = Y + (int64_t)c * ldy;
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            if (!trans) {
                for (int64_t j = imax64(0, i - kl); j <= imin64(n - 1, i + ku); ++j)
                    s += ab[(ku + i - j) + j * ldab] * x[j];
            } else {
                for (int64_t j = imax64(0, i - ku); j <= imin64(n - 1, i + kl); ++j)
                    s += ab[(ku + j - i) + i * ldab] * x[j];
            }
            y[i] = s;
        }
    }
}

/* ||A||_inf (max row abs-sum) when which = 0, ||A||_1 (max column abs-sum)
 * when which = 1. */
ORC_EXPORT double orc_gbnorm(int64_t n, int kl, int ku, const double *ab,
                             int64_t ldab, int which) {
    double best = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        if (which == 0) {
            for (int64_t j = imax64(0, i - kl); j <= imin64(n - 1, i + ku); ++j)
                s += fabs(ab[(ku + i - j) + j * ldab]);
        } else {
            for (int64_t r = imax64(0, i - ku); r <= imin64(n - 1, i + kl); ++r)
                s += fabs(ab[(ku + r - i) + i * ldab]);
        }
        if (s > best) best = s;
    }
    return best;
}

/* Relative residual max_c ||F_c - op(A) X_c||_inf / (||A||_inf ||X_c||_inf)
 * with each residual entry accumulated by Kahan-compensated summation. */
ORC_EXPORT double orc_relres(int64_t n, int kl, int ku, const double *ab,
                             int64_t ldab, int trans, int nrhs,
                             const double *X, int64_t ldx, const double *F,
                             int64_t ldf) {
    double anorm = orc_gbnorm(n, kl, ku, ab, ldab, trans ? 1 : 0);
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double *x = X + (int64_t)c * ldx;
        const double *f = F + (int64_t)c * ldf;
        double rmax = 0.0, xmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double s = f[i], comp = 0.0;
            int64_t lo = trans ? imax64(0, i - ku) : imax64(0, i - kl);
            int64_t hi = trans ? imin64(n - 1, i + kl) : imin64(n - 1, i + ku);
            for (int64_t j = lo; j <= hi; ++j) {
                double a = trans ? ab[(ku + j - i) + i * ldab]
                                 : ab[(ku + i - j) + j * ldab];
                double term = -(a * x[j]) - comp;
                double t = s + term;
                comp = (t - s) - term;
                s = t;
            }
            if (fabs(s) > rmax) rmax = fabs(s);
            if (fabs(x[i]) > xmax) xmax = fabs(x[i]);
        }
        double denom = anorm * xmax;
        double rel = denom > 0.0 ? rmax / denom : (rmax > 0.0 ? INFINITY : 0.0);
        if (rel > worst) worst = rel;
    }
    return worst;
}

/* 1-norm condition estimate kappa_1(A) ~ ||A||_1 ||A^{-1}||_1, with
 * ||A^{-1}||_1 from Hager's (1984) power-type estimator as refined by Higham
 * (1988): at most five sign-vector iterations plus Higham's alternating
 * test vector.  Uses the pivoting LU.  Returns -1 on a singular factor. */
ORC_EXPORT double orc_gbcond1(int64_t n, int kl, int ku, const double *ab,
                              int64_t ldab) {
    if (n == 0) return 0.0;
    work_band b;
    if (make_work_band(&b, n, kl, ku, ab, ldab, 1)) return -1.0;
    int64_t *ipiv = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (lu_piv(&b, ipiv) != 0) { free(ipiv); free(b.w); return -1.0; }
    double *x = (double *)malloc((size_t)n * sizeof(double));
    double *y = (double *)malloc((size_t)n * sizeof(double));
    double *z = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
    double est = 0.0;
    for (int it = 0; it < 5; ++it) {
        memcpy(y, x, (size_t)n * sizeof(double));
        solve_n(&b, ipiv, y);                     /* y = A^{-1} x           */
        double nrm1 = 0.0;
        for (int64_t i = 0; i < n; ++i) nrm1 += fabs(y[i]);
        if (it > 0 && nrm1 <= est) break;         /* no further increase    */
        est = nrm1;
        for (int64_t i = 0; i < n; ++i) z[i] = y[i] >= 0.0 ? 1.0 : -1.0;
        solve_t(&b, ipiv, z);                     /* z = A^{-T} sign(y)     */
        int64_t jmax = 0;
        double ztx = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (fabs(z[i]) > fabs(z[jmax])) jmax = i;
            ztx += z[i] * x[i];
        }
        if (it > 0 && fabs(z[jmax]) <= ztx) break; /* Hager's stopping test */
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        x[jmax] = 1.0;
    }
    /* Higham's extra test vector b_i = (-1)^i (1 + i/(n-1)). */
    for (int64_t i = 0; i < n; ++i) {
        double mag = 1.0 + (n > 1 ? (double)i / (double)(n - 1) : 0.0);
        y[i] = (i % 2 == 0) ? mag : -mag;
    }
    solve_n(&b, ipiv, y);
    double alt = 0.0;
    for (int64_t i = 0; i < n; ++i) alt += fabs(y[i]);
    alt = 2.0 * alt / (3.0 * (double)n);
    if (alt > est) est = alt;
    double anorm = orc_gbnorm(n, kl, ku, ab, ldab, 1);
    free(x); free(y); free(z); free(ipiv); free(b.w);
    return anorm * est;
}

/* Load-balancing ratio of the load-balancing section: with r = nrhs/k and
 * K = K2/K1, R13 = n1/n3 = 1/(1 + K r) + (3/2 + 2 r)/(1/K + r); R12 = R13/2
 * (two-thread inner partitions are twice the size of single-thread ones). */
ORC_EXPORT double orc_r13(double K, double nrhs_over_k) {
    double r = nrhs_over_k;
    return 1.0 / (1.0 + K * r) + (1.5 + 2.0 * r) / (1.0 / K + r);
}

/* ------------------------------------------------------------------------ */
/* Complex bands (double complex; the library's interleaved re/im layout is  */
/* the memory layout of a double complex array): the same textbook banded   */
/* elimination in complex arithmetic.  Partial pivoting takes the first row  */
/* of maximal |Re| + |Im| among rows j..j+kl (LAPACK's choice for complex    */
/* pivots).                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    int kl, uw;
    int64_t ldw;
    double complex *w;
} zwork_band;

static double complex *zref(const zwork_band *b, int64_t i, int64_t j) {
    return &b->w[(b->uw + i - j) + j * b->ldw];
}

static double cabs1(double complex z) { return fabs(creal(z)) + fabs(cimag(z)); }

static int make_zwork_band(zwork_band *b, int64_t n, int kl, int ku,
                           const double complex *ab, int64_t ldab, int pivot) {
    b->n = n;
    b->kl = kl;
    b->uw = pivot ? kl + ku : ku;
    b->ldw = (int64_t)kl + b->uw + 1;
    b->w = (double complex *)calloc((size_t)(b->ldw * (n > 0 ? n : 1)), sizeof(double complex));
    if (!b->w) return -1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = imax64(0, j - ku); i <= imin64(n - 1, j + kl); ++i)
            *zref(b, i, j) = ab[(ku + i - j) + j * ldab];
    return 0;
}

static int64_t zlu(zwork_band *b, int64_t *ipiv) {
    const int64_t n = b->n;
    int64_t info = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t last_row = imin64(n - 1, j + b->kl);
        int64_t last_col = imin64(n - 1, j + b->uw);
        if (ipiv) {
            int64_t r = j;
            double best = cabs1(*zref(b, j, j));
            for (int64_t i = j + 1; i <= last_row; ++i) {
                double v = cabs1(*zref(b, i, j));
                if (v > best) { best = v; r = i; }
            }
            ipiv[j] = r;
            if (*zref(b, r, j) == 0.0) {
                if (info == 0) info = j + 1;
                continue;
            }
            if (r != j)
                for (int64_t c = j; c <= last_col; ++c) {
                    double complex t = *zref(b, j, c);
                    *zref(b, j, c) = *zref(b, r, c);
                    *zref(b, r, c) = t;
                }
        } else if (*zref(b, j, j) == 0.0) {
            return j + 1;
        }
        double complex piv = *zref(b, j, j);
        for (int64_t i = j + 1; i <= last_row; ++i) {
            double complex l = *zref(b, i, j) / piv;
            *zref(b, i, j) = l;
            for (int64_t c = j + 1; c <= last_col; ++c)
                *zref(b, i, c) -= l * *zref(b, j, c);
        }
    }
    return info;
}

/* x <- op(A)^{-1} x; trans 0: A, 1: A^T, 2: A^H. */
static void zsolve(const zwork_band *b, const int64_t *ipiv, int trans, double complex *x) {
    const int64_t n = b->n;
    if (trans == 0) {
        for (int64_t j = 0; j < n; ++j) {
            if (ipiv && ipiv[j] != j) { double complex t = x[j]; x[j] = x[ipiv[j]]; x[ipiv[j]] = t; }
            for (int64_t i = j + 1; i <= imin64(n - 1, j + b->kl); ++i)
                x[i] -= *zref(b, i, j) * x[j];
        }
        for (int64_t j = n - 1; j >= 0; --j) {
            x[j] /= *zref(b, j, j);
            for (int64_t i = imax64(0, j - b->uw); i < j; ++i)
                x[i] -= *zref(b, i, j) * x[j];
        }
        return;
    }
    const int cj = trans == 2;
    for (int64_t j = 0; j < n; ++j) {
        double complex s = x[j];
        for (int64_t i = imax64(0, j - b->uw); i < j; ++i) {
            double complex u = *zref(b, i, j);
            s -= (cj ? conj(u) : u) * x[i];
        }
        double complex d = *zref(b, j, j);
        x[j] = s / (cj ? conj(d) : d);
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        double complex s = x[j];
        for (int64_t i = j + 1; i <= imin64(n - 1, j + b->kl); ++i) {
            double complex l = *zref(b, i, j);
            s -= (cj ? conj(l) : l) * x[i];
        }
        x[j] = s;
        if (ipiv && ipiv[j] != j) { double complex t = x[j]; x[j] = x[ipiv[j]]; x[ipiv[j]] = t; }
    }
}

/* Solve op(A) Z = F in place on B (complex n x nrhs, column-major, ldb >= n);
 * trans 0: A, 1: A^T, 2: A^H.  Returns 0, an argument error, or the 1-based
 * index of the first zero pivot (B untouched). */
ORC_EXPORT int64_t orc_zgbsv(int64_t n, int kl, int ku, const double complex *ab,
                             int64_t ldab, int pivot, int trans, int nrhs,
                             double complex *B, int64_t ldb) {
    if (n < 0) return -1;
    if (kl < 0) return -2;
    if (ku < 0) return -3;
    if (ldab < (int64_t)kl + ku + 1) return -5;
    if (trans < 0 || trans > 2) return -7;
    if (ldb < (n > 1 ? n : 1)) return -10;
    if (n == 0) return 0;
    zwork_band b;
    if (make_zwork_band(&b, n, kl, ku, ab, ldab, pivot)) return -100;
    int64_t *ipiv = pivot ? (int64_t *)malloc((size_t)n * sizeof(int64_t)) : NULL;
    int64_t info = zlu(&b, ipiv);
    if (info == 0)
        for (int c = 0; c < nrhs; ++c) zsolve(&b, ipiv, trans, B + (int64_t)c * ldb);
    free(ipiv);
    free(b.w);
    return info;
}

/* Y = op(A) X for complex bands (trans 0: A, 1: A^T, 2: A^H), plain
 * summation in index order. */
ORC_EXPORT void orc_zgbmv(int64_t n, int kl, int ku, const double complex *ab,
                          int64_t ldab, int trans, int nrhs, const double complex *X,
                          int64_t ldx, double complex *Y, int64_t ldy) {
    for (int c = 0; c < nrhs; ++c) {
        const double complex *x = X + (int64_t)c * ldx;
        double complex *y = Y + (int64_t)c * ldy;
        for (int64_t i = 0; i < n; ++i) {
            double complex s = 0.0;
            if (trans == 0) {
                for (int64_t j = imax64(0, i - kl); j <= imin64(n - 1, i + ku); ++j)
                    s += ab[(ku + i - j) + j * ldab] * x[j];
            } else {
                for (int64_t j = imax64(0, i - ku); j <= imin64(n - 1, i + kl); ++j) {
                    double complex a = ab[(ku + j - i) + i * ldab];
                    s += (trans == 2 ? conj(a) : a) * x[j];
                }
            }
            y[i] = s;
        }
    }
}

/* max_c ||F_c - op(A) Z_c||_inf / (||op(A)||_inf ||Z_c||_inf) with the
 * modulus as the entry norm; residual entries with compensated summation of
 * the real and imaginary parts. */
ORC_EXPORT double orc_zrelres(int64_t n, int kl, int ku, const double complex *ab,
                              int64_t ldab, int trans, int nrhs,
                              const double complex *X, int64_t ldx,
                              const double complex *F, int64_t ldf) {
    double anorm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        if (trans == 0)
            for (int64_t j = imax64(0, i - kl); j <= imin64(n - 1, i + ku); ++j)
                s += cabs(ab[(ku + i - j) + j * ldab]);
        else
            for (int64_t j = imax64(0, i - ku); j <= imin64(n - 1, i + kl); ++j)
                s += cabs(ab[(ku + j - i) + i * ldab]);
        if (s > anorm) anorm = s;
    }
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
        const double complex *x = X + (int64_t)c * ldx;
        const double complex *f = F + (int64_t)c * ldf;
        double rmax = 0.0, xmax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double sr = creal(f[i]), si = cimag(f[i]), cr = 0.0, ci = 0.0;
            int64_t lo = trans ? imax64(0, i - ku) : imax64(0, i - kl);
            int64_t hi = trans ? imin64(n - 1, i + kl) : imin64(n - 1, i + ku);
            for (int64_t j = lo; j <= hi; ++j) {
                double complex a = trans ? ab[(ku + j - i) + i * ldab] : ab[(ku + i - j) + j * ldab];
                if (trans == 2) a = conj(a);
                double complex p = a * x[j];
                double tr = -creal(p) - cr, t = sr + tr;
                cr = (t - sr) - tr; sr = t;
                double ti = -cimag(p) - ci, u = si + ti;
                ci = (u - si) - ti; si = u;
            }
            double r = hypot(sr, si);
            if (r > rmax) rmax = r;
            if (cabs(x[i]) > xmax) xmax = cabs(x[i]);
        }
        double denom = anorm * xmax;
        double rel = denom > 0.0 ? rmax / denom : (rmax > 0.0 ? INFINITY : 0.0);
        if (rel > worst) worst = rel;
    }
    return worst;
}
