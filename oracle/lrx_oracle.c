/*
 * lrx oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, full-recompute reference for the low-rank determinant and
 * Pfaffian update library.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's shared object; the product
 * path never does.  It shares no code with the GPU path.
 *
 * Everything is computed from scratch in IEEE double (real) or double complex,
 * compiled with -ffp-contract=off so that results do not depend on FMA
 * contraction:
 *
 *   - determinant, log|det| and phase by Gaussian elimination with partial
 *     pivoting (pivot = largest modulus in the column, ties -> lowest row).
 *     The low-rank ratio of the paper (matrix determinant lemma, Sec. II.A,
 *     Eqs. det_ratio/det_R) equals det(A_t)/det(A_{t-1}) exactly in exact
 *     arithmetic, so the oracle recomputes both determinants.
 *   - inverse by solving A X = I with the same factorisation (Sherman-Morrison
 *     Eq. det_inv and the Pfaffian Woodbury Eq. pf_inv are identities for it).
 *   - Pfaffian, log|pf| and phase by Parlett-Reid elimination: a congruence
 *     pf(B A B^T) = det(B) pf(A) (Appendix A, Eq. pf->det_pf) that moves the
 *     largest entry of the leading column to position (1,0) and then a block
 *     Schur step (Appendix A, Eq. pf_block) that splits off the leading 2x2
 *     block, whose Pfaffian is its (0,1) entry (Appendix A, 2x2 example).
 *
 * Pins (checked by the CPU tests): Leibniz permutation sums, perfect-matching
 * sums (Appendix A, Eq. pf_def), the 2x2 and 4x4 closed forms, pf^2 = det,
 * pf(B A B^T) = det(B) pf(A), LAPACK slogdet/inv, exact rational elimination.
 *
 * Layout: matrices are row-major, n x n, batch-contiguous.  Complex values are
 * interleaved (re, im) doubles.  Phases are returned as (re, im) pairs for the
 * complex routines and as +-1 (re only) for the real ones.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zdouble;

/* ------------------------------------------------------------------------ */
/* Real LU with partial pivoting: in-place on a (n x n), returns the pivot  */
/* rows and the number of row swaps.  Returns 0 if a zero pivot appeared.   */
/* ------------------------------------------------------------------------ */
static int lu_real(int n, double *a, int *piv, int *nswap)
{
    int ok = 1;
    *nswap = 0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = fabs(a[(size_t)j * n + j]);
        for (int i = j + 1; i < n; ++i) {
            double v = fabs(a[(size_t)i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        piv[j] = p;
        if (p != j) {
            for (int c = 0; c < n; ++c) {
                double t = a[(size_t)j * n + c];
                a[(size_t)j * n + c] = a[(size_t)p * n + c];
                a[(size_t)p * n + c] = t;
            }
            ++*nswap;
        }
        double d = a[(size_t)j * n + j];
        if (d == 0.0) { ok = 0; continue; }
        for (int i = j + 1; i < n; ++i) {
            double l = a[(size_t)i * n + j] / d;
            a[(size_t)i * n + j] = l;
            for (int c = j + 1; c < n; ++c)
                a[(size_t)i * n + c] -= l * a[(size_t)j * n + c];
        }
    }
    return ok;
}

static int lu_cplx(int n, zdouble *a, int *piv, int *nswap)
{
    int ok = 1;
    *nswap = 0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = cabs(a[(size_t)j * n + j]);
        for (int i = j + 1; i < n; ++i) {
            double v = cabs(a[(size_t)i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        piv[j] = p;
        if (p != j) {
            for (int c = 0; c < n; ++c) {
                zdouble t = a[(size_t)j * n + c];
                a[(size_t)j * n + c] = a[(size_t)p * n + c];
                a[(size_t)p * n + c] = t;
            }
            ++*nswap;
        }
        zdouble d = a[(size_t)j * n + j];
        if (d == 0.0) { ok = 0; continue; }
        for (int i = j + 1; i < n; ++i) {
            zdouble l = a[(size_t)i * n + j] / d;
            a[(size_t)i * n + j] = l;
            for (int c = j + 1; c < n; ++c)
                a[(size_t)i * n + c] -= l * a[(size_t)j * n + c];
        }
    }
    return ok;
}

/* Solve (P A) X = P I column by column from the packed LU; X row-major.     */
static void lu_inverse_real(int n, const double *lu, const int *piv, double *x)
{
    double *col = (double *)malloc(sizeof(double) * n);
    for (int e = 0; e < n; ++e) {
        for (int i = 0; i < n; ++i) col[i] = (i == e) ? 1.0 : 0.0;
        for (int j = 0; j < n; ++j) {           /* apply the row swaps */
            int p = piv[j];
            if (p != j) { double t = col[j]; col[j] = col[p]; col[p] = t; }
        }
        for (int i = 0; i < n; ++i) {           /* L y = P e, unit diagonal */
            double s = col[i];
            for (int c = 0; c < i; ++c) s -= lu[(size_t)i * n + c] * col[c];
            col[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {      /* U x = y */
            double s = col[i];
            for (int c = i + 1; c < n; ++c) s -= lu[(size_t)i * n + c] * col[c];
            col[i] = s / lu[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) x[(size_t)i * n + e] = col[i];
    }
    free(col);
}

static void lu_inverse_cplx(int n, const zdouble *lu, const int *piv, zdouble *x)
{
    zdouble *col = (zdouble *)malloc(sizeof(zdouble) * n);
    for (int e = 0; e < n; ++e) {
        for (int i = 0; i < n; ++i) col[i] = (i == e) ? 1.0 : 0.0;
        for (int j = 0; j < n; ++j) {
            int p = piv[j];
            if (p != j) { zdouble t = col[j]; col[j] = col[p]; col[p] = t; }
        }
        for (int i = 0; i < n; ++i) {
            zdouble s = col[i];
            for (int c = 0; c < i; ++c) s -= lu[(size_t)i * n + c] * col[c];
            col[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            zdouble s = col[i];
            for (int c = i + 1; c < n; ++c) s -= lu[(size_t)i * n + c] * col[c];
            col[i] = s / lu[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) x[(size_t)i * n + e] = col[i];
    }
    free(col);
}

/*
 * Batched log|det|, phase and (optionally) inverse.
 *   cplx  : 0 -> double, 1 -> double complex (interleaved)
 *   a     : [batch][n][n] input, not modified
 *   logabs: [batch]; -inf for a singular matrix
 *   phase : [batch][2] (re, im); (0,0) for a singular matrix
 *   inv   : [batch][n][n] (same element type) or NULL; NaN-filled if singular
 * Returns the number of singular matrices.
 */
int orc_slogdet(int cplx, int batch, int n, const double *a, double *logabs,
                double *phase, double *inv)
{
    int nsing = 0;
    size_t nn = (size_t)n * n;
#pragma omp parallel for schedule(dynamic) reduction(+ : nsing)
    for (int b = 0; b < batch; ++b) {
        int *piv = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
        int nswap = 0;
        if (!cplx) {
            double *lu = (double *)malloc(sizeof(double) * (nn ? nn : 1));
            memcpy(lu, a + b * nn, sizeof(double) * nn);
            int ok = lu_real(n, lu, piv, &nswap);
            double la = 0.0, sg = (nswap & 1) ? -1.0 : 1.0;
            for (int j = 0; j < n; ++j) {
                double d = lu[(size_t)j * n + j];
                la += log(fabs(d));
                if (d < 0) sg = -sg;
            }
            if (!ok) { la = -INFINITY; sg = 0.0; ++nsing; }
            logabs[b] = la;
            phase[2 * b] = sg;
            phase[2 * b + 1] = 0.0;
            if (inv) {
                double *x = inv + b * nn;
                if (ok) lu_inverse_real(n, lu, piv, x);
                else for (size_t t = 0; t < nn; ++t) x[t] = NAN;
            }
            free(lu);
        } else {
            zdouble *lu = (zdouble *)malloc(sizeof(zdouble) * (nn ? nn : 1));
            memcpy(lu, a + 2 * b * nn, sizeof(zdouble) * nn);
            int ok = lu_cplx(n, lu, piv, &nswap);
            double la = 0.0;
            zdouble ph = (nswap & 1) ? -1.0 : 1.0;
            for (int j = 0; j < n; ++j) {
                zdouble d = lu[(size_t)j * n + j];
                double m = cabs(d);
                la += log(m);
                if (m > 0) ph *= d / m;
            }
            if (!ok) { la = -INFINITY; ph = 0.0; ++nsing; }
            logabs[b] = la;
            phase[2 * b] = creal(ph);
            phase[2 * b + 1] = cimag(ph);
            if (inv) {
                zdouble *x = (zdouble *)(inv + 2 * b * nn);
                if (ok) lu_inverse_cplx(n, lu, piv, x);
                else for (size_t t = 0; t < nn; ++t) x[t] = NAN;
            }
            free(lu);
        }
        free(piv);
    }
    return nsing;
}

/* ------------------------------------------------------------------------ */
/* Parlett-Reid Pfaffian.                                                   */
/*                                                                          */
/* For j = 0, 2, 4, ...:                                                    */
/*   1. p = the row i > j with the largest |a[i][j]| (ties -> lowest i).    */
/*   2. if p != j+1, exchange rows and columns j+1 and p: a congruence by a */
/*      transposition, which flips the sign of the Pfaffian.                */
/*   3. alpha = a[j][j+1] is the Pfaffian of the leading 2x2 block.         */
/*   4. Schur step: with c = a[j][j+2:] / alpha and w = a[j+1][j+2:],       */
/*      the trailing block becomes A22 + w c^T - c w^T; its Pfaffian times  */
/*      alpha is the Pfaffian of the current matrix.                        */
/* A zero alpha means the whole column is zero below the diagonal, so the  */
/* Pfaffian is zero.  An odd dimension has zero Pfaffian by definition.     */
/* ------------------------------------------------------------------------ */
static void slogpf_real(int n, double *a, double *logabs, double *sign)
{
    double la = 0.0, sg = 1.0;
    if (n & 1) { *logabs = -INFINITY; *sign = 0.0; return; }
    for (int j = 0; j + 1 < n; j += 2) {
        int p = j + 1;
        double best = fabs(a[(size_t)(j + 1) * n + j]);
        for (int i = j + 2; i < n; ++i) {
            double v = fabs(a[(size_t)i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        if (p != j + 1) {
            int q = j + 1;
            for (int c = 0; c < n; ++c) {       /* swap rows q, p */
                double t = a[(size_t)q * n + c];
                a[(size_t)q * n + c] = a[(size_t)p * n + c];
                a[(size_t)p * n + c] = t;
            }
            for (int r = 0; r < n; ++r) {       /* swap columns q, p */
                double t = a[(size_t)r * n + q];
                a[(size_t)r * n + q] = a[(size_t)r * n + p];
                a[(size_t)r * n + p] = t;
            }
            sg = -sg;
        }
        double alpha = a[(size_t)j * n + j + 1];
        if (alpha == 0.0) { *logabs = -INFINITY; *sign = 0.0; return; }
        la += log(fabs(alpha));
        if (alpha < 0) sg = -sg;
        for (int r = j + 2; r < n; ++r) {
            double cr = a[(size_t)j * n + r] / alpha;
            double wr = a[(size_t)(j + 1) * n + r];
            for (int s = j + 2; s < n; ++s) {
                double cs = a[(size_t)j * n + s] / alpha;
                double ws = a[(size_t)(j + 1) * n + s];
                a[(size_t)r * n + s] += wr * cs - cr * ws;
            }
        }
    }
    *logabs = la;
    *sign = sg;
}

static void slogpf_cplx(int n, zdouble *a, double *logabs, zdouble *phase)
{
    double la = 0.0;
    zdouble ph = 1.0;
    if (n & 1) { *logabs = -INFINITY; *phase = 0.0; return; }
    for (int j = 0; j + 1 < n; j += 2) {
        int p = j + 1;
        double best = cabs(a[(size_t)(j + 1) * n + j]);
        for (int i = j + 2; i < n; ++i) {
            double v = cabs(a[(size_t)i * n + j]);
            if (v > best) { best = v; p = i; }
        }
        if (p != j + 1) {
            int q = j + 1;
            for (int c = 0; c < n; ++c) {
                zdouble t = a[(size_t)q * n + c];
                a[(size_t)q * n + c] = a[(size_t)p * n + c];
                a[(size_t)p * n + c] = t;
            }
            for (int r = 0; r < n; ++r) {
                zdouble t = a[(size_t)r * n + q];
                a[(size_t)r * n + q] = a[(size_t)r * n + p];
                a[(size_t)r * n + p] = t;
            }
            ph = -ph;
        }
        zdouble alpha = a[(size_t)j * n + j + 1];
        if (alpha == 0.0) { *logabs = -INFINITY; *phase = 0.0; return; }
        double m = cabs(alpha);
        la += log(m);
        ph *= alpha / m;
        for (int r = j + 2; r < n; ++r) {
            zdouble cr = a[(size_t)j * n + r] / alpha;
            zdouble wr = a[(size_t)(j + 1) * n + r];
            for (int s = j + 2; s < n; ++s) {
                zdouble cs = a[(size_t)j * n + s] / alpha;
                zdouble ws = a[(size_t)(j + 1) * n + s];
                a[(size_t)r * n + s] += wr * cs - cr * ws;
            }
        }
    }
    *logabs = la;
    *phase = ph;
}

/*
 * Batched log|pf| and phase of skew-symmetric matrices (Appendix A).
 *   a: [batch][n][n] (double or interleaved complex), not modified.
 *   phase: [batch][2].  Odd n or a zero Pfaffian -> logabs = -inf, phase 0.
 * Returns the number of zero Pfaffians.
 */
int orc_slogpf(int cplx, int batch, int n, const double *a, double *logabs,
               double *phase)
{
    int nzero = 0;
    size_t nn = (size_t)n * n;
#pragma omp parallel for schedule(dynamic) reduction(+ : nzero)
    for (int b = 0; b < batch; ++b) {
        if (!cplx) {
            double *w = (double *)malloc(sizeof(double) * (nn ? nn : 1));
            memcpy(w, a + b * nn, sizeof(double) * nn);
            double sg;
            slogpf_real(n, w, &logabs[b], &sg);
            phase[2 * b] = sg;
            phase[2 * b + 1] = 0.0;
            if (sg == 0.0) ++nzero;
            free(w);
        } else {
            zdouble *w = (zdouble *)malloc(sizeof(zdouble) * (nn ? nn : 1));
            memcpy(w, a + 2 * b * nn, sizeof(zdouble) * nn);
            zdouble ph;
            slogpf_cplx(n, w, &logabs[b], &ph);
            phase[2 * b] = creal(ph);
            phase[2 * b + 1] = cimag(ph);
            if (ph == 0.0) ++nzero;
            free(w);
        }
    }
    return nzero;
}

/* Number of OpenMP threads the batched routines use (reported by the CPU   */
/* baseline).                                                               */
int orc_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
