/* Matrix-free FP64 products with the FBIE matrices, for sizes where the dense
 * matrices do not fit in memory.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it (through oracle/mf.py).
 *
 * Every entry of the kernel matrix is evaluated from its definition, one row
 * at a time, and used right away:
 *
 *   K_ij = (2/n) (A_i/A_j) eta'_j / (eta_j - eta_i),   i != j,   K_ii = 0,
 *
 * the trapezoidal weight 2 pi/n times the kernels of eqs. (e:N) and (e:M):
 * B_ij = (2 pi/n) N(t_i,t_j) = Im K_ij (matrix B of eq. (e:B)) and
 * D_ij = (2 pi/n) M(t_i,t_j) = Re K_ij (the matrix D of Sec. 3.3).
 * No Cauchy-matrix factorisation (eqs. (e:hD-bt), (e:(I-B)x)) is used: the
 * ratio A_i/A_j and eta'_j stay inside each entry.
 *
 * For columns x (column-major, leading dimension N) the library returns
 *   trans = 0:  ya = (2I + diag(B1) - B) x       (eq. (e:sys))
 *               yc = (D - diag(D1)) x            (the non-circulant part of (e:y), (e:bh))
 *   trans = 1:  ya = (2I + diag(B1) - B^T) x,   yc = (D^T - diag(D1)) x.
 * The block-diagonal circulant part Lhat of (e:y) is added by the caller.
 * Row i gives (B1)_i and (D1)_i; for trans = 0 it is multiplied with x
 * ((Bx)_i = sum_j B_ij x_j; with several columns the rows are taken in blocks
 * of RB so that each x_j is read once per block), for trans = 1 it is
 * scattered ((B^T x)_j += B_ij x_i) into per-thread sums added at the end.
 * Complex inputs are split into real and imaginary arrays of length N.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

enum { RB = 16 };   /* rows per block for products with several columns */

/* Row i of K: kr[j] + i ki[j] = K_ij for j = 0..N-1 (K_ii = 0). */
static void kernel_row(int64_t N, int n, int64_t i, const double* er, const double* ei, const double* pr,
                       const double* pi, const double* ar, const double* ai, double* kr, double* ki)
{
    const double w = 2.0 / n;
    const double eir = er[i], eii = ei[i], air = ar[i], aii = ai[i];
#pragma omp simd
    for (int64_t j = 0; j < N; ++j) {
        /* numerator A_i eta'_j, denominator A_j (eta_j - eta_i) */
        double dr = er[j] - eir, di = ei[j] - eii;
        double nr = air * pr[j] - aii * pi[j], ni = air * pi[j] + aii * pr[j];
        double cr = ar[j] * dr - ai[j] * di, ci = ar[j] * di + ai[j] * dr;
        double s = (j == i) ? 0.0 : w / (cr * cr + ci * ci);     /* K_ii = 0 */
        kr[j] = (nr * cr + ni * ci) * s;
        ki[j] = (ni * cr - nr * ci) * s;
    }
}

enum { SB = 256 };   /* block length of the sums of the one-column product */

/* Neumaier's compensated addition: s + c holds the running sum to about twice
   the working precision */
static inline void csum(double* s, double* c, double y)
{
    const double t = *s + y;
    *c += (fabs(*s) >= fabs(y)) ? ((*s - t) + y) : ((y - t) + *s);
    *s = t;
}

static double total(int64_t N, const double* a)
{
    double s = 0.0;
#pragma omp simd reduction(+ : s)
    for (int64_t j = 0; j < N; ++j) s += a[j];
    return s;
}

static double dot(int64_t N, const double* a, const double* b)
{
    double s = 0.0;
#pragma omp simd reduction(+ : s)
    for (int64_t j = 0; j < N; ++j) s += a[j] * b[j];
    return s;
}

static void axpy(int64_t N, double a, const double* x, double* y)
{
#pragma omp simd
    for (int64_t j = 0; j < N; ++j) y[j] += a * x[j];
}

int gnk_oracle_fbie_rows(int64_t N, int n, int64_t i0, int64_t i1, const double* er, const double* ei,
                         const double* pr, const double* pi, const double* ar, const double* ai, int ncols,
                         const double* x, int trans, double* ya, double* yc, int nthreads);

/* Returns 0, or -1 when a buffer cannot be allocated. nthreads <= 0: OpenMP's default. */
int gnk_oracle_fbie_ops(int64_t N, int n, const double* er, const double* ei, const double* pr, const double* pi,
                        const double* ar, const double* ai, int ncols, const double* x, int trans, double* ya,
                        double* yc, int nthreads)
{
    return gnk_oracle_fbie_rows(N, n, 0, N, er, ei, pr, pi, ar, ai, ncols, x, trans, ya, yc, nthreads);
}

/* The same for the rows i0..i1-1 of the products only (trans = 0; the other
 * entries of ya and yc are not written), or for all rows (trans = 1 needs
 * i0 = 0, i1 = N). Returns -2 for a bad range. */
int gnk_oracle_fbie_rows(int64_t N, int n, int64_t i0, int64_t i1, const double* er, const double* ei,
                         const double* pr, const double* pi, const double* ar, const double* ai, int ncols,
                         const double* x, int trans, double* ya, double* yc, int nthreads)
{
    if (i0 < 0 || i1 > N || i0 > i1 || (trans && (i0 != 0 || i1 != N))) return -2;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    const int nt = omp_get_max_threads();
    const int64_t cols = ncols;
    double* rowB = (double*)malloc(sizeof(double) * (size_t)N * 2);
    double* rowD = rowB ? rowB + N : NULL;
    /* per thread: kernel rows (2N each; RB of them for several columns without trans), the block's
       sums (2 RB cols), and for trans the partial sums of B^T x and D^T x (2N per column) */
    const int64_t rows = (cols > 1 && !trans) ? RB : 1;
    const int64_t per = 2 * N * rows + 2 * RB * cols + (trans ? 2 * N * cols : 0);
    double* work = (double*)calloc((size_t)per * nt, sizeof(double));
    /* several columns without trans: x row by row (x^T, N x cols), so that the block reads x_j once */
    double* xt = (cols > 1 && !trans) ? (double*)malloc(sizeof(double) * (size_t)(N * cols)) : NULL;
    if (!rowB || !work || (cols > 1 && !trans && !xt)) {
        free(rowB);
        free(work);
        free(xt);
        return -1;
    }
    if (xt)
        for (int64_t j = 0; j < N; ++j)
            for (int64_t c = 0; c < cols; ++c) xt[j * cols + c] = x[c * N + j];
#pragma omp parallel num_threads(nt)
    {
        double* kr = work + per * omp_get_thread_num();   /* rows of Re K, N apart */
        double* ki = kr + N * rows;                        /* rows of Im K */
        double* acc = ki + N * rows;                        /* block sums: B x (RB x cols), then D x */
        double* sb = acc + 2 * RB * cols; /* trans: this thread's sum of B_ij x_i over its rows i, per column */
        double* sd = sb + N * cols;       /* trans: the same for D */
        if (cols > 1 && !trans) {
            /* several columns: rows in blocks of RB, each input row x_j read once per block */
#pragma omp for schedule(dynamic, 1)
            for (int64_t b0 = i0; b0 < i1; b0 += RB) {
                const int64_t nb = (i1 - b0 < RB) ? i1 - b0 : RB;
                for (int64_t r = 0; r < nb; ++r) {
                    kernel_row(N, n, b0 + r, er, ei, pr, pi, ar, ai, kr + r * N, ki + r * N);
                    rowB[b0 + r] = total(N, ki + r * N);
                    rowD[b0 + r] = total(N, kr + r * N);
                }
                double* ab = acc;
                double* ad = acc + RB * cols;
                memset(acc, 0, sizeof(double) * 2 * RB * cols);
                for (int64_t j = 0; j < N; ++j) {
                    const double* xj = xt + j * cols;
                    for (int64_t r = 0; r < nb; ++r) {
                        const double b = ki[r * N + j], d = kr[r * N + j];
                        double* abr = ab + r * cols;
                        double* adr = ad + r * cols;
#pragma omp simd
                        for (int64_t c = 0; c < cols; ++c) {
                            abr[c] += b * xj[c];     /* (B x)_i */
                            adr[c] += d * xj[c];     /* (D x)_i */
                        }
                    }
                }
                for (int64_t r = 0; r < nb; ++r)
                    for (int64_t c = 0; c < cols; ++c) {
                        ya[c * N + b0 + r] = ab[r * cols + c];
                        yc[c * N + b0 + r] = ad[r * cols + c];
                    }
            }
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = i0; i < (cols > 1 && !trans ? i0 : i1); ++i) {
            if (cols == 1 && !trans) {
                /* one column: the same entries, used in the loop that forms them; each of
                   the four sums over j is taken in blocks of SB terms whose partial sums are
                   added with compensation (Neumaier), so that the rounding of the sum grows
                   with the block length, not with N */
                const double w = 2.0 / n;
                const double eir = er[i], eii = ei[i], air = ar[i], aii = ai[i];
                double t1 = 0.0, e1 = 0.0, t2 = 0.0, e2 = 0.0, t3 = 0.0, e3 = 0.0, t4 = 0.0, e4 = 0.0;
                for (int64_t j0 = 0; j0 < N; j0 += SB) {
                    const int64_t j1 = (j0 + SB < N) ? j0 + SB : N;
                    double b1 = 0.0, d1 = 0.0, bx = 0.0, dx = 0.0;
#pragma omp simd reduction(+ : b1, d1, bx, dx)
                    for (int64_t j = j0; j < j1; ++j) {
                        double dr = er[j] - eir, di = ei[j] - eii;
                        double nr = air * pr[j] - aii * pi[j], ni = air * pi[j] + aii * pr[j];
                        double cr = ar[j] * dr - ai[j] * di, ci = ar[j] * di + ai[j] * dr;
                        double q = (j == i) ? 0.0 : w / (cr * cr + ci * ci);   /* K_ii = 0 */
                        double kre = (nr * cr + ni * ci) * q, kim = (ni * cr - nr * ci) * q;
                        b1 += kim;
                        d1 += kre;
                        bx += kim * x[j];            /* (B x)_i */
                        dx += kre * x[j];            /* (D x)_i */
                    }
                    csum(&t1, &e1, b1);
                    csum(&t2, &e2, d1);
                    csum(&t3, &e3, bx);
                    csum(&t4, &e4, dx);
                }
                rowB[i] = t1 + e1;
                rowD[i] = t2 + e2;
                ya[i] = t3 + e3;
                yc[i] = t4 + e4;
                continue;
            }
            if (cols == 1) {
                /* one column, transposed: the same entries, scattered in the loop that forms them */
                const double w = 2.0 / n;
                const double eir = er[i], eii = ei[i], air = ar[i], aii = ai[i], xi = x[i];
                double b1 = 0.0, d1 = 0.0, bx = 0.0, dx = 0.0;
#pragma omp simd reduction(+ : b1, d1, bx, dx)
                for (int64_t j = 0; j < N; ++j) {
                    double dr = er[j] - eir, di = ei[j] - eii;
                    double nr = air * pr[j] - aii * pi[j], ni = air * pi[j] + aii * pr[j];
                    double cr = ar[j] * dr - ai[j] * di, ci = ar[j] * di + ai[j] * dr;
                    double s = (j == i) ? 0.0 : w / (cr * cr + ci * ci);     /* K_ii = 0 */
                    double kre = (nr * cr + ni * ci) * s, kim = (ni * cr - nr * ci) * s;
                    b1 += kim;
                    d1 += kre;
                    if (!trans) {
                        bx += kim * x[j];            /* (B x)_i */
                        dx += kre * x[j];            /* (D x)_i */
                    } else {
                        sb[j] += kim * xi;           /* (B^T x)_j += B_ij x_i */
                        sd[j] += kre * xi;           /* (D^T x)_j += D_ij x_i */
                    }
                }
                rowB[i] = b1;
                rowD[i] = d1;
                if (!trans) {
                    ya[i] = bx;
                    yc[i] = dx;
                }
                continue;
            }
            kernel_row(N, n, i, er, ei, pr, pi, ar, ai, kr, ki);
            rowB[i] = total(N, ki);     /* (B1)_i */
            rowD[i] = total(N, kr);     /* (D1)_i */
            for (int64_t c = 0; c < cols; ++c) {
                const double* xc = x + c * N;
                if (!trans) {
                    ya[c * N + i] = dot(N, ki, xc);      /* (B x)_i */
                    yc[c * N + i] = dot(N, kr, xc);      /* (D x)_i */
                } else {
                    axpy(N, xc[i], ki, sb + c * N);      /* (B^T x)_j += B_ij x_i */
                    axpy(N, xc[i], kr, sd + c * N);      /* (D^T x)_j += D_ij x_i */
                }
            }
        }
        if (trans) {
            /* add the threads' partial sums, each thread a range of rows j */
#pragma omp for schedule(static)
            for (int64_t j = 0; j < N; ++j)
                for (int64_t c = 0; c < cols; ++c) {
                    double b = 0.0, d = 0.0;
                    for (int t = 0; t < nt; ++t) {
                        const double* st = work + per * t + 2 * N * rows + 2 * RB * cols;
                        b += st[c * N + j];
                        d += st[N * cols + c * N + j];
                    }
                    ya[c * N + j] = b;
                    yc[c * N + j] = d;
                }
        }
    }
    /* ya = 2x + diag(B1) x - (B x or B^T x),  yc = (D x or D^T x) - diag(D1) x */
    for (int64_t c = 0; c < cols; ++c)
        for (int64_t i = i0; i < i1; ++i) {
            const double xi = x[c * N + i];
            ya[c * N + i] = 2.0 * xi + rowB[i] * xi - ya[c * N + i];
            yc[c * N + i] = yc[c * N + i] - rowD[i] * xi;
        }
    free(rowB);
    free(work);
    free(xt);
    return 0;
}

/* Rows [i0, i1) of K into kr, ki (row-major, (i1 - i0) x N): the same entries,
 * for checks of single rows and for the CPU baseline's timed sample. */
void gnk_oracle_kernel_rows(int64_t N, int n, int64_t i0, int64_t i1, const double* er, const double* ei,
                            const double* pr, const double* pi, const double* ar, const double* ai, double* kr,
                            double* ki, int nthreads)
{
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = i0; i < i1; ++i)
        kernel_row(N, n, i, er, ei, pr, pi, ar, ai, kr + (i - i0) * N, ki + (i - i0) * N);
}

int gnk_oracle_max_threads(void) { return omp_get_max_threads(); }
