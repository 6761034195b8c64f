/*
 * Oracle (test infrastructure only): one-sided (Hestenes) Jacobi SVD in plain
 * C, double precision, real and complex.  Nothing in the product path links or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it, through oracle/oracle.py.
 *
 * What it computes: the thin SVD A = U diag(s) V^H of one r x c matrix, which
 * is the per-face factorisation the truncated tensor SVD needs in step 3 of
 * the paper's Algorithm 1 (Sec. 3.1: "compute a tensor approximation"; the
 * paper allows any tensor approximation there, Sec. 3 remarks).  The SVD
 * itself is textbook linear algebra, not something the paper defines.
 *
 * Method (Hestenes 1958; Demmel & Veselic 1992): orthogonalise the columns of
 * the matrix with the fewer columns (A if r >= c, else A^H) by plane rotations
 * chosen from the 2x2 Gram matrix of each column pair, cyclic-by-row sweeps,
 * until a whole sweep performs no rotation or the sweep cap is hit.  Then the
 * singular values are the column norms, the left vectors the normalised
 * columns and the right vectors the accumulated rotations.  Output sorted by
 * decreasing singular value, ties kept in original column order.
 *
 * Storage: column major, leading dimension = number of rows.  Complex values
 * are interleaved (re, im) pairs, i.e. C99 double complex.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zd;

/* ------------------------------------------------------------------ real */

/* Orthogonalise the n columns (length len) of W in place; accumulate the
 * rotations into the n x n matrix V (initialised to I here).
 * Returns sweeps used, or -1 when the cap was reached without convergence. */
static int hestenes_d(int len, int n, double *W, double *V, int max_sweeps, double tol)
{
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i + (size_t)n * i] = 1.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int i = 0; i < n - 1; ++i) {
            for (int j = i + 1; j < n; ++j) {
                double *wi = W + (size_t)len * i, *wj = W + (size_t)len * j;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int t = 0; t < len; ++t) {
                    alpha += wi[t] * wi[t];
                    beta += wj[t] * wj[t];
                    gamma += wi[t] * wj[t];
                }
                if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
                rotated = 1;
                /* angle that zeroes the off-diagonal of [[alpha,gamma],[gamma,beta]] */
                double zeta = (beta - alpha) / (2.0 * gamma);
                double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
                for (int t = 0; t < len; ++t) {
                    double x = wi[t], y = wj[t];
                    wi[t] = cs * x - sn * y;
                    wj[t] = sn * x + cs * y;
                }
                double *vi = V + (size_t)n * i, *vj = V + (size_t)n * j;
                for (int t = 0; t < n; ++t) {
                    double x = vi[t], y = vj[t];
                    vi[t] = cs * x - sn * y;
                    vj[t] = sn * x + cs * y;
                }
            }
        }
        if (!rotated) return sweep;
    }
    return -1;
}

/* stable ordering by decreasing value */
static void order_desc(int n, const double *s, int *perm)
{
    for (int i = 0; i < n; ++i) perm[i] = i;
    for (int i = 1; i < n; ++i) { /* insertion sort keeps ties in place */
        int p = perm[i], j = i - 1;
        while (j >= 0 && s[perm[j]] < s[p]) { perm[j + 1] = perm[j]; --j; }
        perm[j + 1] = p;
    }
}

/* Thin SVD of the r x c real matrix A (lda >= r).  ns = min(r, c).
 * U: r x ns, s: ns, V: c x ns, all column major with leading dims r, -, c.
 * Returns sweeps used or -1 (not converged within max_sweeps). */
int oracle_svd_d(int r, int c, const double *A, int lda, double *U, double *s, double *V,
                 int max_sweeps, double tol)
{
    int tall = r >= c;
    int len = tall ? r : c, n = tall ? c : r;
    double *W = malloc(sizeof(double) * (size_t)len * n);
    double *R = malloc(sizeof(double) * (size_t)n * n);
    double *nrm = malloc(sizeof(double) * n);
    int *perm = malloc(sizeof(int) * n);
    for (int j = 0; j < n; ++j)
        for (int t = 0; t < len; ++t)
            W[t + (size_t)len * j] = tall ? A[t + (size_t)lda * j] : A[j + (size_t)lda * t];
    int sweeps = hestenes_d(len, n, W, R, max_sweeps, tol);
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int t = 0; t < len; ++t) acc += W[t + (size_t)len * j] * W[t + (size_t)len * j];
        nrm[j] = sqrt(acc);
    }
    order_desc(n, nrm, perm);
    /* tall: A V = W  => U = W/s (r x n), V = R (c x n)
       wide: A^T R = W => A = R diag(s) (W/s)^T  => U = R (r x n), V = W/s (c x n) */
    double *Wn = tall ? U : V;  /* normalised columns go here (len x n) */
    double *Rt = tall ? V : U;  /* rotations go here (n x n) */
    for (int jj = 0; jj < n; ++jj) {
        int j = perm[jj];
        s[jj] = nrm[j];
        double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
        for (int t = 0; t < len; ++t) Wn[t + (size_t)len * jj] = W[t + (size_t)len * j] * inv;
        for (int t = 0; t < n; ++t) Rt[t + (size_t)n * jj] = R[t + (size_t)n * j];
    }
    free(W); free(R); free(nrm); free(perm);
    return sweeps;
}

/* --------------------------------------------------------------- complex */

static int hestenes_z(int len, int n, zd *W, zd *V, int max_sweeps, double tol)
{
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i + (size_t)n * i] = 1.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int i = 0; i < n - 1; ++i) {
            for (int j = i + 1; j < n; ++j) {
                zd *wi = W + (size_t)len * i, *wj = W + (size_t)len * j;
                double alpha = 0.0, beta = 0.0;
                zd g = 0.0;
                for (int t = 0; t < len; ++t) {
                    alpha += creal(wi[t]) * creal(wi[t]) + cimag(wi[t]) * cimag(wi[t]);
                    beta += creal(wj[t]) * creal(wj[t]) + cimag(wj[t]) * cimag(wj[t]);
                    g += conj(wi[t]) * wj[t];
                }
                double ag = cabs(g);
                if (ag == 0.0 || ag <= tol * sqrt(alpha * beta)) continue;
                rotated = 1;
                /* w_j <- e^{-i phi} w_j makes the pair's Gram real, then a real
                   rotation; the combined 2x2 map is unitary */
                zd ph = conj(g) / ag; /* e^{-i phi} */
                double zeta = (beta - alpha) / (2.0 * ag);
                double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
                for (int t = 0; t < len; ++t) {
                    zd x = wi[t], y = wj[t] * ph;
                    wi[t] = cs * x - sn * y;
                    wj[t] = sn * x + cs * y;
                }
                zd *vi = V + (size_t)n * i, *vj = V + (size_t)n * j;
                for (int t = 0; t < n; ++t) {
                    zd x = vi[t], y = vj[t] * ph;
                    vi[t] = cs * x - sn * y;
                    vj[t] = sn * x + cs * y;
                }
            }
        }
        if (!rotated) return sweep;
    }
    return -1;
}

/* Thin SVD of the r x c complex matrix A: A = U diag(s) V^H. */
int oracle_svd_z(int r, int c, const zd *A, int lda, zd *U, double *s, zd *V,
                 int max_sweeps, double tol)
{
    int tall = r >= c;
    int len = tall ? r : c, n = tall ? c : r;
    zd *W = malloc(sizeof(zd) * (size_t)len * n);
    zd *R = malloc(sizeof(zd) * (size_t)n * n);
    double *nrm = malloc(sizeof(double) * n);
    int *perm = malloc(sizeof(int) * n);
    /* wide case works on A^H: A^H R = W  =>  A = R diag(s) (W/s)^H */
    for (int j = 0; j < n; ++j)
        for (int t = 0; t < len; ++t)
            W[t + (size_t)len * j] = tall ? A[t + (size_t)lda * j] : conj(A[j + (size_t)lda * t]);
    int sweeps = hestenes_z(len, n, W, R, max_sweeps, tol);
    for (int j = 0; j < n; ++j) {
        double acc = 0.0;
        for (int t = 0; t < len; ++t) {
            zd w = W[t + (size_t)len * j];
            acc += creal(w) * creal(w) + cimag(w) * cimag(w);
        }
        nrm[j] = sqrt(acc);
    }
    order_desc(n, nrm, perm);
    zd *Wn = tall ? U : V;
    zd *Rt = tall ? V : U;
    for (int jj = 0; jj < n; ++jj) {
        int j = perm[jj];
        s[jj] = nrm[j];
        double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
        for (int t = 0; t < len; ++t) Wn[t + (size_t)len * jj] = W[t + (size_t)len * j] * inv;
        for (int t = 0; t < n; ++t) Rt[t + (size_t)n * jj] = R[t + (size_t)n * j];
    }
    free(W); free(R); free(nrm); free(perm);
    return sweeps;
}

/* ------------------------------------------------------- many faces at once */

/* nf independent faces, face f at A + f*r*c (column major, lda = r).
 * Outputs per face: U + f*r*ns, s + f*ns, V + f*c*ns.  sweeps[f] as above. */
void oracle_svd_faces_d(int r, int c, int nf, const double *A, double *U, double *s,
                        double *V, int *sweeps, int max_sweeps, double tol)
{
    int ns = r < c ? r : c;
#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < nf; ++f)
        sweeps[f] = oracle_svd_d(r, c, A + (size_t)f * r * c, r, U + (size_t)f * r * ns,
                                 s + (size_t)f * ns, V + (size_t)f * c * ns, max_sweeps, tol);
}

void oracle_svd_faces_z(int r, int c, int nf, const zd *A, zd *U, double *s, zd *V,
                        int *sweeps, int max_sweeps, double tol)
{
    int ns = r < c ? r : c;
#pragma omp parallel for schedule(dynamic, 1)
    for (int f = 0; f < nf; ++f)
        sweeps[f] = oracle_svd_z(r, c, A + (size_t)f * r * c, r, U + (size_t)f * r * ns,
                                 s + (size_t)f * ns, V + (size_t)f * c * ns, max_sweeps, tol);
}
