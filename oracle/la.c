/*
 * Dense FP64 linear algebra for the oracle (test infrastructure only):
 * Gauss-Jordan inverse, LU solve with partial pivoting, and least squares by
 * Householder QR.  Plain textbook algorithms, no blocking.
 */
#include "oracle_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

int la_inverse(int n, const double *A, double *Ainv)
{
    double *M = malloc(sizeof(double) * n * 2 * n);
    if (!M) return -1;
    for (int i = 0; i < n; i++) {
        for (int j = 0; j < n; j++) {
            M[i * 2 * n + j] = A[i * n + j];
            M[i * 2 * n + n + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(M[r * 2 * n + c]) > fabs(M[p * 2 * n + c])) p = r;
        if (fabs(M[p * 2 * n + c]) == 0.0) { free(M); return -1; }
        if (p != c)
            for (int j = 0; j < 2 * n; j++) {
                double t = M[c * 2 * n + j];
                M[c * 2 * n + j] = M[p * 2 * n + j];
                M[p * 2 * n + j] = t;
            }
        double piv = M[c * 2 * n + c];
        for (int j = 0; j < 2 * n; j++) M[c * 2 * n + j] /= piv;
        for (int r = 0; r < n; r++) {
            if (r == c) continue;
            double f = M[r * 2 * n + c];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; j++) M[r * 2 * n + j] -= f * M[c * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = M[i * 2 * n + n + j];
    free(M);
    return 0;
}

int la_lu_solve(int n, const double *A, const double *b, double *x)
{
    double *M = malloc(sizeof(double) * n * n);
    int *perm = malloc(sizeof(int) * n);
    if (!M || !perm) { free(M); free(perm); return -1; }
    memcpy(M, A, sizeof(double) * n * n);
    for (int i = 0; i < n; i++) perm[i] = i;
    for (int c = 0; c < n; c++) {
        int p = c;
        for (int r = c + 1; r < n; r++)
            if (fabs(M[r * n + c]) > fabs(M[p * n + c])) p = r;
        if (M[p * n + c] == 0.0) { free(M); free(perm); return -1; }
        if (p != c) {
            for (int j = 0; j < n; j++) {
                double t = M[c * n + j];
                M[c * n + j] = M[p * n + j];
                M[p * n + j] = t;
            }
            int t = perm[c]; perm[c] = perm[p]; perm[p] = t;
        }
        for (int r = c + 1; r < n; r++) {
            double f = M[r * n + c] / M[c * n + c];
            M[r * n + c] = f;
            for (int j = c + 1; j < n; j++) M[r * n + j] -= f * M[c * n + j];
        }
    }
    /* forward substitution on the permuted right-hand side */
    for (int i = 0; i < n; i++) {
        double s = b[perm[i]];
        for (int j = 0; j < i; j++) s -= M[i * n + j] * x[j];
        x[i] = s;
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = x[i];
        for (int j = i + 1; j < n; j++) s -= M[i * n + j] * x[j];
        x[i] = s / M[i * n + i];
    }
    free(M);
    free(perm);
    return 0;
}

/* minimise ||A x - b||_2 for an m x n matrix A (m >= n) by Householder QR */
int la_lsq_qr(int m, int n, const double *A, const double *b, double *x)
{
    if (m < n) return -1;
    double *R = malloc(sizeof(double) * m * n);
    double *y = malloc(sizeof(double) * m);
    double *v = malloc(sizeof(double) * m);
    if (!R || !y || !v) { free(R); free(y); free(v); return -1; }
    memcpy(R, A, sizeof(double) * m * n);
    memcpy(y, b, sizeof(double) * m);
    for (int k = 0; k < n; k++) {
        double nrm = 0.0;
        for (int i = k; i < m; i++) nrm += R[i * n + k] * R[i * n + k];
        nrm = sqrt(nrm);
        if (nrm == 0.0) { free(R); free(y); free(v); return -1; }
        double alpha = (R[k * n + k] > 0) ? -nrm : nrm;
        for (int i = 0; i < m; i++) v[i] = 0.0;
        v[k] = R[k * n + k] - alpha;
        for (int i = k + 1; i < m; i++) v[i] = R[i * n + k];
        double vv = 0.0;
        for (int i = k; i < m; i++) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        for (int j = k; j < n; j++) {
            double s = 0.0;
            for (int i = k; i < m; i++) s += v[i] * R[i * n + j];
            s = 2.0 * s / vv;
            for (int i = k; i < m; i++) R[i * n + j] -= s * v[i];
        }
        double s = 0.0;
        for (int i = k; i < m; i++) s += v[i] * y[i];
        s = 2.0 * s / vv;
        for (int i = k; i < m; i++) y[i] -= s * v[i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = y[i];
        for (int j = i + 1; j < n; j++) s -= R[i * n + j] * x[j];
        if (R[i * n + i] == 0.0) { free(R); free(y); free(v); return -1; }
        x[i] = s / R[i * n + i];
    }
    free(R);
    free(y);
    free(v);
    return 0;
}
