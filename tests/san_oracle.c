/* Host sanitizer driver for the oracle (tests/test_host_sanitizers.py):
 * every exported routine on small deterministic pencils, built with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status 0 when
 * every call returned normally and the cross-checks hold. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int or_cholesky_upper(int n, const double *B, double *U);
void or_trsv_upper(int n, const double *U, double *x);
void or_trsv_upper_t(int n, const double *U, double *x);
void or_matvec(int n, const double *A, const double *x, double *y);
void or_form_c(int n, const double *A, const double *U, double *C);
int or_eig_ql(int n, double *C, double *w, double *Zt);
int or_eig_jacobi(int n, double *C, double *w, double *Zt);
int or_inertia_below(int n, const double *A, const double *B, double sigma);
double or_bisect_eig(int n, const double *A, const double *B, int k);
void or_backsolve(int n, int s, const double *U, double *Y);
int or_gsyeig(int n, int s, int which, int method, const double *A, const double *B, double *lam, double *X);
void or_lanczos(int n, int k, const double *A, const double *U, const double *v0, double *alpha, double *beta,
                double *W);
int or_tridiag_eigvals(int n, const double *d_in, const double *e_in, double *w);

static unsigned long long st = 88172645463325252ull;
static double urand(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) * 0x1p-53 * 2.0 - 1.0;
}

static void sort(double *v, int n)
{
    for (int i = 1; i < n; ++i) {
        const double t = v[i];
        int j = i - 1;
        while (j >= 0 && v[j] > t) {
            v[j + 1] = v[j];
            --j;
        }
        v[j + 1] = t;
    }
}

static int run(int n)
{
    const size_t nn = (size_t)n * n;
    double *A = malloc(nn * sizeof(double)), *B = malloc(nn * sizeof(double)), *U = malloc(nn * sizeof(double));
    double *C = malloc(nn * sizeof(double)), *C2 = malloc(nn * sizeof(double)), *Zt = malloc(nn * sizeof(double));
    double *Zt2 = malloc(nn * sizeof(double)), *w = malloc(n * sizeof(double)), *w2 = malloc(n * sizeof(double));
    double *x = malloc(n * sizeof(double)), *y = malloc(n * sizeof(double)), *X = malloc(nn * sizeof(double));
    double *lam = malloc(n * sizeof(double));
    int bad = 0;
    /* A symmetric; B = G G^T + n I (SPD) */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) A[i * n + j] = A[j * n + i] = urand();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) C[i * n + j] = urand();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = (i == j) ? n : 0.0;
            for (int k = 0; k < n; ++k) s += C[i * n + k] * C[j * n + k];
            B[i * n + j] = s;
        }
    if (or_cholesky_upper(n, B, U) != 0) bad |= 1;
    for (int i = 0; i < n; ++i) x[i] = urand();
    for (int i = 0; i < n; ++i) y[i] = x[i];
    or_trsv_upper(n, U, y);
    or_trsv_upper_t(n, U, y);
    or_matvec(n, A, x, y);
    or_form_c(n, A, U, C);
    for (size_t e = 0; e < nn; ++e) C2[e] = C[e];
    if (or_eig_ql(n, C, w, Zt) != 0) bad |= 2;
    if (or_eig_jacobi(n, C2, w2, Zt2) < 0) bad |= 4;
    sort(w, n);
    sort(w2, n);
    for (int i = 0; i < n; ++i)
        if (fabs(w[i] - w2[i]) > 1e-10 * (1.0 + fabs(w[n - 1]) + fabs(w[0]))) bad |= 8;
    const int below = or_inertia_below(n, A, B, 0.5 * (w[0] + w[n - 1]));
    if (below < 0 || below > n) bad |= 16;
    const double l0 = or_bisect_eig(n, A, B, 0);
    if (fabs(l0 - w[0]) > 1e-8 * (1.0 + fabs(w[0]))) bad |= 32;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) X[(size_t)j * n + i] = Zt[(size_t)j * n + i];
    or_backsolve(n, n, U, X);
    for (int which = 0; which < 2; ++which)
        for (int method = 0; method < 2; ++method) {
            const int s = n > 3 ? 3 : n;
            if (or_gsyeig(n, s, which, method, A, B, lam, X) != 0) bad |= 64;
            if (which == 0 && fabs(lam[0] - w[0]) > 1e-10 * (1.0 + fabs(w[0]))) bad |= 128;
        }
    const int k = n < 8 ? n : 8;
    double *al = malloc(k * sizeof(double)), *be = malloc(k * sizeof(double));
    double *W = malloc((size_t)n * (k + 1) * sizeof(double));
    for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.1 * i;
    or_lanczos(n, k, A, U, x, al, be, W);
    if (or_tridiag_eigvals(k, al, be, w2) != 0) bad |= 256;
    free(al); free(be); free(W);
    free(A); free(B); free(U); free(C); free(C2); free(Zt); free(Zt2); free(w); free(w2); free(x); free(y);
    free(X); free(lam);
    return bad;
}

int main(void)
{
    const int ns[] = {1, 2, 5, 33};
    for (int t = 0; t < 4; ++t) {
        const int bad = run(ns[t]);
        if (bad) {
            printf("n=%d failed checks 0x%x\n", ns[t], bad);
            return 1;
        }
    }
    printf("ok\n");
    return 0;
}
