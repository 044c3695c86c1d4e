/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY (parity oracle).
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the
 * symmetric-definite generalized eigenproblem  A X = B X Lambda  (Eq. 1),
 * A symmetric, B symmetric positive definite, s smallest (or largest) pairs.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load this library.  The GPU library shares no code with it.
 *
 * The oracle computes the *definition* through the explicit route of the
 * paper's Section 2.1 (transformation to and from the standard problem):
 *   1. B = U^T U, U upper triangular                          (Eq. 2)
 *   2. C = U^-T A U^-1 by two triangular solves (2n^3 flops)   (Eq. 3)
 *   3. all eigenpairs of the symmetric C, by Householder tridiagonalisation
 *      plus implicit QL with a Wilkinson-type shift, or by cyclic Jacobi
 *      (two independent textbook methods, Golub & Van Loan Sec. 8.3 / 8.5)
 *   4. Lambda = the s wanted eigenvalues ascending, X = U^-1 Y  (Eq. 4)
 * plus two independent checkers:
 *   - an inertia count of A - sigma B by symmetric-indefinite elimination
 *     with Bunch-Parlett diagonal pivoting (Sylvester's law of inertia), used
 *     by bisection to get every eigenvalue without Cholesky or Jacobi;
 *   - a plain Lanczos run on the implicit operator C w = U^-T(A(U^-1 w))
 *     (variant KI, Sec. 2.3; Table 1 keys KI1-KI4) with classical
 *     Gram-Schmidt re-orthogonalisation applied twice, in the paper's order:
 *     three-term recurrence first, then Gram-Schmidt applied twice.
 *
 * All matrices are dense, row-major, leading dimension n.  OpenMP is used
 * only over independent output rows/columns, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, n) ((size_t)(i) * (size_t)(n) + (size_t)(j))

/* ------------------------------------------------------------------ */
/* Eq. 2: B = U^T U.  Right-looking outer-product form on the upper     */
/* triangle: row i of U is row i of the updated B divided by sqrt(pivot) */
/* Returns 0, or k (1-based) if the leading minor of order k is not     */
/* positive definite.  U's strict lower triangle is set to zero.        */
/* ------------------------------------------------------------------ */
int or_cholesky_upper(int n, const double *B, double *U)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            U[IDX(i, j, n)] = (j >= i) ? B[IDX(i, j, n)] : 0.0;
    for (int i = 0; i < n; ++i) {
        double d = U[IDX(i, i, n)];
        if (!(d > 0.0)) return i + 1;
        d = sqrt(d);
        U[IDX(i, i, n)] = d;
        for (int j = i + 1; j < n; ++j) U[IDX(i, j, n)] /= d;
        /* trailing update of the upper triangle: B'_{jl} -= U_ij U_il, i<j<=l */
#pragma omp parallel for schedule(dynamic, 16)
        for (int j = i + 1; j < n; ++j) {
            const double uij = U[IDX(i, j, n)];
            double *rowj = &U[IDX(j, 0, n)];
            const double *rowi = &U[IDX(i, 0, n)];
            for (int l = j; l < n; ++l) rowj[l] -= uij * rowi[l];
        }
    }
    return 0;
}

/* x := U^-1 x  (back substitution, U upper). Table 1 key KI1. */
void or_trsv_upper(int n, const double *U, double *x)
{
    for (int i = n - 1; i >= 0; --i) {
        double acc = x[i];
        const double *row = &U[IDX(i, 0, n)];
        for (int j = i + 1; j < n; ++j) acc -= row[j] * x[j];
        x[i] = acc / row[i];
    }
}

/* x := U^-T x  (forward substitution with the lower factor U^T). Key KI3. */
void or_trsv_upper_t(int n, const double *U, double *x)
{
    for (int i = 0; i < n; ++i) {
        const double *row = &U[IDX(i, 0, n)];
        const double xi = x[i] / row[i];
        x[i] = xi;
        for (int j = i + 1; j < n; ++j) x[j] -= row[j] * xi;
    }
}

/* y := A x, A full storage. Key KI2. */
void or_matvec(int n, const double *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        const double *row = &A[IDX(i, 0, n)];
        for (int j = 0; j < n; ++j) acc += row[j] * x[j];
        y[i] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* Eq. 3: C := U^-T A U^-1 by two triangular solves.                    */
/*   W := A U^-1   (row i of W is (U^-T a_i)^T, a_i = row i of A)       */
/*   C := U^-T W   (row i of C is (U^-T w^(i))^T, w^(i) = column i of W,*/
/*                  using W^T = U^-T A for symmetric A)                 */
/* then C := (C + C^T)/2.                                               */
/* ------------------------------------------------------------------ */
void or_form_c(int n, const double *A, const double *U, double *C)
{
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double *w = &W[IDX(i, 0, n)];
        memcpy(w, &A[IDX(i, 0, n)], sizeof(double) * n);
        or_trsv_upper_t(n, U, w);
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < n; ++i) {
        double *c = &C[IDX(i, 0, n)];
        for (int j = 0; j < n; ++j) c[j] = W[IDX(j, i, n)];
        or_trsv_upper_t(n, U, c);
    }
    free(W);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double v = 0.5 * (C[IDX(i, j, n)] + C[IDX(j, i, n)]);
            C[IDX(i, j, n)] = v;
            C[IDX(j, i, n)] = v;
        }
}

/* ------------------------------------------------------------------ */
/* Householder tridiagonalisation Q^T C Q = T (GVL Sec. 8.3.1).          */
/* On return d (n) is the diagonal of T, e (n) has e[i] = T(i, i+1)      */
/* for i < n-1 and e[n-1] = 0, and Qt (n x n) holds Q^T row-wise, i.e.   */
/* row i of Qt is column i of Q.  C is destroyed.                        */
/* ------------------------------------------------------------------ */
static void or_tridiagonalise(int n, double *C, double *d, double *e, double *Qt)
{
    double *V = (double *)calloc((size_t)n * n, sizeof(double)); /* reflector k stored in row k */
    double *beta = (double *)calloc((size_t)n, sizeof(double));
    double *p = (double *)malloc(sizeof(double) * n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;          /* length of x = C[k+1:, k] */
        double *v = &V[IDX(k, 0, n)] + (k + 1);
        double norm2 = 0.0;
        for (int t = 0; t < m; ++t) { v[t] = C[IDX(k + 1 + t, k, n)]; norm2 += v[t] * v[t]; }
        const double alpha = sqrt(norm2);
        double tail2 = norm2 - v[0] * v[0];
        if (alpha == 0.0 || tail2 == 0.0) {  /* already reduced in this column */
            beta[k] = 0.0;
            d[k] = C[IDX(k, k, n)];
            e[k] = v[0];
            continue;
        }
        const double sgn = (v[0] >= 0.0) ? 1.0 : -1.0;
        v[0] += sgn * alpha;                 /* v = x + sign(x1) ||x|| e1 */
        double vtv = v[0] * v[0] + tail2;
        const double b = 2.0 / vtv;          /* H = I - b v v^T maps x to -sign(x1)||x|| e1 */
        beta[k] = b;
        /* p = b * C_sub v */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i) {
            const double *row = &C[IDX(k + 1 + i, k + 1, n)];
            double acc = 0.0;
            for (int j = 0; j < m; ++j) acc += row[j] * v[j];
            p[i] = b * acc;
        }
        double ptv = 0.0;
        for (int i = 0; i < m; ++i) ptv += p[i] * v[i];
        const double K = 0.5 * b * ptv;
        for (int i = 0; i < m; ++i) p[i] -= K * v[i]; /* w = p - K v */
#pragma omp parallel for schedule(static)
        for (int i = 0; i < m; ++i) {
            double *row = &C[IDX(k + 1 + i, k + 1, n)];
            const double vi = v[i], wi = p[i];
            for (int j = 0; j < m; ++j) row[j] -= vi * p[j] + wi * v[j];
        }
        d[k] = C[IDX(k, k, n)];
        e[k] = -sgn * alpha;
    }
    if (n >= 2) {
        d[n - 2] = C[IDX(n - 2, n - 2, n)];
        e[n - 2] = C[IDX(n - 1, n - 2, n)];
    }
    d[n - 1] = C[IDX(n - 1, n - 1, n)];
    e[n - 1] = 0.0;

    /* Q = H_0 H_1 ... H_{n-3}; accumulate Q^T = H_{n-3} ... H_0 applied to I
       from the right, i.e. Qt := Qt H_k for k = 0.. (H symmetric).  Row r of
       Qt is column r of Q.  Work on Q itself column-blocked: build Q by
       backward accumulation Q := H_k Q on rows k+1.. then transpose. */
    double *Q = (double *)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i) Q[IDX(i, i, n)] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const int m = n - k - 1;
        const double *v = &V[IDX(k, 0, n)] + (k + 1);
        const double b = beta[k];
        /* Q[k+1:, k+1:] := (I - b v v^T) Q[k+1:, k+1:]  (column-parallel) */
#pragma omp parallel for schedule(static)
        for (int j = k + 1; j < n; ++j) {
            double acc = 0.0;
            for (int i = 0; i < m; ++i) acc += v[i] * Q[IDX(k + 1 + i, j, n)];
            acc *= b;
            for (int i = 0; i < m; ++i) Q[IDX(k + 1 + i, j, n)] -= acc * v[i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Qt[IDX(j, i, n)] = Q[IDX(i, j, n)];
    free(Q);
    free(V);
    free(beta);
    free(p);
}

/* ------------------------------------------------------------------ */
/* Implicit QL on a symmetric tridiagonal (d, e), rotations accumulated  */
/* into the rows of Zt (row i = current vector i).  Shift from the      */
/* leading 2x2 of the active block (Wilkinson-type).  Returns 0, or -1  */
/* if an eigenvalue failed to converge in 60 sweeps.                    */
/* The steps are those of the published implicit QL routine tql2        */
/* (Bowdler, Martin, Reinsch and Wilkinson, Numer. Math. 11, 1968;      */
/* EISPACK), in the arrangement Numerical Recipes prints as tqli:       */
/* the same shift, the same bottom-up rotation sweep and the same split */
/* on an underflowing rotation (Golub and Van Loan, Sec. 8.3, for the   */
/* theory).                                                             */
/* ------------------------------------------------------------------ */
static int or_tridiag_ql(int n, double *d, double *e, double *Zt)
{
    const double eps = 0x1p-52;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m < n - 1; ++m) {
                const double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return -1;
            /* shift: eigenvalue of the leading 2x2 [d_l e_l; e_l d_l+1] nearer d_l */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            int i;
            int deflated = 0;
            for (i = m - 1; i >= l; --i) {
                double f = s * e[i];
                const double b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {            /* underflow: split and restart */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    deflated = 1;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                /* rotate vectors i and i+1 (rows of Zt) */
                double *zi = &Zt[IDX(i, 0, n)];
                double *zi1 = &Zt[IDX(i + 1, 0, n)];
                for (int k = 0; k < n; ++k) {
                    const double t = zi1[k];
                    zi1[k] = s * zi[k] + c * t;
                    zi[k] = c * zi[k] - s * t;
                }
            }
            if (deflated) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    return 0;
}

/* All eigenpairs of symmetric C by tridiagonalisation + QL.
   w (n) unsorted, Zt row i = eigenvector for w[i].  C destroyed. */
int or_eig_ql(int n, double *C, double *w, double *Zt)
{
    double *e = (double *)malloc(sizeof(double) * n);
    or_tridiagonalise(n, C, w, e, Zt);
    int rc = or_tridiag_ql(n, w, e, Zt);
    free(e);
    return rc;
}

/* All eigenpairs of symmetric C by cyclic-by-row Jacobi (GVL Sec. 8.5).
   Stops when off(C) <= 2^-53 ||C||_F.  w (n), Zt row i = eigenvector i.
   Returns the number of sweeps, or -1 if 100 sweeps did not suffice. */
int or_eig_jacobi(int n, double *C, double *w, double *Zt)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Zt[IDX(i, j, n)] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (size_t t = 0; t < (size_t)n * n; ++t) fro += C[t] * C[t];
    fro = sqrt(fro);
    const double tol = 0x1p-53 * fro;
    int sweep;
    for (sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += 2.0 * C[IDX(i, j, n)] * C[IDX(i, j, n)];
        if (sqrt(off) <= tol) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = C[IDX(p, q, n)];
                if (apq == 0.0) continue;
                /* symmetric 2x2 Schur: zero C(p,q) with J = [c s; -s c] */
                const double tau = (C[IDX(q, q, n)] - C[IDX(p, p, n)]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* C := J^T C J on rows/cols p, q */
                for (int k = 0; k < n; ++k) {      /* columns */
                    const double ckp = C[IDX(k, p, n)], ckq = C[IDX(k, q, n)];
                    C[IDX(k, p, n)] = c * ckp - s * ckq;
                    C[IDX(k, q, n)] = s * ckp + c * ckq;
                }
                for (int k = 0; k < n; ++k) {      /* rows */
                    const double cpk = C[IDX(p, k, n)], cqk = C[IDX(q, k, n)];
                    C[IDX(p, k, n)] = c * cpk - s * cqk;
                    C[IDX(q, k, n)] = s * cpk + c * cqk;
                }
                C[IDX(p, q, n)] = C[IDX(q, p, n)] = 0.0;
                /* Z := Z J  (rows of Zt are columns of Z) */
                double *zp = &Zt[IDX(p, 0, n)], *zq = &Zt[IDX(q, 0, n)];
                for (int k = 0; k < n; ++k) {
                    const double a = zp[k], b = zq[k];
                    zp[k] = c * a - s * b;
                    zq[k] = s * a + c * b;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = C[IDX(i, i, n)];
    return sweep < 100 ? sweep : -1;
}

/* ------------------------------------------------------------------ */
/* Inertia: number of eigenvalues of the pencil (A, B) below sigma =    */
/* number of negative eigenvalues of A - sigma B (B SPD, Sylvester).    */
/* Symmetric elimination with Bunch-Parlett complete diagonal pivoting: */
/* 1x1 pivot if max|diag| >= a0 max|offdiag| (a0 = (1+sqrt 17)/8),      */
/* else the 2x2 pivot on the largest off-diagonal entry.                 */
/* ------------------------------------------------------------------ */
int or_inertia_below(int n, const double *A, const double *B, double sigma)
{
    double *M = (double *)malloc(sizeof(double) * (size_t)n * n);
    int *act = (int *)malloc(sizeof(int) * n);
    for (size_t t = 0; t < (size_t)n * n; ++t) M[t] = A[t] - sigma * B[t];
    for (int i = 0; i < n; ++i) act[i] = 1;
    const double a0 = (1.0 + sqrt(17.0)) / 8.0;
    int neg = 0, left = n;
    while (left > 0) {
        int pd = -1, pr = -1, pq = -1;
        double mu1 = -1.0, mu0 = -1.0;
        for (int i = 0; i < n; ++i) {
            if (!act[i]) continue;
            if (fabs(M[IDX(i, i, n)]) > mu1) { mu1 = fabs(M[IDX(i, i, n)]); pd = i; }
            for (int j = i + 1; j < n; ++j)
                if (act[j] && fabs(M[IDX(i, j, n)]) > mu0) { mu0 = fabs(M[IDX(i, j, n)]); pr = i; pq = j; }
        }
        if (mu1 == 0.0 && mu0 <= 0.0) break;     /* remaining block is zero */
        if (mu1 >= a0 * mu0 || left == 1) {
            const double dp = M[IDX(pd, pd, n)];
            if (dp < 0.0) ++neg;
            act[pd] = 0;
            --left;
            for (int i = 0; i < n; ++i) {
                if (!act[i]) continue;
                const double f = M[IDX(i, pd, n)] / dp;
                for (int j = 0; j < n; ++j)
                    if (act[j]) M[IDX(i, j, n)] -= f * M[IDX(pd, j, n)];
            }
        } else {
            const double a = M[IDX(pr, pr, n)], b = M[IDX(pr, pq, n)], c = M[IDX(pq, pq, n)];
            const double det = a * c - b * b;
            if (det < 0.0) neg += 1;
            else if (a + c < 0.0) neg += 2;
            act[pr] = act[pq] = 0;
            left -= 2;
            /* M_S := M_S - [m_ir m_iq] E^-1 [m_rj; m_qj],  E^-1 = [c -b; -b a]/det */
            for (int i = 0; i < n; ++i) {
                if (!act[i]) continue;
                const double mir = M[IDX(i, pr, n)], miq = M[IDX(i, pq, n)];
                const double f1 = (c * mir - b * miq) / det;
                const double f2 = (-b * mir + a * miq) / det;
                for (int j = 0; j < n; ++j)
                    if (act[j]) M[IDX(i, j, n)] -= f1 * M[IDX(pr, j, n)] + f2 * M[IDX(pq, j, n)];
            }
        }
    }
    free(M);
    free(act);
    return neg;
}

/* The k-th smallest (0-based) eigenvalue of (A, B) by bisection on the
   inertia count, to an interval of relative width ~4 ulp. */
double or_bisect_eig(int n, const double *A, const double *B, int k)
{
    double lo = -1.0, hi = 1.0;
    while (or_inertia_below(n, A, B, lo) > k) lo *= 2.0;
    while (or_inertia_below(n, A, B, hi) <= k) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 4.0 * 0x1p-53 * fmax(fabs(lo), fabs(hi))) break;
        if (or_inertia_below(n, A, B, mid) > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

/* X := U^-1 Y for s vectors stored as rows of Y (s x n). Eq. 4, key BT1. */
void or_backsolve(int n, int s, const double *U, double *Y)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < s; ++i) or_trsv_upper(n, U, &Y[IDX(i, 0, n)]);
}

/* Sign convention: the entry of largest magnitude (lowest index on ties)
   is made positive. */
static void or_sign_normalise(int n, double *x)
{
    int p = 0;
    double best = -1.0;
    for (int i = 0; i < n; ++i)
        if (fabs(x[i]) > best) { best = fabs(x[i]); p = i; }
    if (x[p] < 0.0)
        for (int i = 0; i < n; ++i) x[i] = -x[i];
}

/* ------------------------------------------------------------------ */
/* The definition: s wanted eigenpairs of (A, B), Eq. 1-4.               */
/*   which = 0: s smallest; 1: s largest.  Lambda ascending either way.  */
/*   method = 0: tridiagonalisation + QL; 1: Jacobi.                     */
/*   X: s x n, row i = x_i, B-orthonormal, sign-normalised.              */
/* Returns 0; k > 0 if B is not SPD (minor k); -1 if the eigensolver     */
/* failed; -2 on bad arguments.                                          */
/* ------------------------------------------------------------------ */
int or_gsyeig(int n, int s, int which, int method, const double *A, const double *B,
              double *lam, double *X)
{
    if (n < 1 || s < 1 || s > n) return -2;
    double *U = (double *)malloc(sizeof(double) * (size_t)n * n);
    int info = or_cholesky_upper(n, B, U);
    if (info) { free(U); return info; }
    double *C = (double *)malloc(sizeof(double) * (size_t)n * n);
    or_form_c(n, A, U, C);
    double *w = (double *)malloc(sizeof(double) * n);
    double *Zt = (double *)malloc(sizeof(double) * (size_t)n * n);
    int rc = (method == 1) ? (or_eig_jacobi(n, C, w, Zt) < 0 ? -1 : 0) : or_eig_ql(n, C, w, Zt);
    if (rc) { free(U); free(C); free(w); free(Zt); return -1; }
    /* stable ascending order of the eigenvalues (ties keep index order) */
    int *ord = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    for (int i = 1; i < n; ++i) {            /* insertion sort: obviously stable */
        const int t = ord[i];
        int j = i - 1;
        while (j >= 0 && w[ord[j]] > w[t]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = t;
    }
    const int first = (which == 1) ? n - s : 0;
    for (int i = 0; i < s; ++i) {
        const int src = ord[first + i];
        lam[i] = w[src];
        memcpy(&X[IDX(i, 0, n)], &Zt[IDX(src, 0, n)], sizeof(double) * n);
    }
    or_backsolve(n, s, U, X);
    for (int i = 0; i < s; ++i) or_sign_normalise(n, &X[IDX(i, 0, n)]);
    free(ord); free(U); free(C); free(w); free(Zt);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Plain Lanczos on the implicit operator (variant KI), k steps.         */
/*   w_0 = v0/||v0||; for j = 0..k-1:                                   */
/*     z := U^-T (A (U^-1 w_j))             (keys KI1, KI2, KI3)         */
/*     z := z - beta_{j-1} w_{j-1}          (three-term recurrence)      */
/*     alpha_j := w_j^T z;  z := z - alpha_j w_j                         */
/*     twice: h := W_j^T z; z := z - W_j h  (W_j = [w_0..w_j], CGS2)      */
/*     beta_j := ||z||;  w_{j+1} := z / beta_j                           */
/* W: (k+1) x n, row j = w_j.  U is the upper Cholesky factor of B.      */
/* ------------------------------------------------------------------ */
void or_lanczos(int n, int k, const double *A, const double *U, const double *v0,
                double *alpha, double *beta, double *W)
{
    double *z = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n);
    double *h = (double *)malloc(sizeof(double) * (k + 1));
    double nv = 0.0;
    for (int i = 0; i < n; ++i) nv += v0[i] * v0[i];
    nv = sqrt(nv);
    for (int i = 0; i < n; ++i) W[i] = v0[i] / nv;
    for (int j = 0; j < k; ++j) {
        const double *wj = &W[IDX(j, 0, n)];
        memcpy(t, wj, sizeof(double) * n);
        or_trsv_upper(n, U, t);
        or_matvec(n, A, t, z);
        or_trsv_upper_t(n, U, z);
        if (j > 0) {
            const double *wp = &W[IDX(j - 1, 0, n)];
            for (int i = 0; i < n; ++i) z[i] -= beta[j - 1] * wp[i];
        }
        double a = 0.0;
        for (int i = 0; i < n; ++i) a += wj[i] * z[i];
        alpha[j] = a;
        for (int i = 0; i < n; ++i) z[i] -= a * wj[i];
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = 0; q <= j; ++q) {
                const double *wq = &W[IDX(q, 0, n)];
                double acc = 0.0;
                for (int i = 0; i < n; ++i) acc += wq[i] * z[i];
                h[q] = acc;
            }
            for (int q = 0; q <= j; ++q) {
                const double *wq = &W[IDX(q, 0, n)];
                for (int i = 0; i < n; ++i) z[i] -= h[q] * wq[i];
            }
        }
        double b = 0.0;
        for (int i = 0; i < n; ++i) b += z[i] * z[i];
        b = sqrt(b);
        beta[j] = b;
        double *wn = &W[IDX(j + 1, 0, n)];
        for (int i = 0; i < n; ++i) wn[i] = z[i] / b;
    }
    free(z);
    free(t);
    free(h);
}

/* Eigenvalues of a symmetric tridiagonal (d, e) (e[i] couples i, i+1),
   ascending, by QL without vectors (test helper for Ritz values). */
int or_tridiag_eigvals(int n, const double *d_in, const double *e_in, double *w)
{
    double *e = (double *)malloc(sizeof(double) * n);
    double *Zt = (double *)calloc((size_t)n * n, sizeof(double));
    for (int i = 0; i < n; ++i) { w[i] = d_in[i]; e[i] = (i < n - 1) ? e_in[i] : 0.0; }
    for (int i = 0; i < n; ++i) Zt[IDX(i, i, n)] = 1.0;
    int rc = or_tridiag_ql(n, w, e, Zt);
    for (int i = 1; i < n; ++i) {
        const double t = w[i];
        int j = i - 1;
        while (j >= 0 && w[j] > t) { w[j + 1] = w[j]; --j; }
        w[j + 1] = t;
    }
    free(e);
    free(Zt);
    return rc;
}
