// k_tridiag.hip -- eigenpairs of the Lanczos tridiagonal T_m (key KI5,
// Section 2.3: the extremal eigenvalues of T_m approximate those of C).
//
//  * Eigenvalues: Sturm-sequence bisection.  One wave64 per wanted index;
//    each round evaluates the inertia count at 64 interior points of the
//    current interval at once (multisection), shrinking it 65x per round.
//  * Eigenvectors: inverse iteration with T - theta I factored by Gaussian
//    elimination with partial pivoting (a third super-diagonal appears on
//    row swaps), every wanted index in parallel.  Eigenvalues closer than
//    1e-3 ||T|| form a cluster whose vectors one workgroup then makes
//    orthonormal in order (Gram-Schmidt, one more solve, Gram-Schmidt).
//  * The recurrences are inherently sequential; a wave runs them uniformly
//    with the operands of 64 consecutive rows held one per lane and read
//    with readlane, so the loop never waits on memory.
#include "internal.h"
#include "tridiag_dev.h"

namespace {

using namespace tdg;

__global__ __launch_bounds__(64) void k_tri_bisect(const double *__restrict__ alpha,
                                                   const double *__restrict__ beta, int64_t m,
                                                   int64_t nwant, int which, double *theta)
{
    const int64_t i = blockIdx.x;
    int64_t idx;
    if (i < nwant) idx = (which == 0) ? i : m - nwant + i;
    else idx = (which == 0) ? m - 1 : 0;
    const double v = bisect_index(alpha, beta, m, idx);
    if (threadIdx.x == 0) theta[i] = v;
}

// Eigenvalues of T with ascending indices first .. first+count-1 into
// theta[0..count); theta[count] = the largest (which = 0) or smallest
// (which = 1) eigenvalue, theta[count+1] = the other extreme -- the ends
// that bound ||T||.
__global__ __launch_bounds__(64) void k_tri_bisect_range(const double *__restrict__ alpha,
                                                         const double *__restrict__ beta, int64_t m,
                                                         int64_t first, int64_t count, int which,
                                                         double *theta)
{
    const int64_t i = blockIdx.x;
    int64_t idx;
    if (i < count) idx = first + i;
    else if (i == count) idx = (which == 0) ? m - 1 : 0;
    else idx = (which == 0) ? 0 : m - 1;
    const double v = bisect_index(alpha, beta, m, idx);
    if (threadIdx.x == 0) theta[i] = v;
}

__device__ double block_dot(const double *a, const double *b, int64_t m, double *sbuf)
{
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) v = fma(a[i], b[i], v);
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sbuf[0] + sbuf[1]) + (sbuf[2] + sbuf[3]);
}

__device__ __forceinline__ double tnorm_of(const double *theta, int64_t nwant)
{
    return fmax(fmax(fabs(theta[0]), fabs(theta[nwant - 1])), fabs(theta[nwant]));
}

// Inverse iteration, one workgroup per wanted eigenvalue, all in parallel.
// Scratch per index j (7 m doubles): LU factors (5 m), the vector, spare.
// Ritz values equal to within 10 u ||T|| are moved apart by that amount so
// their factorisations differ.
__global__ __launch_bounds__(256) void k_tri_invit(const double *__restrict__ alpha,
                                                   const double *__restrict__ beta, int64_t m,
                                                   int64_t nwant, const double *__restrict__ theta,
                                                   double *S, int64_t lds, double *scratch,
                                                   double *lastcomp, int iters)
{
    __shared__ double sbuf[4];
    const int64_t j = blockIdx.x;
    const double tn = tnorm_of(theta, nwant);
    const double pivtiny = EPS * fmax(tn, 0x1p-1000);
    const double pert = 10.0 * EPS * fmax(tn, 0x1p-1000);
    int64_t q = j;
    while (q > 0 && theta[q] - theta[q - 1] < pert) --q;
    const double lam = theta[j] + (double)(j - q) * pert;
    double *f = scratch + j * 7 * m;
    double *x = f + 5 * m;
    if (threadIdx.x < 64) tri_lu(alpha, beta, m, lam, pivtiny, f);
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x)
        x[t] = 2.0 * ((double)(mix64(0x5DEECE66Dull * (uint64_t)(j + 1) + (uint64_t)t) >> 11) * 0x1p-53) - 1.0;
    __syncthreads();
    for (int it = 0; it < iters; ++it) {
        if (threadIdx.x < 64) tri_solve(f, m, x);
        __syncthreads();
        const double nrm = sqrt(block_dot(x, x, m, sbuf));
        const double inv = (nrm > 0.0) ? 1.0 / nrm : 0.0;
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) x[t] *= inv;
        __syncthreads();
    }
    if (S)
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) S[j * lds + t] = x[t];
    if (lastcomp && threadIdx.x == 0) lastcomp[j] = fabs(x[m - 1]);
}

// x -= S_c (S_c^T x) twice over the cluster columns p0..p1-1 (one wave per
// column for the projections); then x /= ||x||.
__device__ void cgs2_normalise(const double *S, int64_t lds, int64_t p0, int64_t p1, int64_t m,
                               double *x, double *h, double *sbuf)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int pass = 0; pass < 2 && p1 > p0; ++pass) {
        for (int64_t p = p0 + wv; p < p1; p += blockDim.x / 64) {
            const double *sp = S + p * lds;
            double d = 0.0;
            for (int64_t t = lane; t < m; t += 64) d = fma(sp[t], x[t], d);
            for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
            if (lane == 0) h[p - p0] = d;
        }
        __syncthreads();
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
            double v = x[t];
            for (int64_t p = p0; p < p1; ++p) v = fma(-h[p - p0], S[p * lds + t], v);
            x[t] = v;
        }
        __syncthreads();
    }
    const double nrm = sqrt(block_dot(x, x, m, sbuf));
    const double inv = (nrm > 0.0) ? 1.0 / nrm : 0.0;
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) x[t] *= inv;
    __syncthreads();
}

// Eigenvalues closer than 1e-3 ||T|| form a cluster; the workgroup of its
// first index makes the cluster's vectors orthonormal in order: for each
// later member, Gram-Schmidt against the earlier ones, one more inverse-
// iteration solve with the member's stored factors, and Gram-Schmidt again.
__global__ __launch_bounds__(256) void k_tri_cluster(int64_t m, int64_t nwant,
                                                     const double *__restrict__ theta, double *S,
                                                     int64_t lds, double *scratch, double *lastcomp)
{
    __shared__ double sbuf[4];
    const int64_t i0 = blockIdx.x;
    const double ortol = 1e-3 * tnorm_of(theta, nwant);
    if (i0 > 0 && theta[i0] - theta[i0 - 1] <= ortol) return;
    int64_t i1 = i0 + 1;
    while (i1 < nwant && theta[i1] - theta[i1 - 1] <= ortol) ++i1;
    if (i1 == i0 + 1) return;
    double *h = scratch + i0 * 7 * m + 6 * m;
    for (int64_t j = i0 + 1; j < i1; ++j) {
        double *f = scratch + j * 7 * m;
        double *x = f + 5 * m;
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) x[t] = S[j * lds + t];
        __syncthreads();
        cgs2_normalise(S, lds, i0, j, m, x, h, sbuf);
        if (threadIdx.x < 64) tri_solve(f, m, x);
        __syncthreads();
        cgs2_normalise(S, lds, i0, j, m, x, h, sbuf);
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) S[j * lds + t] = x[t];
        if (lastcomp && threadIdx.x == 0) lastcomp[j] = fabs(x[m - 1]);
        __syncthreads();
    }
}

// nconv = #{ i in [i0, i0 + cnt) : |beta_m| lastcomp[i] <= tol ||T|| },
// ||T|| ~ max |theta| over the nwant computed values and the opposite extreme
// Optionally *maxratio = max_i |beta_m| lastcomp[i] / (tol ||T||) over the
// same range (the distance to convergence of the slowest pair).
__global__ __launch_bounds__(64) void k_conv_count(const double *theta, const double *lastcomp,
                                                   const double *beta_m, int64_t nwant, int64_t i0,
                                                   int64_t cnt, int tn_extra, double tol, int *nconv,
                                                   double *maxratio)
{
    double tn = fmax(fmax(fabs(theta[0]), fabs(theta[nwant - 1])), fabs(theta[nwant]));
    if (tn_extra) tn = fmax(tn, fabs(theta[nwant + 1]));
    const double bm = fabs(*beta_m);
    int c = 0;
    double mr = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i0 + cnt; i += 64) {
        c += (bm * lastcomp[i] <= tol * tn);
        mr = fmax(mr, bm * lastcomp[i] / fmax(tol * tn, 0x1p-1000));
    }
    for (int o = 32; o > 0; o >>= 1) {
        c += __shfl_xor(c, o);
        mr = fmax(mr, __shfl_xor(mr, o));
    }
    if (threadIdx.x == 0) {
        *nconv = c;
        if (maxratio) *maxratio = mr;
    }
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

int launch_tri_bisect(const double *alpha, const double *beta, int64_t m, int64_t nwant, int which,
                      double *theta, hipStream_t st)
{
    hipLaunchKernelGGL(k_tri_bisect, dim3((unsigned)(nwant + 1)), dim3(64), 0, st, alpha, beta, m,
                       nwant, which, theta);
    return ok();
}

int launch_tri_bisect_range(const double *alpha, const double *beta, int64_t m, int64_t first,
                            int64_t count, int which, double *theta, hipStream_t st)
{
    hipLaunchKernelGGL(k_tri_bisect_range, dim3((unsigned)(count + 2)), dim3(64), 0, st, alpha, beta, m, first,
                       count, which, theta);
    return ok();
}

int launch_tri_vectors(const double *alpha, const double *beta, int64_t m, int64_t nwant,
                       const double *theta, double *S, int64_t lds, double *scratch, int clustered,
                       double *lastcomp, hipStream_t st)
{
    // convergence checks need only |e_m^T s_i|: two inverse iterations from a
    // random start suffice at converged Ritz values; Ritz vectors get three
    hipLaunchKernelGGL(k_tri_invit, dim3((unsigned)nwant), dim3(256), 0, st, alpha, beta, m, nwant,
                       theta, S, lds, scratch, lastcomp, S ? 3 : 2);
    if (ok()) return GSYEIG_EHIP;
    if (clustered && S) {
        hipLaunchKernelGGL(k_tri_cluster, dim3((unsigned)nwant), dim3(256), 0, st, m, nwant, theta, S,
                           lds, scratch, lastcomp);
        return ok();
    }
    return 0;
}

int launch_conv_count(const double *theta, const double *lastcomp, const double *beta_m,
                      int64_t nwant, int64_t i0, int64_t cnt, int tn_extra, double tol, int *nconv,
                      hipStream_t st, double *maxratio)
{
    hipLaunchKernelGGL(k_conv_count, dim3(1), dim3(64), 0, st, theta, lastcomp, beta_m, nwant, i0, cnt,
                       tn_extra, tol, nconv, maxratio);
    return ok();
}
