// k_check.hip -- FP64 accuracy of computed pairs, the metrics of the
// paper's Tables 3 and 7 plus the per-pair normwise backward error:
//   rho_F = ||A X - B X L||_F / max(||A||_F, ||B||_F)
//   omega = ||I - X^T B X||_F
//   eta_i = ||A x_i - l_i B x_i||_2 / ((||A||_F + |l_i| ||B||_F) ||x_i||_2)
// A X and B X come from the FP64 tile contraction; this file holds the
// reductions.
#include "internal.h"

namespace {

constexpr int FRO_ROWS = 16;  // rows per partial sum

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ double block_sum(double v, double *sbuf)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sbuf[0] + sbuf[1]) + (sbuf[2] + sbuf[3]);
}

// mode 0: full row-major matrix; mode 2: strict lower triangle counted twice
// plus diag[] squared.
__global__ __launch_bounds__(256) void k_fro_parts(const double *A, int64_t lda, int64_t n, int mode,
                                                   const double *diag, double *part)
{
    __shared__ double sbuf[4];
    double v = 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * FRO_ROWS;
    for (int rr = 0; rr < FRO_ROWS; ++rr) {
        const int64_t i = r0 + rr;
        if (i >= n) break;
        const double *row = A + i * lda;
        if (mode == 0) {
            for (int64_t j = threadIdx.x; j < n; j += 256) v = fma(row[j], row[j], v);
        } else {
            for (int64_t j = threadIdx.x; j < i; j += 256) v = fma(2.0 * row[j], row[j], v);
            if (threadIdx.x == 0) v = fma(diag[i], diag[i], v);
        }
    }
    v = block_sum(v, sbuf);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// column i: out[2i] = ||AX_i - l_i BX_i||^2, out[2i+1] = ||x_i||^2
__global__ __launch_bounds__(256) void k_check_cols(const double *AX, const double *BX, int64_t ldr,
                                                    const double *X, int64_t ldx, int64_t n,
                                                    const double *lam, double *out)
{
    __shared__ double sbuf[4];
    const int64_t i = blockIdx.x;
    const double l = lam[i];
    double r2 = 0.0, x2 = 0.0;
    for (int64_t t = threadIdx.x; t < n; t += 256) {
        const double r = AX[i * ldr + t] - l * BX[i * ldr + t];
        r2 = fma(r, r, r2);
        const double xv = X[i * ldx + t];
        x2 = fma(xv, xv, x2);
    }
    r2 = block_sum(r2, sbuf);
    x2 = block_sum(x2, sbuf);
    if (threadIdx.x == 0) {
        out[2 * i] = r2;
        out[2 * i + 1] = x2;
    }
}

// res[0] = eta_max, [1] = rho_F, [2] = omega, [3] = ||A||_F, [4] = ||B||_F
__global__ __launch_bounds__(256) void k_check_finalize(const double *cols, int64_t s, const double *G,
                                                        int64_t ldg, const double *partA, int PA,
                                                        const double *partB, int PB,
                                                        const double *lam, double *res)
{
    __shared__ double sbuf[4];
    double a = 0.0, b = 0.0;
    for (int p = threadIdx.x; p < PA; p += 256) a += partA[p];
    for (int p = threadIdx.x; p < PB; p += 256) b += partB[p];
    const double nA = sqrt(block_sum(a, sbuf));
    const double nB = sqrt(block_sum(b, sbuf));
    double emax = 0.0, rsum = 0.0;
    for (int64_t i = threadIdx.x; i < s; i += 256) {
        const double e = sqrt(cols[2 * i]) / ((nA + fabs(lam[i]) * nB) * sqrt(cols[2 * i + 1]));
        emax = fmax(emax, e);
        rsum += cols[2 * i];
    }
    for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[threadIdx.x >> 6] = emax;
    __syncthreads();
    emax = fmax(fmax(sbuf[0], sbuf[1]), fmax(sbuf[2], sbuf[3]));
    rsum = block_sum(rsum, sbuf);
    double o2 = 0.0;
    for (int64_t t = threadIdx.x; t < s * s; t += 256) {
        const int64_t i = t % s, j = t / s;
        const double d = ((i == j) ? 1.0 : 0.0) - G[j * ldg + i];
        o2 = fma(d, d, o2);
    }
    o2 = block_sum(o2, sbuf);
    if (threadIdx.x == 0) {
        res[0] = emax;
        res[1] = sqrt(rsum) / fmax(nA, nB);
        res[2] = sqrt(o2);
        res[3] = nA;
        res[4] = nB;
    }
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

int fro_parts(int64_t n) { return (int)cdiv(n, FRO_ROWS); }

int launch_fro_norm_parts(const double *A, int64_t lda, int64_t n, int mode, const double *diag,
                          double *part, hipStream_t st)
{
    hipLaunchKernelGGL(k_fro_parts, dim3((unsigned)fro_parts(n)), dim3(256), 0, st, A, lda, n, mode,
                       diag, part);
    return ok();
}

int launch_check_cols(const double *AX, const double *BX, int64_t ldr, const double *X, int64_t ldx,
                      int64_t n, int64_t s, const double *lam, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_cols, dim3((unsigned)s), dim3(256), 0, st, AX, BX, ldr, X, ldx, n, lam,
                       out);
    return ok();
}

int launch_check_finalize(const double *cols, int64_t s, const double *G, int64_t ldg,
                          const double *partA, int PA, const double *partB, int PB,
                          const double *lam, double *res, hipStream_t st)
{
    hipLaunchKernelGGL(k_check_finalize, dim3(1), dim3(256), 0, st, cols, s, G, ldg, partA, PA, partB,
                       PB, lam, res);
    return ok();
}
