// k_factor.hip -- Cholesky diagonal blocks (Eq. 2), diagonal-block inverses,
// block back-substitution X = U^-1 Y (Eq. 4) and sign normalisation.
//
// Storage: B/U row-major, U upper.  A row-major upper U viewed column-major
// is the lower factor L = U^T, so every kernel here reads row segments of U.
#include "internal.h"

namespace {

// One workgroup factors the kb-th diagonal block of B in LDS (right-looking
// on the upper triangle), writes U_kk back over B's upper triangle, and
// writes Dinv_kk = U_kk^-1 (64 x 64 row-major, zero outside the block).
// A non-positive pivot records the global 1-based index in *info (first
// failure wins) and is replaced by 1 so the sweep continues without NaNs.
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_diag(T *B, int64_t ldb, int64_t n, int64_t kb,
                                                    double *Dinv, int *info)
{
    __shared__ double a[NB][NB + 1];
    __shared__ double x[NB][NB + 1];
    const int tid = threadIdx.x;
    const int64_t r0 = kb * NB;
    const int r = (int)((n - r0) < NB ? (n - r0) : NB);
    for (int t = tid; t < NB * NB; t += 256) {
        const int i = t / NB, j = t % NB;
        a[i][j] = (i < r && j < r && j >= i) ? (double)B[(r0 + i) * ldb + r0 + j] : 0.0;
        x[i][j] = 0.0;
    }
    __shared__ double s_d[NB];
    // Right-looking on unscaled rows (the LDL^T form): step j subtracts
    // a_ji a_jl / p_j from a_il (j < i <= l), p_j = a_jj; row j is scaled by
    // 1 / sqrt(p_j) at the end.  Thread (g, l) = (tid >> 6, tid & 63) updates
    // column l in rows i = j + 1 + g, + 4, ...; one barrier per step.
    const int l = tid & 63, g = tid >> 6;
    for (int j = 0; j < r; ++j) {
        __syncthreads();
        double p = a[j][j];
        if (!(p > 0.0)) p = 1.0;  // recorded below; the sweep continues without NaNs
        if (l > j && l < r) {
            const double f = a[j][l] / p;
            for (int i = j + 1 + g; i <= l; i += 4) a[i][l] -= a[j][i] * f;
        }
    }
    __syncthreads();
    if (tid < 64) {
        double p = (tid < r) ? a[tid][tid] : 1.0;
        const bool bad = !(p > 0.0);
        if (bad) p = 1.0;
        s_d[tid] = sqrt(p);
        // the first non-positive pivot of the block (blocks run in order)
        const unsigned long long m = __ballot(bad);
        if (tid == 0 && m) atomicCAS(info, 0, (int)(r0 + __ffsll((long long)m)));
    }
    __syncthreads();
    for (int t = tid; t < NB * NB; t += 256) {
        const int i = t >> 6, c = t & 63;
        if (i < r && c < r && c > i) a[i][c] /= s_d[i];
    }
    __syncthreads();
    if (tid < r) a[tid][tid] = s_d[tid];
    __syncthreads();
    // inverse of the upper-triangular block, one column per thread
    if (tid < r) {
        const int j = tid;
        x[j][j] = 1.0 / a[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += a[i][k] * x[k][j];
            x[i][j] = -s / a[i][i];
        }
    }
    __syncthreads();
    for (int t = tid; t < NB * NB; t += 256) {
        const int i = t / NB, j = t % NB;
        if (i < r && j < r && j >= i) B[(r0 + i) * ldb + r0 + j] = (T)a[i][j];
        Dinv[kb * NB * NB + t] = (i < r && j < r) ? x[i][j] : 0.0;
    }
}

// Dinv_I = U_II^-1 for every diagonal block of an existing factor U.
template <typename T>
__global__ __launch_bounds__(256) void k_diag_inv(const T *U, int64_t ldu, int64_t n, double *Dinv)
{
    __shared__ double a[NB][NB + 1];
    __shared__ double x[NB][NB + 1];
    const int tid = threadIdx.x;
    const int64_t kb = blockIdx.x;
    const int64_t r0 = kb * NB;
    const int r = (int)((n - r0) < NB ? (n - r0) : NB);
    for (int t = tid; t < NB * NB; t += 256) {
        const int i = t / NB, j = t % NB;
        a[i][j] = (i < r && j < r && j >= i) ? (double)U[(r0 + i) * ldu + r0 + j] : 0.0;
        x[i][j] = 0.0;
    }
    __syncthreads();
    if (tid < r) {
        const int j = tid;
        x[j][j] = 1.0 / a[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += a[i][k] * x[k][j];
            x[i][j] = -s / a[i][i];
        }
    }
    __syncthreads();
    for (int t = tid; t < NB * NB; t += 256) {
        const int i = t / NB, j = t % NB;
        Dinv[kb * NB * NB + t] = (i < r && j < r) ? x[i][j] : 0.0;
    }
}

__global__ void k_copy_diag(const double *B, int64_t ldb, int64_t n, double *d)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = B[i * ldb + i];
}

// X_kb := Dinv_kb Y_kb in place for s columns (column-major Y); each
// workgroup owns four whole columns, so no other workgroup touches them.
__global__ __launch_bounds__(256) void k_trsm_diag(const double *Dinv_kb, int r, double *Yk,
                                                   int64_t ldy, int64_t s)
{
    __shared__ double y[4][NB];
    const int tid = threadIdx.x;
    const int c = tid >> 6, i = tid & 63;
    const int64_t col = (int64_t)blockIdx.x * 4 + c;
    const bool live = col < s;
    y[c][i] = (live && i < r) ? Yk[col * ldy + i] : 0.0;
    __syncthreads();
    if (!live || i >= r) return;
    double acc = 0.0;
    for (int k = i; k < r; ++k) acc += Dinv_kb[i * NB + k] * y[c][k];
    Yk[col * ldy + i] = acc;
}

// Column i: find the entry of largest magnitude (lowest index on ties) and
// flip the column if it is negative.
__global__ __launch_bounds__(256) void k_sign_normalise(double *X, int64_t ldx, int64_t n)
{
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double *x = X + (int64_t)blockIdx.x * ldx;
    const int tid = threadIdx.x;
    double best = -1.0;
    int64_t bi = n;
    for (int64_t i = tid; i < n; i += 256) {
        const double v = fabs(x[i]);
        if (v > best) { best = v; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) {
            const double v2 = sv[tid + off];
            const int64_t i2 = si[tid + off];
            if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
        }
        __syncthreads();
    }
    const int64_t p = si[0];
    if (p >= n) return;
    const bool flip = x[p] < 0.0;
    __syncthreads();
    if (flip)
        for (int64_t i = tid; i < n; i += 256) x[i] = -x[i];
}

// W = fl32(upper triangle of B), zero below the diagonal; row r per blockIdx.y
__global__ void k_upper_to_f32(const double *__restrict__ B, int64_t ldb, float *__restrict__ W,
                               int64_t ldw, int64_t n, int64_t r0)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = r0 + blockIdx.y;
    if (c < n && r < n) W[r * ldw + c] = (c >= r) ? (float)B[r * ldb + c] : 0.0f;
}

}  // namespace

int launch_upper_to_f32(const double *B, int64_t ldb, float *W, int64_t ldw, int64_t n, hipStream_t st)
{
    for (int64_t r0 = 0; r0 < n; r0 += 65535) {
        const int64_t nr = std::min<int64_t>(65535, n - r0);
        hipLaunchKernelGGL(k_upper_to_f32, dim3((unsigned)cdiv(n, 256), (unsigned)nr), dim3(256), 0, st, B,
                           ldb, W, ldw, n, r0);
        if (hipGetLastError() != hipSuccess) return GSYEIG_EHIP;
    }
    return 0;
}

int launch_potrf_diag(double *B, int64_t ldb, int64_t n, int64_t kb, double *Dinv, int *info,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_potrf_diag<double>, dim3(1), dim3(256), 0, st, B, ldb, n, kb, Dinv, info);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_potrf_diag_f32(float *B, int64_t ldb, int64_t n, int64_t kb, double *Dinv, int *info,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_potrf_diag<float>, dim3(1), dim3(256), 0, st, B, ldb, n, kb, Dinv, info);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_diag_inv(const double *U, int64_t ldu, int64_t n, double *Dinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_inv<double>, dim3((unsigned)cdiv(n, NB)), dim3(256), 0, st, U, ldu, n, Dinv);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_diag_inv_f32(const float *U, int64_t ldu, int64_t n, double *Dinv, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_inv<float>, dim3((unsigned)cdiv(n, NB)), dim3(256), 0, st, U, ldu, n, Dinv);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_copy_diag(const double *B, int64_t ldb, int64_t n, double *d, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_diag, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, B, ldb, n, d);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

// X = U^-1 Y by block back-substitution from the last block row up:
//   X_kb = Dinv_kb Y_kb;   Y_{0:kb} -= U_{0:kb, kb} X_kb  (MFMA update, FP64).
// U may be stored FP64 or FP32; right-hand sides and arithmetic are FP64.
template <typename T>
static int backsolve_t(const T *U, int64_t ldu, int64_t n, int64_t s, const double *Dinv, double *Y,
                       int64_t ldy, hipStream_t st)
{
    const int64_t nblk = cdiv(n, NB);
    for (int64_t kb = nblk - 1; kb >= 0; --kb) {
        const int64_t r0 = kb * NB;
        const int r = (int)((n - r0) < NB ? (n - r0) : NB);
        hipLaunchKernelGGL(k_trsm_diag, dim3((unsigned)cdiv(s, 4)), dim3(256), 0, st,
                           Dinv + kb * NB * NB, r, Y + r0, ldy, s);
        if (hipGetLastError() != hipSuccess) return GSYEIG_EHIP;
        if (kb == 0) break;
        GemmDesc d{};
        d.m = r0; d.n = s; d.k = r;
        d.A = U + r0; d.lda = ldu; d.a_layout = 1;          // A(i,k) = U[i, r0 + k]
        d.a_f32 = sizeof(T) == 4;
        d.B = Y + r0; d.ldb = ldy; d.b_layout = 0;          // B(k,j) = X[r0 + k, j]
        d.C = Y; d.ldc = ldy; d.c_layout = 0;
        d.alpha = -1.0; d.beta = 1.0;
        if (launch_gemm(d, st)) return GSYEIG_EHIP;
    }
    return 0;
}

int launch_backsolve(const double *U, int64_t ldu, int64_t n, int64_t s, const double *Dinv,
                     double *Y, int64_t ldy, hipStream_t st)
{
    return backsolve_t<double>(U, ldu, n, s, Dinv, Y, ldy, st);
}

int launch_backsolve_f32(const float *U, int64_t ldu, int64_t n, int64_t s, const double *Dinv,
                         double *Y, int64_t ldy, hipStream_t st)
{
    return backsolve_t<float>(U, ldu, n, s, Dinv, Y, ldy, st);
}

int launch_sign_normalise(double *X, int64_t ldx, int64_t n, int64_t s, hipStream_t st)
{
    if (s <= 0) return 0;
    hipLaunchKernelGGL(k_sign_normalise, dim3((unsigned)s), dim3(256), 0, st, X, ldx, n);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}
