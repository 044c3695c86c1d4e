// k_ke.hip -- key GS2 of the paper's variants KE and TD (Section 2.1,
// Table 1): the explicit standard-form matrix C = U^-T A U^-1 (Eq. 3),
// formed by two block triangular solves with all n columns as right-hand
// sides, so that the Lanczos loop of variant KE (Section 2.3) is one
// symmetric matrix-vector product per step.
//
//   T2 = U^-T A          (A symmetric: its row-major storage is its
//                         column-major storage)
//   T1 = T2^T = A U^-1   (tiled transpose through LDS)
//   C  = U^-T T1         = U^-T A U^-1
//   C  = (C + C^T) / 2   (exactly symmetric, as the SYMV's diagonal tiles
//                         read both triangles)
//
// The solves are the matrix-core block solves of the factor (right-looking
// over 512-row super-blocks with their explicit inverses), i.e. 2 n^3 flops
// of FP64 products; C is column-major with leading dimension ldc, which for
// a symmetric matrix is also its row-major storage.
#include <algorithm>

#include "internal.h"

namespace {

constexpr int TT = 64;  // transpose tile

// Y = X^T for n x n column-major X, Y (distinct buffers); 64x64 tiles
// through LDS (padded against bank conflicts), 256 threads per tile.
__global__ __launch_bounds__(256) void k_transpose(const double *__restrict__ X, int64_t ldx,
                                                   double *__restrict__ Y, int64_t ldy, int64_t n)
{
    __shared__ double t[TT][TT + 1];
    const int64_t i0 = (int64_t)blockIdx.x * TT, j0 = (int64_t)blockIdx.y * TT;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < TT; r += 4) {  // column j0 + r of X, rows i0 + tx
        const int64_t i = i0 + tx, j = j0 + r;
        t[r][tx] = (i < n && j < n) ? X[j * ldx + i] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < TT; r += 4) {  // column i0 + r of Y, rows j0 + tx
        const int64_t i = j0 + tx, j = i0 + r;
        if (i < n && j < n) Y[j * ldy + i] = t[tx][r];
    }
}

// C = (C + C^T) / 2 in place: one workgroup per tile pair (I, J), J >= I
// (blockIdx.x enumerates the upper block triangle), both tiles through LDS.
__global__ __launch_bounds__(256) void k_symmetrise_tiles(double *C, int64_t ldc, int64_t n, int nb)
{
    __shared__ double a[TT][TT + 1], b[TT][TT + 1];
    // tile index -> (I, J), J >= I, rows of the upper block triangle in order
    int64_t t = blockIdx.x;
    int I = 0;
    while (t >= nb - I) {
        t -= nb - I;
        ++I;
    }
    const int J = I + (int)t;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)I * TT, c0 = (int64_t)J * TT;
    for (int r = ty; r < TT; r += 4) {
        const int64_t i = r0 + tx, j = c0 + r;   // a[r][tx] = C(i, j): tile (I, J)
        a[r][tx] = (i < n && j < n) ? C[j * ldc + i] : 0.0;
        const int64_t i2 = c0 + tx, j2 = r0 + r; // b[r][tx] = C(i2, j2): tile (J, I)
        b[r][tx] = (i2 < n && j2 < n) ? C[j2 * ldc + i2] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < TT; r += 4) {
        // C(r0 + tx, c0 + r) and C(c0 + r, r0 + tx) both become the mean
        const double v = 0.5 * (a[r][tx] + b[tx][r]);
        const int64_t i = r0 + tx, j = c0 + r;
        if (i < n && j < n) {
            C[j * ldc + i] = v;
            C[i * ldc + j] = v;
        }
    }
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

int launch_transpose(const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t n, hipStream_t st)
{
    const unsigned nb = (unsigned)cdiv(n, TT);
    hipLaunchKernelGGL(k_transpose, dim3(nb, nb), dim3(256), 0, st, X, ldx, Y, ldy, n);
    return ok();
}

int launch_symmetrise(double *C, int64_t ldc, int64_t n, hipStream_t st)
{
    const int nb = (int)cdiv(n, TT);
    const int64_t tiles = (int64_t)nb * (nb + 1) / 2;
    hipLaunchKernelGGL(k_symmetrise_tiles, dim3((unsigned)tiles), dim3(256), 0, st, C, ldc, n, nb);
    return ok();
}

// GS2: C = U^-T A U^-1 into C (n x n, ldc), T a second n x n scratch (ldt).
// The factor is given as U = D (I + W) (W, sb from the super-block solves'
// side data) or, with W == nullptr, as U itself with its super-block
// inverses sb.  A is only read.
int form_c(const double *A, int64_t lda, const double *U, int64_t ldu, const double *W, int64_t ldw,
           const double *sb, int64_t n, double *C, int64_t ldc, double *T, int64_t ldt, hipStream_t st)
{
    int rc;
    auto solve_t = [&](double *V, int64_t ldv, double *X, int64_t ldx) {
        if (W) return launch_trsm_w(1, W, 0, ldw, n, sb, V, ldv, X, ldx, n, 0, st);
        return launch_trsm_sb(1, U, 0, ldu, n, sb, V, ldv, X, ldx, n, 0, st);
    };
    if ((rc = launch_blk_copy(A, lda, T, ldt, n, n, st))) return rc;    // T = A
    if ((rc = solve_t(T, ldt, C, ldc))) return rc;                      // C = U^-T A (T destroyed)
    if ((rc = launch_transpose(C, ldc, T, ldt, n, st))) return rc;      // T = A U^-1
    if ((rc = solve_t(T, ldt, C, ldc))) return rc;                      // C = U^-T A U^-1
    return launch_symmetrise(C, ldc, n, st);
}
