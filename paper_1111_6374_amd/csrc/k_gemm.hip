// k_gemm.hip -- FP64 dense tile contraction on CDNA4 matrix cores.
//
// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j) over logical indices,
// with each operand's storage chosen by a layout code (column-major,
// row-major, or symmetric-from-lower-triangle).  Used where the path is a
// dense contraction: the Cholesky panel and trailing SYRK update (Eq. 2),
// the Ritz vectors Y = V_m S (key KI5), the block back-substitution update
// (Eq. 4) and the FP64 residual check.
//
// Tiling: one 256-thread workgroup owns a 64x64 tile of C; its four wave64s
// each own a 32x32 quadrant = 2x2 blocks of v_mfma_f64_16x16x4_f64.  K is
// staged through LDS 16 at a time, the next slab prefetched into registers
// while the current one is multiplied.
#include "internal.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 16;
constexpr int LDS_PAD = 2;  // keeps the 16-wide operand reads on distinct banks

template <int L>
__device__ __forceinline__ double load_op(const double *p, int64_t ld, int64_t i, int64_t j,
                                          const double *diag)
{
    if constexpr (L == 0) return p[j * ld + i];
    else if constexpr (L == 1) return p[i * ld + j];
    else {
        if (i == j) return diag[i];
        return (i > j) ? p[i * ld + j] : p[j * ld + i];
    }
}

struct Args {
    int64_t m, n, k;
    const double *A; int64_t lda;
    const double *B; int64_t ldb;
    double *C; int64_t ldc; int c_row;
    double alpha, beta;
    const double *a_diag;
    int upper_only;
};

template <int AL, int BL>
__global__ __launch_bounds__(256) void k_gemm_f64(Args g)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t tm0 = (int64_t)blockIdx.x * TM;
    const int64_t tn0 = (int64_t)blockIdx.y * TN;
    if (g.upper_only && tm0 > tn0 + TN - 1) return;  // tile strictly below the diagonal

    __shared__ double As[TK][TM + LDS_PAD];
    __shared__ double Bs[TK][TN + LDS_PAD];

    // global -> register staging: 4 elements of A and 4 of B per thread
    double ra[4], rb[4];
    auto fetch = [&](int64_t k0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int ii, kk;
            if constexpr (AL == 0) { ii = tid & 63; kk = (tid >> 6) + 4 * p; }
            else { kk = tid & 15; ii = (tid >> 4) + 16 * p; }
            const int64_t gi = tm0 + ii, gk = k0 + kk;
            ra[p] = (gi < g.m && gk < g.k) ? load_op<AL>(g.A, g.lda, gi, gk, g.a_diag) : 0.0;
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int kk, jj;
            if constexpr (BL == 1) { jj = tid & 63; kk = (tid >> 6) + 4 * p; }
            else { kk = tid & 15; jj = (tid >> 4) + 16 * p; }
            const int64_t gk = k0 + kk, gj = tn0 + jj;
            rb[p] = (gk < g.k && gj < g.n) ? load_op<BL>(g.B, g.ldb, gk, gj, nullptr) : 0.0;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int ii, kk;
            if constexpr (AL == 0) { ii = tid & 63; kk = (tid >> 6) + 4 * p; }
            else { kk = tid & 15; ii = (tid >> 4) + 16 * p; }
            As[kk][ii] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int kk, jj;
            if constexpr (BL == 1) { jj = tid & 63; kk = (tid >> 6) + 4 * p; }
            else { kk = tid & 15; jj = (tid >> 4) + 16 * p; }
            Bs[kk][jj] = rb[p];
        }
    };

    const int wm = wave & 1, wn = wave >> 1;
    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};

    const int li = lane & 15, lk = lane >> 4;
    fetch(0);
    for (int64_t k0 = 0; k0 < g.k; k0 += TK) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + TK < g.k) fetch(k0 + TK);
#pragma unroll
        for (int kq = 0; kq < TK / 4; ++kq) {
            const int kr = kq * 4 + lk;
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kr][wm * 32 + a * 16 + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kr][wn * 32 + b * 16 + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }

    // D layout of the FP64 16x16 block: lane holds column (lane & 15) and
    // rows (lane >> 4) + 4 r, r = 0..3 (checked on gfx950)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = tm0 + wm * 32 + a * 16 + lk + 4 * r;
                const int64_t j = tn0 + wn * 32 + b * 16 + li;
                if (i >= g.m || j >= g.n) continue;
                if (g.upper_only && i > j) continue;
                double *cp = g.c_row ? &g.C[i * g.ldc + j] : &g.C[j * g.ldc + i];
                double v = g.alpha * acc[a][b][r];
                if (g.beta != 0.0) v += g.beta * *cp;
                *cp = v;
            }
}

template <int AL, int BL>
int run(const Args &a, hipStream_t st)
{
    dim3 grid((unsigned)cdiv(a.m, TM), (unsigned)cdiv(a.n, TN));
    hipLaunchKernelGGL((k_gemm_f64<AL, BL>), grid, dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

}  // namespace

int launch_gemm_f64(const GemmDesc &d, hipStream_t st)
{
    if (d.m <= 0 || d.n <= 0) return 0;
    Args a{d.m, d.n, d.k, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.c_layout == 1,
           d.alpha, d.beta, d.a_diag, d.upper_only};
    if (d.k <= 0) {  // C = beta C: run with a zero-length K loop
        a.k = 0;
    }
    switch (d.a_layout * 2 + d.b_layout) {
        case 0: return run<0, 0>(a, st);
        case 1: return run<0, 1>(a, st);
        case 2: return run<1, 0>(a, st);
        case 3: return run<1, 1>(a, st);
        case 4: return run<2, 0>(a, st);
        case 5: return run<2, 1>(a, st);
        default: return GSYEIG_EHIP;
    }
}
