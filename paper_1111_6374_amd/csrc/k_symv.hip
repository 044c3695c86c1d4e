// k_symv.hip -- y = A x for symmetric A in full storage, key KI2 of
// variant KI (Table 1), reading only the upper triangle (n(n+1)/2 values).
//
// Work items are runs of up to SYMV_CH 64x64 tiles along one block row I of
// the upper triangle.  Each tile A_IJ (J >= I) is loaded once and used twice:
//   row part     y_I += A_IJ x_J           (summed over the run)
//   column part  y_J += A_IJ^T x_I  (J > I; the diagonal tile is applied
//                                    once, from full storage)
// Partial results go to a scratch area and a second kernel sums them in a
// fixed order, so the result is bitwise reproducible run to run.  A may be
// stored in FP64 or FP32 (mixed mode); arithmetic and vectors are FP64.
#include <mutex>
#include <vector>

#include "internal.h"

#define SYMV_CH 4

namespace {

__global__ __launch_bounds__(256) void k_symv_tiles(const double *__restrict__ A, int64_t lda,
                                                    int64_t n, int nblk, int maxch,
                                                    const double *__restrict__ x,
                                                    const int2 *__restrict__ items,
                                                    double *__restrict__ Pr,
                                                    double *__restrict__ Pc)
{
    __shared__ double s_part[4][NB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int2 it = items[blockIdx.x];
    const int I = it.x, J0 = it.y;
    const int J1 = (J0 + SYMV_CH < nblk) ? J0 + SYMV_CH : nblk;
    const int64_t r0 = (int64_t)I * NB;
    const int c = 16 * w + (lane & 15);
    const int rg = lane >> 4;
    const double *Arow = A + (r0 + rg) * lda;

    double a[SYMV_CH][16], xj[SYMV_CH];
#pragma unroll
    for (int t = 0; t < SYMV_CH; ++t) {
        const int J = J0 + t;
        const int64_t col = (int64_t)J * NB + c;
        const bool colok = (J < J1) && (col < n);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const bool ok = colok && (r0 + rg + 4 * q < n);
            a[t][q] = ok ? Arow[(int64_t)(4 * q) * lda + col] : 0.0;
        }
        xj[t] = colok ? x[col] : 0.0;
    }
    double xi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) xi[q] = (r0 + rg + 4 * q < n) ? x[r0 + rg + 4 * q] : 0.0;

    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
#pragma unroll
    for (int t = 0; t < SYMV_CH; ++t) {
        const int J = J0 + t;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = fma(a[t][q], xj[t], acc[q]);
        if (J < J1 && J > I) {
            double cs = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) cs = fma(a[t][q], xi[q], cs);
            cs += __shfl_xor(cs, 16);
            cs += __shfl_xor(cs, 32);
            if (rg == 0) Pc[((int64_t)J * nblk + I) * NB + c] = cs;
        }
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double v = acc[q];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        acc[q] = v;
    }
    if ((lane & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) s_part[w][rg + 4 * q] = acc[q];
    }
    __syncthreads();
    if (tid < NB) {
        const int ch = (J0 - I) / SYMV_CH;
        Pr[((int64_t)I * maxch + ch) * NB + tid] =
            s_part[0][tid] + s_part[1][tid] + s_part[2][tid] + s_part[3][tid];
    }
}

// The same work items with A stored FP32.  Each lane loads two adjacent
// columns (8 bytes) and 32 lanes cover a whole 64-column tile row (two full
// 128-byte lines), so one wave instruction reads two complete tile rows:
// lane & 31 picks the column pair, rg = 2 w + (lane >> 5) one of 8 row
// groups (rows rg + 8 q, q < 8).  Column partials of the four waves are
// folded in LDS in a fixed order.  Every load is issued unconditionally from
// a clamped in-bounds address and masked afterwards, so the loads of a work
// item are all in flight together.  PAIR (lda even): 8-byte pair loads; a
// pair that starts inside a row of length lda >= n+1 stays inside the row.
template <bool PAIR>
__global__ __launch_bounds__(256) void k_symv_tiles_f32(const float *__restrict__ A, int64_t lda,
                                                        int64_t n, int nblk, int maxch,
                                                        const double *__restrict__ x,
                                                        const int2 *__restrict__ items,
                                                        double *__restrict__ Pr,
                                                        double *__restrict__ Pc)
{
    __shared__ double s_col[4][NB];
    __shared__ double s_row[NB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int2 it = items[blockIdx.x];
    const int I = it.x, J0 = it.y;
    const int J1 = (J0 + SYMV_CH < nblk) ? J0 + SYMV_CH : nblk;
    const int64_t r0 = (int64_t)I * NB;
    const int c = 2 * (lane & 31);          // first of the lane's two columns in the tile
    const int rg = 2 * w + (lane >> 5);     // row group: rows rg + 8 q
    float2 a[SYMV_CH][8];  // kept FP32 in registers, widened at the multiply
    double xj[SYMV_CH][2];
#pragma unroll
    for (int t = 0; t < SYMV_CH; ++t) {
        const int J = J0 + t;
        const int64_t col = (int64_t)J * NB + c;
        const bool live = J < J1;
        const bool c0ok = live && col < n, c1ok = live && col + 1 < n;
        const int64_t cc = c0ok ? col : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t row = r0 + rg + 8 * q;
            const bool rok = row < n;
            const float *p = A + (rok ? row : 0) * lda + cc;
            float2 v;
            if constexpr (PAIR) {
                v = *reinterpret_cast<const float2 *>(p);
            } else {
                v.x = p[0];
                v.y = p[c1ok ? 1 : 0];
            }
            a[t][q].x = (rok && c0ok) ? v.x : 0.0f;
            a[t][q].y = (rok && c1ok) ? v.y : 0.0f;
        }
        xj[t][0] = c0ok ? x[col] : 0.0;
        xj[t][1] = c1ok ? x[col + 1] : 0.0;
    }
    double xi[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xi[q] = (r0 + rg + 8 * q < n) ? x[r0 + rg + 8 * q] : 0.0;

    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
#pragma unroll
    for (int t = 0; t < SYMV_CH; ++t) {
        const int J = J0 + t;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            acc[q] = fma((double)a[t][q].y, xj[t][1], fma((double)a[t][q].x, xj[t][0], acc[q]));
        if (J < J1 && J > I) {  // uniform over the workgroup
            double c0 = 0.0, c1 = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                c0 = fma((double)a[t][q].x, xi[q], c0);
                c1 = fma((double)a[t][q].y, xi[q], c1);
            }
            c0 += __shfl_xor(c0, 32);
            c1 += __shfl_xor(c1, 32);
            if (lane < 32) {
                s_col[w][c] = c0;
                s_col[w][c + 1] = c1;
            }
            __syncthreads();
            if (tid < NB)
                Pc[((int64_t)J * nblk + I) * NB + tid] = (s_col[0][tid] + s_col[1][tid]) + (s_col[2][tid] + s_col[3][tid]);
            __syncthreads();
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double v = acc[q];
        for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
        acc[q] = v;
    }
    if ((lane & 31) == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) s_row[rg + 8 * q] = acc[q];
    }
    __syncthreads();
    if (tid < NB) {
        const int ch = (J0 - I) / SYMV_CH;
        Pr[((int64_t)I * maxch + ch) * NB + tid] = s_row[tid];
    }
}

// FP64 A with lda and n even: 16-byte loads of column pairs.  Lane ->
// columns cp = 2 (lane & 31), cp + 1 of a tile and row group rg = 2 w +
// (lane >> 5) (rows rg + 8 q, q < 8), so one wave instruction reads two whole
// 512-byte tile rows.  Row parts are summed inside the wave, column parts of
// the four waves meet once in LDS in a fixed order; x_J is staged in LDS.
// Loads come from clamped in-bounds addresses and are masked by bits (with
// n even a column pair is wholly inside or wholly outside the matrix).
template <int CH>
__global__ __launch_bounds__(256) void k_symv_tiles_q(const double *__restrict__ A, int64_t lda, int64_t n,
                                                      int nblk, int maxch, const double *__restrict__ x,
                                                      const int2 *__restrict__ items, double *__restrict__ Pr,
                                                      double *__restrict__ Pc)
{
    __shared__ double s_x[CH * NB];
    __shared__ double s_col[CH][4][NB];
    __shared__ double s_row[NB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int2 it = items[blockIdx.x];
    const int I = it.x, J0 = it.y;
    const int J1 = (J0 + CH < nblk) ? J0 + CH : nblk;
    const int64_t r0 = (int64_t)I * NB;
    const int cp = 2 * (lane & 31);
    const int rg = 2 * w + (lane >> 5);
    double2 a[CH][8];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const int64_t col = (int64_t)(J0 + t) * NB + cp;
        const bool cok = (J0 + t < J1) && col < n;
        const int64_t cc = cok ? col : 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t row = r0 + rg + 8 * q;
            const unsigned long long m = (cok && row < n) ? ~0ull : 0ull;
            const double2 v = *reinterpret_cast<const double2 *>(A + (row < n ? row : 0) * lda + cc);
            a[t][q].x = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v.x) & m));
            a[t][q].y = __longlong_as_double((long long)((unsigned long long)__double_as_longlong(v.y) & m));
        }
    }
    for (int e = tid; e < CH * NB; e += 256) {
        const int64_t col = (int64_t)J0 * NB + e;
        s_x[e] = (J0 + e / NB < J1 && col < n) ? x[col] : 0.0;
    }
    double xi[8], acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t row = r0 + rg + 8 * q;
        xi[q] = (row < n) ? x[row] : 0.0;
        acc[q] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const double x0 = s_x[t * NB + cp], x1 = s_x[t * NB + cp + 1];
        double c0 = 0.0, c1 = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc[q] = fma(a[t][q].y, x1, fma(a[t][q].x, x0, acc[q]));
            c0 = fma(a[t][q].x, xi[q], c0);
            c1 = fma(a[t][q].y, xi[q], c1);
        }
        c0 += __shfl_xor(c0, 32);
        c1 += __shfl_xor(c1, 32);
        if (lane < 32) {
            s_col[t][w][cp] = c0;
            s_col[t][w][cp + 1] = c1;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        double v = acc[q];
        for (int o = 1; o < 32; o <<= 1) v += __shfl_xor(v, o);
        acc[q] = v;
    }
    if ((lane & 31) == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) s_row[rg + 8 * q] = acc[q];
    }
    __syncthreads();
    if (tid < NB) {
        const int ch = (J0 - I) / CH;
        Pr[((int64_t)I * maxch + ch) * NB + tid] = s_row[tid];
    }
    for (int e = tid; e < CH * NB; e += 256) {
        const int t = e / NB, c = e % NB, J = J0 + t;
        if (J < J1 && J > I)
            Pc[((int64_t)J * nblk + I) * NB + c] = (s_col[t][0][c] + s_col[t][1][c]) + (s_col[t][2][c] + s_col[t][3][c]);
    }
}

// The same product with A stored FP32, lda and n multiples of 4: 16-byte
// loads.  Lane -> column quad cl = 4 (lane & 15) of a tile and row group
// rg = 4 w + (lane >> 4) (rows rg + 16 q, q < 4), so one wave instruction
// reads four whole 256-byte tile rows.  A row part is summed inside its wave
// (over the 16 column quads); column parts of the four waves meet once in
// LDS, in a fixed order.  x_J of the CH tiles is staged in LDS while the
// tile loads are in flight.  Every load is issued from a clamped in-bounds
// address and masked afterwards (with n % 4 == 0 a column quad is wholly
// inside or wholly outside the matrix).
template <int CH>
__global__ __launch_bounds__(256) void k_symv_tiles_f32q(const float *__restrict__ A, int64_t lda,
                                                         int64_t n, int nblk, int maxch,
                                                         const double *__restrict__ x,
                                                         const int2 *__restrict__ items,
                                                         double *__restrict__ Pr,
                                                         double *__restrict__ Pc)
{
    __shared__ double s_x[CH * NB];
    __shared__ double s_col[CH][4][NB];
    __shared__ double s_row[NB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int2 it = items[blockIdx.x];
    const int I = it.x, J0 = it.y;
    const int J1 = (J0 + CH < nblk) ? J0 + CH : nblk;
    const int64_t r0 = (int64_t)I * NB;
    const int cl = 4 * (lane & 15);
    const int rg = 4 * w + (lane >> 4);
    float4 a[CH][4];
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const int64_t col = (int64_t)(J0 + t) * NB + cl;
        const bool cok = (J0 + t < J1) && col < n;
        const int64_t cc = cok ? col : 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t row = r0 + rg + 16 * q;
            // mask by bits, not by a select, so that no load is predicated
            const unsigned m = (cok && row < n) ? 0xffffffffu : 0u;
            const float4 v = *reinterpret_cast<const float4 *>(A + (row < n ? row : 0) * lda + cc);
            a[t][q] = make_float4(__uint_as_float(__float_as_uint(v.x) & m), __uint_as_float(__float_as_uint(v.y) & m),
                                  __uint_as_float(__float_as_uint(v.z) & m), __uint_as_float(__float_as_uint(v.w) & m));
        }
    }
    for (int e = tid; e < CH * NB; e += 256) {
        const int64_t col = (int64_t)J0 * NB + e;
        s_x[e] = (J0 + e / NB < J1 && col < n) ? x[col] : 0.0;
    }
    double xi[4], acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t row = r0 + rg + 16 * q;
        xi[q] = (row < n) ? x[row] : 0.0;
        acc[q] = 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < CH; ++t) {
        const double x0 = s_x[t * NB + cl], x1 = s_x[t * NB + cl + 1];
        const double x2 = s_x[t * NB + cl + 2], x3 = s_x[t * NB + cl + 3];
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = a[t][q];
            acc[q] = fma((double)v.w, x3, fma((double)v.z, x2, fma((double)v.y, x1, fma((double)v.x, x0, acc[q]))));
            c0 = fma((double)v.x, xi[q], c0);
            c1 = fma((double)v.y, xi[q], c1);
            c2 = fma((double)v.z, xi[q], c2);
            c3 = fma((double)v.w, xi[q], c3);
        }
        c0 += __shfl_xor(c0, 16);
        c1 += __shfl_xor(c1, 16);
        c2 += __shfl_xor(c2, 16);
        c3 += __shfl_xor(c3, 16);
        c0 += __shfl_xor(c0, 32);
        c1 += __shfl_xor(c1, 32);
        c2 += __shfl_xor(c2, 32);
        c3 += __shfl_xor(c3, 32);
        if (lane < 16) {
            s_col[t][w][cl] = c0;
            s_col[t][w][cl + 1] = c1;
            s_col[t][w][cl + 2] = c2;
            s_col[t][w][cl + 3] = c3;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double v = acc[q];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        acc[q] = v;
    }
    if ((lane & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) s_row[rg + 16 * q] = acc[q];
    }
    __syncthreads();
    if (tid < NB) {
        const int ch = (J0 - I) / CH;
        Pr[((int64_t)I * maxch + ch) * NB + tid] = s_row[tid];
    }
    for (int e = tid; e < CH * NB; e += 256) {
        const int t = e / NB, c = e % NB, J = J0 + t;
        if (J < J1 && J > I)
            Pc[((int64_t)J * nblk + I) * NB + c] = (s_col[t][0][c] + s_col[t][1][c]) + (s_col[t][2][c] + s_col[t][3][c]);
    }
}

// y_K = sum of the row parts of block row K + column parts of tiles (I, K),
// I < K.  256 threads: thread (q, t) sums every 4th partial of element t,
// reading 2 KB of contiguous partials per step; a fixed-order LDS fold ends it.
__global__ __launch_bounds__(256) void k_symv_reduce(const double *__restrict__ Pr,
                                                     const double *__restrict__ Pc, int nblk,
                                                     int maxch, int64_t n, double *__restrict__ y, int ch)
{
    __shared__ double sred[4][NB];
    const int K = blockIdx.x, t = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int nch = (nblk - K + ch - 1) / ch;
    double s = 0.0;
    for (int ch = q; ch < nch; ch += 4) s += Pr[((int64_t)K * maxch + ch) * NB + t];
    const double *pc = Pc + (int64_t)K * nblk * NB + t;
    int I = q;
    for (; I + 12 < K; I += 16) {
        const double a0 = pc[(int64_t)I * NB], a1 = pc[(int64_t)(I + 4) * NB];
        const double a2 = pc[(int64_t)(I + 8) * NB], a3 = pc[(int64_t)(I + 12) * NB];
        s += (a0 + a1) + (a2 + a3);
    }
    for (; I < K; I += 4) s += pc[(int64_t)I * NB];
    sred[q][t] = s;
    __syncthreads();
    if (q == 0) {
        const int64_t row = (int64_t)K * NB + t;
        if (row < n) y[row] = (sred[0][t] + sred[1][t]) + (sred[2][t] + sred[3][t]);
    }
}

}  // namespace

// Launch of the tile pass over the work list `items` (nitems runs of up to
// SYMV_CH tiles), partials into Pr (nblk x maxch x 64) and Pc (nblk x nblk
// x 64); the kernel variant follows the storage type and alignment of A.
template <typename T>
static int symv_tiles_launch(hipStream_t st, int64_t n, const T *A, int64_t lda, const double *x, const int2 *items,
                             int64_t nitems, double *pr, double *pc, int maxch)
{
    const int nblk = (int)cdiv(n, NB);
    // FP32 storage with 16-byte rows of 4: the quad-load kernel (measured
    // 0.441 ms against 0.547 ms for the pair-load one at n = 32768, MI355X)
    const bool quad = sizeof(T) == 4 && lda % 4 == 0 && n % 4 == 0;
    const dim3 grid((unsigned)nitems);
    if constexpr (sizeof(T) == 8) {
        // 16-byte column pairs when rows and n are even (measured 0.203 ms
        // against 0.230 ms for the 8-byte kernel at n = 16384, MI355X)
        if (lda % 2 == 0 && n % 2 == 0)
            hipLaunchKernelGGL(k_symv_tiles_q<SYMV_CH>, grid, dim3(256), 0, st, A, lda, n, nblk, maxch, x, items, pr,
                               pc);
        else
            hipLaunchKernelGGL(k_symv_tiles, grid, dim3(256), 0, st, A, lda, n, nblk, maxch, x, items, pr, pc);
    } else if (quad)
        hipLaunchKernelGGL(k_symv_tiles_f32q<SYMV_CH>, grid, dim3(256), 0, st, A, lda, n, nblk, maxch, x, items, pr,
                           pc);
    else if (lda % 2 == 0)
        hipLaunchKernelGGL(k_symv_tiles_f32<true>, grid, dim3(256), 0, st, A, lda, n, nblk, maxch, x, items, pr, pc);
    else
        hipLaunchKernelGGL(k_symv_tiles_f32<false>, grid, dim3(256), 0, st, A, lda, n, nblk, maxch, x, items, pr,
                           pc);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

// The tile pass of y = A x: partials into Pr / Pc (maxch chunk slots of
// SYMV_CH tiles per block row), summed by k_symv_reduce or by the KI3 sweep.
template <typename T>
static int symv_tiles_t(gsyeig_ctx *ctx, int64_t n, const T *A, int64_t lda, const double *x, double **Pr_out,
                        double **Pc_out, int *maxch_out)
{
    const int nblk = (int)cdiv(n, NB);
    const int ch = SYMV_CH;
    const int maxch = (int)cdiv(nblk, ch);
    int rc;
    if (ctx->symv_map_n != n) {
        std::vector<int2> items;
        for (int I = 0; I < nblk; ++I)
            for (int J0 = I; J0 < nblk; J0 += ch) items.push_back(make_int2(I, J0));
        void *p;
        if ((rc = ws_get(ctx, WS_SYMVMAP, items.size() * sizeof(int2), &p))) return rc;
        HIP_TRY(hipMemcpyAsync(p, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice,
                               ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->symv_map_n = n;
        ctx->symv_items = (int64_t)items.size();
    }
    void *pr, *pc;
    if ((rc = ws_get(ctx, WS_SYMV_PR, sizeof(double) * (size_t)nblk * maxch * NB, &pr))) return rc;
    if ((rc = ws_get(ctx, WS_SYMV_PC, sizeof(double) * (size_t)nblk * nblk * NB, &pc))) return rc;
    const int2 *items = (const int2 *)ctx->ws[WS_SYMVMAP];
    if ((rc = symv_tiles_launch<T>(ctx->stream, n, A, lda, x, items, ctx->symv_items, (double *)pr, (double *)pc,
                                   maxch)))
        return rc;
    *Pr_out = (double *)pr;
    *Pc_out = (double *)pc;
    *maxch_out = maxch;
    return 0;
}

template <typename T>
static int launch_symv_t(gsyeig_ctx *ctx, int64_t n, const T *A, int64_t lda, const double *x, double *y)
{
    double *pr, *pc;
    int maxch, rc;
    if ((rc = symv_tiles_t<T>(ctx, n, A, lda, x, &pr, &pc, &maxch))) return rc;
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_symv_reduce, dim3(nblk), dim3(256), 0, ctx->stream, (const double *)pr,
                       (const double *)pc, nblk, maxch, n, y, SYMV_CH);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_symv(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x, double *y)
{
    return launch_symv_t<double>(ctx, n, A, lda, x, y);
}

int launch_symv_f32(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x, double *y)
{
    return launch_symv_t<float>(ctx, n, A, lda, x, y);
}

int launch_symv_partials(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x, double **Pr,
                         double **Pc, int *maxch, int *ch)
{
    *ch = SYMV_CH;
    return symv_tiles_t<double>(ctx, n, A, lda, x, Pr, Pc, maxch);
}

int launch_symv_partials_f32(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x, double **Pr,
                             double **Pc, int *maxch, int *ch)
{
    *ch = SYMV_CH;
    return symv_tiles_t<float>(ctx, n, A, lda, x, Pr, Pc, maxch);
}

// ------------------------------------------------------------ KI2, no allocation
// gsyeig_symv_noalloc keeps the work list and the partials of the tile pass
// in one file-scope device array sized for n <= GSYEIG_NOALLOC_MAX_N; every
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel: its device address on the
// current device comes from hipGetSymbolAddress, once per device.
namespace {

constexpr int64_t NA_NBLK = GSYEIG_NOALLOC_MAX_N / NB;
constexpr int64_t NA_MAXCH = (NA_NBLK + SYMV_CH - 1) / SYMV_CH;
constexpr size_t NA_ITEMS_BYTES = ((size_t)NA_NBLK * NA_MAXCH * sizeof(int2) + 255) & ~(size_t)255;
constexpr size_t NA_PR_BYTES = (size_t)NA_NBLK * NA_MAXCH * NB * sizeof(double);
constexpr size_t NA_PC_BYTES = (size_t)NA_NBLK * NA_NBLK * NB * sizeof(double);
constexpr size_t NA_BYTES = NA_ITEMS_BYTES + NA_PR_BYTES + NA_PC_BYTES;
static_assert(GSYEIG_NOALLOC_MAX_N % NB == 0, "the maximum is a whole number of tiles");

}  // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

namespace {

constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
void *na_ptr[NA_MAX_DEVICES];

// The work list of the tile pass, the same runs in the same order as the
// host-built list of launch_symv: row I holds ceil((nblk - I) / ch) runs.
__global__ void k_symv_items(int2 *items, int nblk, int ch)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nblk) return;
    int64_t off = 0;
    for (int i = 0; i < I; ++i) off += (nblk - i + ch - 1) / ch;
    for (int J0 = I, t = 0; J0 < nblk; J0 += ch, ++t) items[off + t] = make_int2(I, J0);
}

}  // namespace

// Device address of the scratch array on the current device (resolved on
// the first use per device; the lock keeps concurrent first calls apart).
int noalloc_scratch(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEVICES) return GSYEIG_EHIP;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return GSYEIG_EHIP;
        }
        na_ptr[dev] = p;
    }
    *out = na_ptr[dev];
    return 0;
}

extern "C" int gsyeig_symv_noalloc(void *hip_stream, int64_t n, const double *A, int64_t lda, const double *x,
                                   double *y)
{
    if (n < 1) return -2;
    if (n > GSYEIG_NOALLOC_MAX_N) return GSYEIG_ETOOBIG;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!x) return -5;
    if (!y) return -6;
    void *base = nullptr;
    int rc;
    if ((rc = noalloc_scratch(&base))) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    const int nblk = (int)cdiv(n, NB);
    const int maxch = (int)cdiv(nblk, SYMV_CH);
    int64_t nitems = 0;
    for (int I = 0; I < nblk; ++I) nitems += cdiv(nblk - I, SYMV_CH);
    int2 *items = (int2 *)base;
    double *pr = (double *)((char *)base + NA_ITEMS_BYTES);
    double *pc = (double *)((char *)base + NA_ITEMS_BYTES + NA_PR_BYTES);
    // every scratch value is written before it is read: nothing to clear
    hipLaunchKernelGGL(k_symv_items, dim3((unsigned)cdiv(nblk, 64)), dim3(64), 0, st, items, nblk, SYMV_CH);
    if (hipGetLastError() != hipSuccess) return GSYEIG_EHIP;
    if ((rc = symv_tiles_launch<double>(st, n, A, lda, x, items, nitems, pr, pc, maxch))) return rc;
    hipLaunchKernelGGL(k_symv_reduce, dim3(nblk), dim3(256), 0, st, (const double *)pr, (const double *)pc, nblk,
                       maxch, n, y, SYMV_CH);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}
