// k_trsv.hip -- triangular solves with the Cholesky factor, keys KI1 and KI3
// of variant KI (Section 2.3, Table 1):
//     KI1: x = U^-1 b   (back substitution, block rows from the bottom up)
//     KI3: x = U^-T b   (forward substitution with U^T, block columns)
//
// Both stream the n(n+1)/2 triangle of U once.  The dependency chain runs
// over the n/64 diagonal blocks, so each sweep is one persistent launch:
//   * workgroup slots are handed out by an atomic ticket in chain order, so a
//     workgroup only ever waits on blocks owned by workgroups that started
//     before it (forward progress without co-residency assumptions);
//   * block I streams its 64-row (KI1) or 64-column (KI3) panel of U; tiles
//     of U never wait, only the solved values they multiply do;
//   * solved values are published through a staging vector that is all
//     NaN-sentinel between launches: the producer writes each value with an
//     agent-scope atomic store and a consumer polls exactly the values it
//     needs until they are not the sentinel.  Every value carries its own
//     readiness, so no flags, fences or cache write-backs sit on the chain;
//   * the block solve is split around the chain: with Dinv_I = U_II^-1 and
//     M_I = Dinv_I U_{I,I+1} precomputed, y_I = Dinv_I (b_I - sum over the
//     far tiles) is formed while block I+1 is still being solved, and once
//     x_{I+1} arrives each wave finishes its own 4 rows of
//     x_I = y_I - M_I x_{I+1} with no workgroup barrier on the chain (the
//     U^-T sweep uses Dinv_I^T and M'_I = Dinv_I^T U_{I-1,I}^T the same way).
//     The last workgroup to retire restores the sentinels.
//
// Layout: 1024 threads = 16 wave64s per block.  In a 64x64 tile, wave w owns
// rows 4w..4w+3 and lane l owns column l, so every load instruction reads one
// full 512-byte row segment.  Tiles are consumed in groups of GRP: the
// values of a group are polled while the next group's tiles stream in, and
// all addresses are clamped in range so no branch separates the two.
#include "chain.h"

#define GRP 4

namespace {

using namespace chain;

// ------------------------------------------------------------------ KI1
__global__ __launch_bounds__(1024) void k_trsv_n(const double *__restrict__ U, int64_t ldu,
                                                 int64_t n, int nblk,
                                                 const double *__restrict__ Dinv,
                                                 const double *__restrict__ Mn,
                                                 const double *b, double *x, PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_r[NB];
    __shared__ double s_y[NB];
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = nblk - 1 - take_ticket(ctl, nblk);
    __syncthreads();
    const int I = s_blk;
    const int64_t r0 = (int64_t)I * NB;
    const bool has_next = I < nblk - 1;

    // Dinv_I: thread t -> row t>>4, columns (t&15)*4..+3;  M_I: rows 4w..4w+3, column l
    const int drow = tid >> 4, dq = tid & 15;
    double dinv[4], mrow[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dinv[k] = Dinv[(int64_t)I * NB * NB + drow * NB + dq * 4 + k];
#pragma unroll
    for (int r = 0; r < 4; ++r) mrow[r] = has_next ? Mn[(int64_t)I * NB * NB + (4 * w + r) * NB + l] : 0.0;

    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int ntile = nblk - 2 - I;  // far tiles j = nblk-1 .. I+2
    if (ntile > 0) {
        // rows 4w..4w+3 of block I all exist (block I is not the last one)
        const double *Ur = U + (r0 + 4 * w) * ldu;
        const int64_t cmax = n - 1;
        // tile index t (0-based from the right) -> column of this lane, clamped
        auto colof = [&](int t) {
            const int j = (t < ntile) ? nblk - 1 - t : I + 2;
            const int64_t cc = (int64_t)j * NB + l;
            return cc < cmax ? cc : cmax;
        };
        double cur[GRP][4], nxt[GRP][4];
#pragma unroll
        for (int g = 0; g < GRP; ++g) {
            const int64_t cc = colof(g);
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[g][r] = Ur[(int64_t)r * ldu + cc];
        }
        for (int t0 = 0; t0 < ntile; t0 += GRP) {
            unsigned long long v[GRP];
#pragma unroll
            for (int g = 0; g < GRP; ++g) v[g] = ld_bits(stage + colof(t0 + g));
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int64_t cc = colof(t0 + GRP + g);
#pragma unroll
                for (int r = 0; r < 4; ++r) nxt[g][r] = Ur[(int64_t)r * ldu + cc];
            }
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int t = t0 + g;
                const int64_t col = (int64_t)(nblk - 1 - t) * NB + l;
                const bool live = (t < ntile) && (col < n);
                const double xv = settle(v[g], stage + colof(t), ctl);
                const double xj = live ? xv : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = fma(cur[g][r], xj, acc[r]);
            }
#pragma unroll
            for (int g = 0; g < GRP; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = nxt[g][r];
        }
    }
    // y_I = Dinv_I (b_I - far row sums)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = wave_sum(acc[r]);
    if (l < 4) {
        const int row = 4 * w + l;
        const double a = (l == 0) ? acc[0] : (l == 1) ? acc[1] : (l == 2) ? acc[2] : acc[3];
        s_r[row] = ((r0 + row < n) ? b[r0 + row] : 0.0) - a;
    }
    __syncthreads();
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) y = fma(dinv[k], s_r[dq * 4 + k], y);
    y += __shfl_xor(y, 1);
    y += __shfl_xor(y, 2);
    y += __shfl_xor(y, 4);
    y += __shfl_xor(y, 8);
    if (dq == 0) s_y[drow] = y;
    __syncthreads();
    // chain: each wave finishes rows 4w..4w+3 of x_I = y_I - M_I x_{I+1}
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (has_next) {
        const int64_t cn = (int64_t)(I + 1) * NB + l;
        const int64_t cc = cn < n ? cn : n - 1;
        const double xv = settle(ld_bits(stage + cc), stage + cc, ctl);
        const double xn = (cn < n) ? xv : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) part[r] = wave_sum(mrow[r] * xn);
    }
    if (l < 4) {
        const int row = 4 * w + l;
        const double p = (l == 0) ? part[0] : (l == 1) ? part[1] : (l == 2) ? part[2] : part[3];
        if (r0 + row < n) {
            const double xi = s_y[row] - p;
            st_bits(stage + r0 + row, (unsigned long long)__double_as_longlong(xi));
            x[r0 + row] = xi;
        }
    }
    retire(ctl, stage, n, nblk, &s_last);
}

// ------------------------------------------------------------------ KI3
__global__ __launch_bounds__(1024) void k_trsv_t(const double *__restrict__ U, int64_t ldu,
                                                 int64_t n, int nblk,
                                                 const double *__restrict__ Dinv,
                                                 const double *__restrict__ Mt,
                                                 const double *b, double *x, PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_part[16][NB];
    __shared__ double s_r[NB];
    __shared__ double s_y[NB];
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = take_ticket(ctl, nblk);
    __syncthreads();
    const int I = s_blk;
    const int64_t c0 = (int64_t)I * NB;
    const int64_t col = c0 + l;
    const bool colok = col < n;
    const int64_t colc = colok ? col : n - 1;

    // Dinv_I^T: thread t -> output column t>>4, rows (t&15)*4..+3; M'_I: rows 4w..4w+3, column l
    const int dcol = tid >> 4, dq = tid & 15;
    double dinv[4], mrow[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) dinv[k] = Dinv[(int64_t)I * NB * NB + (dq * 4 + k) * NB + dcol];
#pragma unroll
    for (int r = 0; r < 4; ++r) mrow[r] = (I > 0) ? Mt[(int64_t)I * NB * NB + (4 * w + r) * NB + l] : 0.0;

    double acc = 0.0;
    const int ntile = I - 1;  // far tiles j = 0 .. I-2
    if (ntile > 0) {
        // tile j covers rows j*64 + 4w + r (all < n since j < I) and column col
        auto rowof = [&](int t) { return (int64_t)((t < ntile) ? t : ntile - 1) * NB + 4 * w; };
        double cur[GRP][4], nxt[GRP][4];
#pragma unroll
        for (int g = 0; g < GRP; ++g) {
            const int64_t rr = rowof(g);
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[g][r] = U[(rr + r) * ldu + colc];
        }
        for (int t0 = 0; t0 < ntile; t0 += GRP) {
            // lane p < 16 polls value r = p & 3 of tile g = p >> 2 of the group;
            // the other lanes repeat those addresses
            const int p = l & 15;
            const int64_t prow = rowof(t0 + (p >> 2)) + (p & 3);
            const unsigned long long pv = ld_bits(stage + prow);
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int64_t rr = rowof(t0 + GRP + g);
#pragma unroll
                for (int r = 0; r < 4; ++r) nxt[g][r] = U[(rr + r) * ldu + colc];
            }
            const double zmine = settle(pv, stage + prow, ctl);
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const bool live = (t0 + g < ntile);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double zv = rdlane(zmine, g * 4 + r);
                    acc = fma(cur[g][r], live ? zv : 0.0, acc);
                }
            }
#pragma unroll
            for (int g = 0; g < GRP; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = nxt[g][r];
        }
    }
    // y_I = Dinv_I^T (b_I - far column sums)
    s_part[w][l] = acc;
    __syncthreads();
    if (tid < NB) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += s_part[q][tid];
        s_r[tid] = ((c0 + tid < n) ? b[c0 + tid] : 0.0) - s;
    }
    __syncthreads();
    double y = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) y = fma(dinv[k], s_r[dq * 4 + k], y);
    y += __shfl_xor(y, 1);
    y += __shfl_xor(y, 2);
    y += __shfl_xor(y, 4);
    y += __shfl_xor(y, 8);
    if (dq == 0) s_y[dcol] = y;
    __syncthreads();
    // chain: each wave finishes entries 4w..4w+3 of x_I = y_I - M'_I x_{I-1}
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (I > 0) {
        const int64_t rp = (int64_t)(I - 1) * NB + l;  // block I-1 is complete
        const double xp = settle(ld_bits(stage + rp), stage + rp, ctl);
#pragma unroll
        for (int r = 0; r < 4; ++r) part[r] = wave_sum(mrow[r] * xp);
    }
    if (l < 4) {
        const int e = 4 * w + l;
        const double p = (l == 0) ? part[0] : (l == 1) ? part[1] : (l == 2) ? part[2] : part[3];
        if (c0 + e < n) {
            const double xi = s_y[e] - p;
            st_bits(stage + c0 + e, (unsigned long long)__double_as_longlong(xi));
            x[c0 + e] = xi;
        }
    }
    retire(ctl, stage, n, nblk, &s_last);
}

// M_i = Dinv_i U_{i,i+1} (i < nblk-1) and M'_i = Dinv_i^T U_{i-1,i}^T (i > 0),
// 64x64 row-major each; entries that would touch columns >= n are zero.
__global__ __launch_bounds__(256) void k_make_m(const double *__restrict__ U, int64_t ldu, int64_t n,
                                                const double *__restrict__ Dinv, double *Mn,
                                                double *Mt)
{
    __shared__ double d[NB][NB + 1];
    __shared__ double t[NB][NB + 1];
    const int i = blockIdx.x, nblk = gridDim.x;
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += 256) d[e / NB][e % NB] = Dinv[(int64_t)i * NB * NB + e];
    // U_{i,i+1}: rows i*64+a, columns (i+1)*64+c
    for (int e = tid; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        const int64_t row = (int64_t)i * NB + a, cl = (int64_t)(i + 1) * NB + c;
        t[a][c] = (i + 1 < nblk && row < n && cl < n) ? U[row * ldu + cl] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        double s = 0.0;
        for (int k = 0; k < NB; ++k) s = fma(d[a][k], t[k][c], s);
        Mn[(int64_t)i * NB * NB + e] = s;
    }
    __syncthreads();
    // U_{i-1,i}: rows (i-1)*64+b, columns i*64+k
    for (int e = tid; e < NB * NB; e += 256) {
        const int bb = e / NB, k = e % NB;
        const int64_t row = (int64_t)(i - 1) * NB + bb, cl = (int64_t)i * NB + k;
        t[bb][k] = (i > 0 && cl < n) ? U[row * ldu + cl] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < NB * NB; e += 256) {
        const int a = e / NB, bb = e % NB;
        double s = 0.0;
        for (int k = 0; k < NB; ++k) s = fma(d[k][a], t[bb][k], s);
        Mt[(int64_t)i * NB * NB + e] = s;
    }
}

}  // namespace

int launch_make_m(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *M,
                  hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_make_m, dim3(nblk), dim3(256), 0, st, U, ldu, n, Dinv, M,
                       M + (int64_t)nblk * NB * NB);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_trsv_n(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *M,
                  const double *b, double *x, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_trsv_n, dim3(nblk), dim3(1024), 0, st, U, ldu, n, nblk, Dinv, M, b, x, ctl);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_trsv_t(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *M,
                  const double *b, double *x, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_trsv_t, dim3(nblk), dim3(1024), 0, st, U, ldu, n, nblk, Dinv,
                       M + (int64_t)nblk * NB * NB, b, x, ctl);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}
