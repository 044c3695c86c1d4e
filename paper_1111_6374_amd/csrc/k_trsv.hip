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
//   * the 64x64 diagonal solve is a product with Dinv_I = U_II^-1 held in
//     registers.  The last workgroup to retire restores the sentinels.
//
// Tile lane map (64x64 tile, 4 wave64s): wave w owns tile columns
// 16w..16w+15, lane l reads column 16w + (l & 15) of rows (l >> 4) + 4q,
// q = 0..15 -- four 128-byte row segments per load instruction.
#include "internal.h"

namespace {

__device__ __forceinline__ unsigned long long ld_bits(const double *p)
{
    return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_bits(double *p, unsigned long long v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Finish a poll started with ld_bits: spin (bounded) while the value is the
// sentinel.  An expired wait records an error and yields 0.
__device__ __forceinline__ double settle(unsigned long long v, const double *p, unsigned *err)
{
    unsigned it = 0;
    while (v == STAGE_SENTINEL) {
        if (++it > SPIN_LIMIT) {
            __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0.0;
        }
        __builtin_amdgcn_s_sleep(1);
        v = ld_bits(p);
    }
    return __longlong_as_double((long long)v);
}

// Chain position of this workgroup.  A counter left inconsistent by an
// earlier failure is reported (GSYEIG_ESPIN) and folded into range, so every
// index stays in bounds.
__device__ int take_ticket(PCtl *ctl, int nblk)
{
    unsigned t = atomicAdd(&ctl->ticket, 1u);
    if (t >= (unsigned)nblk) {
        __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t %= (unsigned)nblk;
    }
    return (int)t;
}

// Count this workgroup out; the last one restores the staging sentinels and
// resets the counters for the next launch.
__device__ void retire(PCtl *ctl, double *stage, int64_t nstage, int nblk, int *s_last)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned d = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        *s_last = (d == (unsigned)nblk - 1u);
    }
    __syncthreads();
    if (*s_last) {
        for (int64_t j = threadIdx.x; j < nstage; j += blockDim.x) st_bits(stage + j, STAGE_SENTINEL);
        if (threadIdx.x == 0) {
            __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ------------------------------------------------------------------ KI1
__global__ __launch_bounds__(256) void k_trsv_n(const double *__restrict__ U, int64_t ldu,
                                                int64_t n, int nblk,
                                                const double *__restrict__ Dinv,
                                                const double *b, double *x, PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_part[4][NB];
    __shared__ double s_r[NB];
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = nblk - 1 - take_ticket(ctl, nblk);
    __syncthreads();
    const int I = s_blk;
    const int64_t r0 = (int64_t)I * NB;
    const int c = 16 * w + (lane & 15);
    const int rg = lane >> 4;

    // Dinv row for the diagonal solve: thread t -> row t>>2, columns (t&3)*16..+15
    const int drow = tid >> 2, dq = tid & 3;
    double dinv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) dinv[k] = Dinv[(int64_t)I * NB * NB + drow * NB + dq * 16 + k];

    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;

    const double *Urow = U + (r0 + rg) * ldu;
    auto load_tile = [&](double *t, int j) {
        const int64_t col = (int64_t)j * NB + c;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const bool ok = (r0 + rg + 4 * q < n) && (col < n);
            t[q] = ok ? Urow[(int64_t)(4 * q) * ldu + col] : 0.0;
        }
    };
    double a[16];
    if (nblk - 1 > I) load_tile(a, nblk - 1);
    for (int j = nblk - 1; j > I; --j) {
        const int64_t col = (int64_t)j * NB + c;
        const bool colok = col < n;
        const unsigned long long v = colok ? ld_bits(stage + col) : 0ull;
        double an[16];
        if (j - 1 > I) load_tile(an, j - 1);
        const double xj = colok ? settle(v, stage + col, &ctl->err) : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = fma(a[q], xj, acc[q]);
        if (j - 1 > I) {
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = an[q];
        }
    }
    // row sums: reduce over the 16 lanes sharing a row, then over the 4 waves
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
        const int64_t row = r0 + tid;
        const double bi = (row < n) ? b[row] : 0.0;
        s_r[tid] = bi - (s_part[0][tid] + s_part[1][tid] + s_part[2][tid] + s_part[3][tid]);
    }
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) v = fma(dinv[k], s_r[dq * 16 + k], v);
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    if (dq == 0 && r0 + drow < n) {
        st_bits(stage + r0 + drow, (unsigned long long)__double_as_longlong(v));
        x[r0 + drow] = v;
    }
    retire(ctl, stage, n, nblk, &s_last);
}

// ------------------------------------------------------------------ KI3
__global__ __launch_bounds__(256) void k_trsv_t(const double *__restrict__ U, int64_t ldu,
                                                int64_t n, int nblk,
                                                const double *__restrict__ Dinv,
                                                const double *b, double *x, PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_r[NB];
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = take_ticket(ctl, nblk);
    __syncthreads();
    const int I = s_blk;
    const int64_t c0 = (int64_t)I * NB;
    const int c = 16 * w + (lane & 15);
    const int rg = lane >> 4;
    const int64_t col = c0 + c;
    const bool colok = col < n;

    // Dinv^T product: thread t -> output column t>>2, rows (t&3)*16..+15
    const int dcol = tid >> 2, dq = tid & 3;
    double dinv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) dinv[k] = Dinv[(int64_t)I * NB * NB + (dq * 16 + k) * NB + dcol];

    // rows of U above block I are complete 64-row blocks (J < I), so only the
    // column can be out of range.
    auto load_tile = [&](double *t, int j) {
        const double *Ut = U + ((int64_t)j * NB + rg) * ldu + col;
#pragma unroll
        for (int q = 0; q < 16; ++q) t[q] = colok ? Ut[(int64_t)(4 * q) * ldu] : 0.0;
    };
    double acc = 0.0;
    double a[16];
    if (I > 0) load_tile(a, 0);
    for (int j = 0; j < I; ++j) {
        const double *zs = stage + (int64_t)j * NB + rg;
        unsigned long long v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = ld_bits(zs + 4 * q);
        double an[16];
        if (j + 1 < I) load_tile(an, j + 1);
#pragma unroll
        for (int q = 0; q < 16; ++q) acc = fma(a[q], settle(v[q], zs + 4 * q, &ctl->err), acc);
        if (j + 1 < I) {
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = an[q];
        }
    }
    // column sums: reduce over the 4 row groups of the wave
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (rg == 0) s_r[c] = (colok ? b[col] : 0.0) - acc;
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) v = fma(dinv[k], s_r[dq * 16 + k], v);
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    if (dq == 0 && c0 + dcol < n) {
        st_bits(stage + c0 + dcol, (unsigned long long)__double_as_longlong(v));
        x[c0 + dcol] = v;
    }
    retire(ctl, stage, n, nblk, &s_last);
}

}  // namespace

int launch_trsv_n(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *b,
                  double *x, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_trsv_n, dim3(nblk), dim3(256), 0, st, U, ldu, n, nblk, Dinv, b, x, ctl);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_trsv_t(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *b,
                  double *x, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL(k_trsv_t, dim3(nblk), dim3(256), 0, st, U, ldu, n, nblk, Dinv, b, x, ctl);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}
