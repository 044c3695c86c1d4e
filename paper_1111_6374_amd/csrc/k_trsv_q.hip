// k_trsv_q.hip -- KI1 / KI3 (Section 2.3, Table 1) on U = D (I + W) as a
// work queue of independent items instead of one workgroup per tile.
//
// The per-tile sweeps (k_trsv_w.hip) give each 64-row tile one workgroup
// that streams its whole row panel of W as the solved values arrive.  The
// chain is then paced by fair-share bandwidth: when super-block T has been
// solved, every workgroup above it wants its 64 x 512 block of column block
// T at once, and the workgroup on the critical path gets 1/256 of HBM.
// Here the panel products are items of their own, taken from one queue in
// the order the chain needs their results:
//
//   KI1 (x = U^-1 b, bottom-up), for each super-block S from the last:
//     far items (i, T), T >= S + 2, for the tiles i of S:
//         p[i][T] = W_{i,T} x_T                       (64 sums, published)
//     link items (i):   x_i = Uinv_ii-row . b_S - sum_T p[i][T] - W_{i,S+1} x_{S+1}
//
//   KI3 (x = U^-T b, top-down), for each super-block S from the first:
//     far items (j, T), T <= S - 2, for the tiles j of S:
//         q[j][T] = (W_{T,j})^T y_T                   (64 sums, published)
//     link items (j):   y_j = b_j - sum_T q[j][T] - (W_{S-1,j})^T y_{S-1}
//     finish items (j') of S - 1:  x_S' = Uinv_{S-1}^T y_{S-1}  (off the chain)
//
// Every item waits only on results of items earlier in the queue, and an
// item is taken only by a running workgroup, so the queue drains whatever
// the residency.  A link item loads its link block and forms its diagonal
// part before it waits; its critical path is the poll of the neighbour
// super-block's values, one 32-term product per lane and a reduction.  The
// far partials sit in sentinel-initialised buffers (nblk x nsb x 64 each);
// the link item that consumes a partial restores the sentinel, the last
// workgroup restores the staging vector and the ticket, so launches need no
// host memset.  Summation orders are fixed (bitwise reproducible).  W may
// be stored FP64 or FP32; Uinv blocks, vectors and arithmetic are FP64.
#include <algorithm>
#include <vector>

#include "chain.h"

#define TPS 8          // tiles per super-block
#define SBR (TPS * NB) // super-block rows

namespace {

using namespace chain;

// queue item: x = tile, y = column (KI1) / row (KI3) super-block of a far
// item, or LINK / FINISH
constexpr int LINK = -1, FINISH = -2;

__device__ __forceinline__ int next_item(PCtl *ctl, int *s_q)
{
    __syncthreads();  // every wave is done with the previous item's LDS
    if (threadIdx.x == 0) *s_q = (int)atomicAdd(&ctl->ticket, 1u);
    __syncthreads();
    return *s_q;
}

// Inline bounded wait on K values per lane (no call, so nothing live is
// spilled around it): v[c] holds a first poll of addr(c) for the lanes and
// slots in `live`; slots still holding the sentinel are polled again, the
// whole wave together, until none is left.  After `lim` repolls the wait
// expires: the error is recorded and the missing values read 0.0.
template <int K, typename A>
__device__ __forceinline__ void wait_all(unsigned long long (&v)[K], unsigned live, A addr, PCtl *ctl, unsigned lim)
{
    unsigned it = 0;
    for (;;) {
        bool pend = false;
#pragma unroll
        for (int c = 0; c < K; ++c) pend |= ((live >> c) & 1u) && v[c] == STAGE_SENTINEL;
        if (!__any(pend)) break;
        if (++it > lim) {
            __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (v[c] == STAGE_SENTINEL) v[c] = 0ull;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (((live >> c) & 1u) && v[c] == STAGE_SENTINEL) v[c] = ld_bits(addr(c));
    }
}

// The context's bound on repolls of one wait, read once per workgroup at
// the start (0 selects SPIN_LIMIT).
__device__ __forceinline__ unsigned spin_limit_of(PCtl *ctl)
{
    const unsigned s = __hip_atomic_load(&ctl->spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return s ? s : SPIN_LIMIT;
}

// Wave 0 polls the 512 staged values of a super-block (entries >= n read
// as 0) into s_v; every wave may read them after the barrier.
__device__ __forceinline__ void poll_block(const double *stage, int64_t base, int64_t n, PCtl *ctl, unsigned lim,
                                           double *s_v)
{
    const int tid = threadIdx.x, l = tid & 63;
    if (tid < 64) {
        const double *p0 = stage + base + l;
        const int cols = (int)((n - base < SBR) ? n - base : SBR);  // entries of the block inside n
        unsigned live = 0;
        unsigned long long v[TPS];
#pragma unroll
        for (int g = 0; g < TPS; ++g) {
            const bool ok = g * NB + l < cols;
            live |= (ok ? 1u : 0u) << g;
            v[g] = ok ? ld_bits(p0 + g * NB) : 0ull;
        }
        wait_all<TPS>(v, live, [&](int g) { return p0 + g * NB; }, ctl, lim);
#pragma unroll
        for (int g = 0; g < TPS; ++g) s_v[g * NB + l] = __longlong_as_double((long long)v[g]);
    }
    __syncthreads();
}

// Sum of the far partials of one row (or column) position: the entries
// base[T * NB] for T = T0 + lane_t + 16 c (< T1), taken by this lane and
// restored to the sentinel; the caller folds the lanes.
__device__ __forceinline__ double take_partials(double *base, int T0, int T1, int lane_t, int stride_t, PCtl *ctl,
                                                unsigned lim)
{
    double f = 0.0;
    for (int Ta = T0; Ta < T1; Ta += 8 * stride_t) {
        unsigned live = 0;
        unsigned long long v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int Tq = Ta + lane_t + stride_t * c;
            const bool ok = Tq < T1;
            live |= (ok ? 1u : 0u) << c;
            v[c] = ok ? ld_bits(base + (int64_t)Tq * NB) : 0ull;
        }
        wait_all<8>(v, live, [&](int c) { return base + (int64_t)(Ta + lane_t + stride_t * c) * NB; }, ctl, lim);
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if ((live >> c) & 1u) {
                f += __longlong_as_double((long long)v[c]);
                st_bits(base + (int64_t)(Ta + lane_t + stride_t * c) * NB, STAGE_SENTINEL);
            }
    }
    return f;
}

// w[g][r] = W[r0 + r][c0 + g * 64 + l] (0 for columns >= n) from four
// wave-uniform row pointers and one lane offset.  Rows are below the last
// super-block, so every row exists; a read past column n (masked) stays
// inside the next row of W, which also exists (W holds n rows of ldw >= n
// entries and c0 + 511 < n + 512 <= 2 ldw for the rows read here).
template <typename T>
__device__ __forceinline__ void load_rows4(const T *__restrict__ W, int64_t ldw, int64_t r0, int64_t c0, int64_t n, int l,
                                           double (&w)[TPS][4])
{
    const T *row[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) row[r] = W + (r0 + r) * ldw + c0;
    const int cols = (int)((n - c0 < SBR) ? n - c0 : SBR);  // columns of the block inside n
#pragma unroll
    for (int g = 0; g < TPS; ++g) {
        const int o = g * NB + l;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double v = (double)row[r][o];
            w[g][r] = (o < cols) ? v : 0.0;
        }
    }
}

// w[k] = W[rb + k][c] for k < 32: one wave-uniform pointer stepped by ldw
template <typename T>
__device__ __forceinline__ void load_cols32(const T *__restrict__ W, int64_t ldw, int64_t rb, int64_t c, double (&w)[32])
{
    const T *p = W + rb * ldw;
    const int o = (int)c;
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        w[k] = (double)p[o];
        p += ldw;
    }
}

// ------------------------------------------------------------------ KI1
template <typename T>
__global__ __launch_bounds__(1024) void k_trsvq_n(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk, int nsb,
                                                  const double *__restrict__ Uinv, const double *b, double *x,
                                                  PCtl *ctl, const int2 *__restrict__ items, int nitems, double *P)
{
    __shared__ int s_q, s_last;
    __shared__ double s_v[SBR];
    double *stage = ctl_stage(ctl);
    const unsigned lim = spin_limit_of(ctl);
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row pointers stay scalar
    for (;;) {
        const int qn = next_item(ctl, &s_q);
        if (qn >= nitems) break;
        const int2 it = items[qn];
        const int i = it.x, S = i / TPS, loc = i % TPS;
        const int64_t r0 = (int64_t)i * NB + 4 * w;  // this wave's first row
        if (it.y >= 0) {
            // far item: rows of tile i (all < n: S is not the last super-block)
            // times column block T, as soon as x_T is published
            const int64_t c0 = (int64_t)it.y * SBR;
            double wv[TPS][4];
            load_rows4(W, ldw, r0, c0, n, l, wv);
            poll_block(stage, c0, n, ctl, lim, s_v);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int g = 0; g < TPS; ++g) {
                const double xv = s_v[g * NB + l];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = fma(wv[g][r], xv, acc[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = wave_sum(acc[r]);
            if (l < 4) {
                const double v = (l == 0) ? acc[0] : (l == 1) ? acc[1] : (l == 2) ? acc[2] : acc[3];
                st_bits(P + ((int64_t)i * nsb + it.y) * NB + 4 * w + l, (unsigned long long)__double_as_longlong(v));
            }
            continue;
        }
        // link item of tile i
        const int64_t s0 = (int64_t)S * SBR;
        const bool has_next = S + 1 < nsb;
        const int rowl = loc * NB + 4 * w;  // local row (in S) of this wave's first row
        // diagonal part: Uinv_SS[rowl + r][k] b_S[k], k >= the tile's first row
        double y[4] = {0.0, 0.0, 0.0, 0.0};
        {
            const double *Ub = Uinv + (int64_t)S * SBR * SBR + (int64_t)rowl * SBR;
#pragma unroll
            for (int c = 0; c < TPS; ++c) {
                if (c < loc) continue;
                const int64_t kk = s0 + (int64_t)c * NB + l;
                const double bv = (kk < n) ? b[kk] : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fma(Ub[r * SBR + c * NB + l], bv, y[r]);
            }
        }
        // far partials: lane l takes rows r0 + (l & 3) of super-blocks
        // S + 2 + (l >> 2) + 16 k; a fixed shuffle tree sums them per row
        double f = 0.0;
        {
            const int64_t row = r0 + (l & 3);
            if (row < n)
                f = take_partials(P + (int64_t)i * nsb * NB + 4 * w + (l & 3), S + 2, nsb, l >> 2, 16, ctl, lim);
            f += __shfl_xor(f, 4);
            f += __shfl_xor(f, 8);
            f += __shfl_xor(f, 16);
            f += __shfl_xor(f, 32);
        }
        // the link block's loads after the other parts' (register budget)
        __syncthreads();
        double lk[TPS][4];
        if (has_next) load_rows4(W, ldw, r0, s0 + SBR, n, l, lk);
        if (has_next) {
            poll_block(stage, s0 + SBR, n, ctl, lim, s_v);
#pragma unroll
            for (int g = 0; g < TPS; ++g) {
                const double xv = s_v[g * NB + l];
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fma(-lk[g][r], xv, y[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) y[r] = wave_sum(y[r]);
        if (l < 4) {
            const int64_t row = r0 + l;
            const double xi = ((l == 0) ? y[0] : (l == 1) ? y[1] : (l == 2) ? y[2] : y[3]) - f;
            if (row < n) {
                st_bits(stage + row, (unsigned long long)__double_as_longlong(xi));
                x[row] = xi;
            }
        }
    }
    retire(ctl, stage, n, gridDim.x, &s_last);
}

// ------------------------------------------------------------------ KI3
// KI3's right-hand side: b, or (Pr != nullptr) the SYMV tile partials
// summed in the order of k_symv_reduce (bitwise the same b).
struct QRowSums {
    const double *Pr, *Pc;
    int maxch, ch;
};

template <typename T>
__global__ __launch_bounds__(1024) void k_trsvq_t(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk, int nsb,
                                                  const double *__restrict__ Uinv, const double *b, double *x,
                                                  PCtl *ctl, QRowSums rs, const int2 *__restrict__ items, int nitems,
                                                  double *Q)
{
    __shared__ int s_q, s_last;
    __shared__ double s_v[SBR];
    __shared__ double s_part[16][NB];
    __shared__ double s_rs[4][NB];
    double *stage = ctl_stage(ctl);  // holds y
    const unsigned lim = spin_limit_of(ctl);
    const int tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: row pointers stay scalar
    for (;;) {
        const int qn = next_item(ctl, &s_q);
        if (qn >= nitems) break;
        const int2 it = items[qn];
        const int j = it.x, S = j / TPS;
        const int64_t col = (int64_t)j * NB + l;
        const bool colok = col < n;
        if (it.y >= 0) {
            // far item: rows of super-block T (all < n) times this tile's columns
            double wv[32];
            load_cols32(W, ldw, (int64_t)it.y * SBR + 32 * w, col, wv);
            poll_block(stage, (int64_t)it.y * SBR, n, ctl, lim, s_v);
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 32; ++k) acc = fma(wv[k], s_v[32 * w + k], acc);
            s_part[w][l] = acc;
            __syncthreads();
            if (w == 0 && colok) {
                double sm = 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) sm += s_part[q][l];
                st_bits(Q + ((int64_t)j * nsb + it.y) * NB + l, (unsigned long long)__double_as_longlong(sm));
            }
            continue;
        }
        if (it.y == FINISH) {
            // x of tile j from the complete y_S: x_a = sum_{k <= a} Uinv_SS[k][a] y_k
            const int64_t s0 = (int64_t)S * SBR;
            const int a = (j % TPS) * NB + l;  // local column
            // off the chain: poll first, then stream the column of Uinv
            poll_block(stage, s0, n, ctl, lim, s_v);
            const double *up = Uinv + (int64_t)S * SBR * SBR + (int64_t)(32 * w) * SBR + a;
            double acc = 0.0;
#pragma unroll 8
            for (int k = 0; k < 32; ++k) acc = fma(up[k * SBR], (32 * w + k <= a) ? s_v[32 * w + k] : 0.0, acc);
            s_part[w][l] = acc;
            __syncthreads();
            if (w == 0 && colok) {
                double sm = 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) sm += s_part[q][l];
                x[col] = sm;
            }
            continue;
        }
        // link item of tile j
        const bool has_prev = S > 0;
        if (rs.Pr && w < 4) {
            const int K = j, q = w;
            const int nch = (nblk - K + rs.ch - 1) / rs.ch;
            double sm = 0.0;
#pragma unroll 8
            for (int c = q; c < nch; c += 4) sm += rs.Pr[((int64_t)K * rs.maxch + c) * NB + l];
            const double *pc = rs.Pc + (int64_t)K * nblk * NB + l;
            int I = q;
#pragma unroll 4
            for (; I + 12 < K; I += 16) {
                const double a0 = pc[(int64_t)I * NB], a1 = pc[(int64_t)(I + 4) * NB];
                const double a2 = pc[(int64_t)(I + 8) * NB], a3 = pc[(int64_t)(I + 12) * NB];
                sm += (a0 + a1) + (a2 + a3);
            }
#pragma unroll 4
            for (; I < K; I += 4) sm += pc[(int64_t)I * NB];
            s_rs[q][l] = sm;
        }
        // far partials: wave w sums the super-blocks T = w, w + 16, ... < S - 1
        double f = 0.0;
        if (colok) f = take_partials(Q + (int64_t)j * nsb * NB + l, 0, S - 1, w, 16, ctl, lim);
        // the link block's loads after the other parts' (register budget)
        __syncthreads();
        double lk[32];
        if (has_prev) load_cols32(W, ldw, (int64_t)(S - 1) * SBR + 32 * w, col, lk);
        double acc = 0.0;
        if (has_prev) {
            poll_block(stage, (int64_t)(S - 1) * SBR, n, ctl, lim, s_v);
#pragma unroll
            for (int k = 0; k < 32; ++k) acc = fma(lk[k], s_v[32 * w + k], acc);
        }
        s_part[w][l] = f + acc;
        __syncthreads();
        if (w == 0 && colok) {
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) sm += s_part[q][l];
            const double be = rs.Pr ? (s_rs[0][l] + s_rs[1][l]) + (s_rs[2][l] + s_rs[3][l]) : b[col];
            st_bits(stage + col, (unsigned long long)__double_as_longlong(be - sm));
        }
    }
    retire(ctl, stage, n, gridDim.x, &s_last);
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

// resident 1024-thread workgroups of a kernel on the current device
template <typename K>
int resident_blocks(K kern)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, 1024, 0) != hipSuccess ||
        per_cu < 1)
        return 256;
    return per_cu * cus;
}

}  // namespace

// The two queues for n (host-built, cached per n in the context) and the
// sentinel-filled partial buffers.
int trsvq_prepare(gsyeig_ctx *ctx, int64_t n, TrsvQ *q)
{
    const int nblk = (int)cdiv(n, NB), nsb = (int)cdiv(n, SBR);
    const size_t pbytes = sizeof(double) * (size_t)nblk * nsb * NB;
    int rc;
    if (ctx->trsvq_n != n) {
        std::vector<int2> qn, qt;
        for (int S = nsb - 1; S >= 0; --S) {
            const int i0 = S * TPS, i1 = std::min(nblk, i0 + TPS);
            for (int T = nsb - 1; T >= S + 2; --T)
                for (int i = i0; i < i1; ++i) qn.push_back(make_int2(i, T));
            for (int i = i0; i < i1; ++i) qn.push_back(make_int2(i, LINK));
        }
        for (int S = 0; S < nsb; ++S) {
            const int j0 = S * TPS, j1 = std::min(nblk, j0 + TPS);
            for (int T = 0; T <= S - 2; ++T)
                for (int j = j0; j < j1; ++j) qt.push_back(make_int2(j, T));
            for (int j = j0; j < j1; ++j) qt.push_back(make_int2(j, LINK));
            if (S >= 1)
                for (int j = (S - 1) * TPS; j < S * TPS; ++j) qt.push_back(make_int2(j, FINISH));
        }
        for (int j = (nsb - 1) * TPS; j < nblk; ++j) qt.push_back(make_int2(j, FINISH));
        const size_t ib = ((qn.size() + qt.size()) * sizeof(int2) + 255) & ~(size_t)255;
        void *p;
        ctx->trsvq_n = -1;
        if ((rc = ws_get(ctx, WS_TRSVQ, ib + 2 * pbytes, &p))) return rc;
        char *base = (char *)p;
        HIP_TRY(hipMemcpyAsync(base, qn.data(), qn.size() * sizeof(int2), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(base + qn.size() * sizeof(int2), qt.data(), qt.size() * sizeof(int2),
                               hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemsetAsync(base + ib, 0xFF, 2 * pbytes, ctx->stream));  // the sentinel: all ones
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->trsvq_n = n;
        ctx->trsvq_nitems_n = (int)qn.size();
        ctx->trsvq_nitems_t = (int)qt.size();
        ctx->trsvq_pbytes = ib;
    }
    char *base = (char *)ctx->ws[WS_TRSVQ];
    q->items_n = (const int2 *)base;
    q->nitems_n = ctx->trsvq_nitems_n;
    q->items_t = (const int2 *)base + ctx->trsvq_nitems_n;
    q->nitems_t = ctx->trsvq_nitems_t;
    q->P = (double *)(base + ctx->trsvq_pbytes);
    q->Q = (double *)(base + ctx->trsvq_pbytes + pbytes);
    q->nsb = nsb;
    return 0;
}

template <typename T>
static int trsvq_n_t(const T *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                     const TrsvQ &q, hipStream_t st)
{
    static int grid = 0;
    if (!grid) grid = resident_blocks(k_trsvq_n<T>);
    const int nblk = (int)cdiv(n, NB);
    const int g = std::min(grid, q.nitems_n);
    hipLaunchKernelGGL((k_trsvq_n<T>), dim3(g), dim3(1024), 0, st, W, ldw, n, nblk, q.nsb, sbw, b, x, ctl, q.items_n,
                       q.nitems_n, q.P);
    return ok();
}

template <typename T>
static int trsvq_t_t(const T *W, int64_t ldw, int64_t n, const double *sbw, const double *b, const double *Pr,
                     const double *Pc, int maxch, int ch, double *x, PCtl *ctl, const TrsvQ &q, hipStream_t st)
{
    static int grid = 0;
    if (!grid) grid = resident_blocks(k_trsvq_t<T>);
    const int nblk = (int)cdiv(n, NB);
    const int g = std::min(grid, q.nitems_t);
    hipLaunchKernelGGL((k_trsvq_t<T>), dim3(g), dim3(1024), 0, st, W, ldw, n, nblk, q.nsb, sbw, b, x, ctl,
                       QRowSums{Pr, Pc, maxch, ch}, q.items_t, q.nitems_t, q.Q);
    return ok();
}

int launch_trsvq_n(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                   const TrsvQ &q, hipStream_t st)
{
    return trsvq_n_t<double>(W, ldw, n, sbw, b, x, ctl, q, st);
}

int launch_trsvq_n_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                       PCtl *ctl, const TrsvQ &q, hipStream_t st)
{
    return trsvq_n_t<float>(W, ldw, n, sbw, b, x, ctl, q, st);
}

int launch_trsvq_t(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, const double *Pr,
                   const double *Pc, int maxch, int ch, double *x, PCtl *ctl, const TrsvQ &q, hipStream_t st)
{
    return trsvq_t_t<double>(W, ldw, n, sbw, b, Pr, Pc, maxch, ch, x, ctl, q, st);
}

int launch_trsvq_t_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, const double *Pr,
                       const double *Pc, int maxch, int ch, double *x, PCtl *ctl, const TrsvQ &q, hipStream_t st)
{
    return trsvq_t_t<float>(W, ldw, n, sbw, b, Pr, Pc, maxch, ch, x, ctl, q, st);
}
