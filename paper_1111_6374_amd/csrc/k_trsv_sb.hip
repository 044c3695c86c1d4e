// k_trsv_sb.hip -- KI1 / KI3 (Section 2.3, Table 1) with super-block chain
// links: the triangular factor is cut into SB x SB diagonal super-blocks
// (SB = TPS * 64) that are applied through their explicit inverses, so the
// dependency chain of a sweep has n/SB links instead of n/64.
//
// KI1, x = U^-1 b, super-block S (rows), from the bottom:
//     x_S = Y_S - N_S x_{S+1},
//     Y_S = Uinv_SS (b_S - sum_{T >= S+2} U_ST x_T),   N_S = Uinv_SS U_{S,S+1}
// KI3, x = U^-T b, from the top:
//     x_S = Y'_S - N'_S x_{S-1},
//     Y'_S = Uinv_SS^T (b_S - sum_{T <= S-2} U_TS^T x_T),  N'_S = Uinv_SS^T U_{S-1,S}^T
// Y_S needs only x two links back, so it is formed off the critical path;
// each link then costs one publish/poll latency plus a product with N_S
// rows prefetched into registers before the awaited values exist.
//
// One 1024-thread workgroup owns each 64-row tile i (tile loc of super-block
// S); waves own 4 rows, lanes own columns.  Partial right-hand sides r'_S are
// exchanged between the tiles of a super-block through a second staging
// vector.  Tickets, staging, bounded waits and the reset are those of the
// 64-row chained kernels (chain.h).
#include <algorithm>

#include "chain.h"

#define TPS 8          // tiles per super-block
#define SBR (TPS * NB) // super-block rows
#define GRP2 2

namespace {

using namespace chain;

// ------------------------------------------------------------------ KI1
template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_sb_n(const T *__restrict__ U, int64_t ldu,
                                                    int64_t n, int nblk,
                                                    const double *__restrict__ Uinv,
                                                    const double *__restrict__ N,
                                                    const double *b, double *x, double *rstage,
                                                    PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = nblk - 1 - take_ticket(ctl, nblk);
    __syncthreads();
    const int i = s_blk;
    const int S = i / TPS, loc = i % TPS;
    const int nsb = (nblk + TPS - 1) / TPS;
    const int64_t r0 = (int64_t)i * NB;
    const int64_t s0 = (int64_t)S * SBR;
    const bool has_next = S < nsb - 1;
    const int rowl = loc * NB + 4 * w;  // local row (in super-block S) of this wave's first row

    // far tiles: j = nblk-1 down to (S+2)*TPS
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int jlo = (S + 2) * TPS;
    const int ntile = nblk - jlo;
    if (ntile > 0) {
        const T *Ur = U + (r0 + 4 * w) * ldu;  // rows of a non-last tile exist
        const int64_t cmax = n - 1;
        auto colof = [&](int t) {
            const int j = (t < ntile) ? nblk - 1 - t : jlo;
            const int64_t cc = (int64_t)j * NB + l;
            return cc < cmax ? cc : cmax;
        };
        double cur[GRP2][4], nxt[GRP2][4];
#pragma unroll
        for (int g = 0; g < GRP2; ++g) {
            const int64_t cc = colof(g);
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[g][r] = (double)Ur[(int64_t)r * ldu + cc];
        }
        for (int t0 = 0; t0 < ntile; t0 += GRP2) {
            unsigned long long v[GRP2];
#pragma unroll
            for (int g = 0; g < GRP2; ++g) v[g] = ld_bits(stage + colof(t0 + g));
#pragma unroll
            for (int g = 0; g < GRP2; ++g) {
                const int64_t cc = colof(t0 + GRP2 + g);
#pragma unroll
                for (int r = 0; r < 4; ++r) nxt[g][r] = (double)Ur[(int64_t)r * ldu + cc];
            }
#pragma unroll
            for (int g = 0; g < GRP2; ++g) {
                const int t = t0 + g;
                const int64_t col = (int64_t)(nblk - 1 - t) * NB + l;
                const bool live = (t < ntile) && (col < n);
                const double xv = settle(v[g], stage + colof(t), &ctl->err);
                const double xj = live ? xv : 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] = fma(cur[g][r], xj, acc[r]);
            }
#pragma unroll
            for (int g = 0; g < GRP2; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = nxt[g][r];
        }
    }
    // r'_i = b_i - far sums, published for the other tiles of S
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = wave_sum(acc[r]);
    if (l < 4) {
        const int64_t row = r0 + 4 * w + l;
        const double a = (l == 0) ? acc[0] : (l == 1) ? acc[1] : (l == 2) ? acc[2] : acc[3];
        if (row < n) st_bits(rstage + row, (unsigned long long)__double_as_longlong(b[row] - a));
    }
    // N_S rows rowl..rowl+3, columns c*64 + l: independent of the chain, loaded
    // now so they are in registers a link before x_{S+1} can arrive
    double nr[TPS][4];
#pragma unroll
    for (int c = 0; c < TPS; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            nr[c][r] = has_next ? N[(int64_t)S * SBR * SBR + (int64_t)(rowl + r) * SBR + c * NB + l] : 0.0;
    // Y rows: Uinv_SS[rowl + r][k] r'_S[k], k >= rowl (upper triangle), k = c*64 + l.
    // All r' polls are issued together and settled before any product, so
    // the exchange costs one round trip and the Uinv loads pipeline.
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    {
        unsigned long long rb[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const int64_t kk = s0 + (int64_t)c * NB + l;
            rb[c] = ld_bits(rstage + (kk < n ? kk : n - 1));
        }
        double rv[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const int64_t kk = s0 + (int64_t)c * NB + l;
            // entries past n stay 0 (U^-1 rows beyond n are zero)
            rv[c] = (c >= loc && kk < n) ? settle(rb[c], rstage + kk, &ctl->err) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            if (c < loc) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                y[r] = fma(Uinv[(int64_t)S * SBR * SBR + (int64_t)(rowl + r) * SBR + c * NB + l], rv[c], y[r]);
        }
    }
    // the link: x_{S+1} arrives; y - N_S x_{S+1} is folded into one wave sum
    if (has_next) {
        unsigned long long v[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            int64_t kk = s0 + SBR + (int64_t)c * NB + l;
            kk = kk < n ? kk : n - 1;
            v[c] = ld_bits(stage + kk);
        }
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const int64_t k0 = s0 + SBR + (int64_t)c * NB + l;
            const int64_t kk = k0 < n ? k0 : n - 1;
            const double xv = settle(v[c], stage + kk, &ctl->err);
            const double xn = (k0 < n) ? xv : 0.0;
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = fma(-nr[c][r], xn, y[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = wave_sum(y[r]);
    if (l < 4) {
        const int64_t row = r0 + 4 * w + l;
        const double xi = (l == 0) ? y[0] : (l == 1) ? y[1] : (l == 2) ? y[2] : y[3];
        if (row < n) {
            st_bits(stage + row, (unsigned long long)__double_as_longlong(xi));
            x[row] = xi;
        }
    }
    retire(ctl, stage, n, nblk, &s_last, rstage);
}

// ------------------------------------------------------------------ KI3
template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_sb_t(const T *__restrict__ U, int64_t ldu,
                                                    int64_t n, int nblk,
                                                    const double *__restrict__ UinvT,
                                                    const double *__restrict__ Nt,
                                                    const double *b, double *x, double *rstage,
                                                    PCtl *ctl)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_part[16][NB];
    double *stage = ctl_stage(ctl);
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid == 0) s_blk = take_ticket(ctl, nblk);
    __syncthreads();
    const int i = s_blk;
    const int S = i / TPS, loc = i % TPS;
    const int64_t c0 = (int64_t)i * NB;
    const int64_t s0 = (int64_t)S * SBR;
    const int64_t col = c0 + l;
    const bool colok = col < n;
    const int64_t colc = colok ? col : n - 1;
    const bool has_prev = S > 0;
    const int al = loc * NB + 4 * w;  // local index (in S) of this wave's first output

    // far tiles: rows of super-blocks T <= S-2, i.e. tiles j < (S-1)*TPS
    double acc = 0.0;
    const int ntile = (S - 1) * TPS;
    if (ntile > 0) {
        auto rowof = [&](int t) { return (int64_t)((t < ntile) ? t : ntile - 1) * NB + 4 * w; };
        double cur[GRP2][4], nxt[GRP2][4];
#pragma unroll
        for (int g = 0; g < GRP2; ++g) {
            const int64_t rr = rowof(g);
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[g][r] = (double)U[(rr + r) * ldu + colc];
        }
        for (int t0 = 0; t0 < ntile; t0 += GRP2) {
            const int p = l & 7;  // lane p < 8 polls value p&3 of tile p>>2 of the group
            const int64_t prow = rowof(t0 + (p >> 2)) + (p & 3);
            const unsigned long long pv = ld_bits(stage + prow);
#pragma unroll
            for (int g = 0; g < GRP2; ++g) {
                const int64_t rr = rowof(t0 + GRP2 + g);
#pragma unroll
                for (int r = 0; r < 4; ++r) nxt[g][r] = (double)U[(rr + r) * ldu + colc];
            }
            const double zmine = settle(pv, stage + prow, &ctl->err);
#pragma unroll
            for (int g = 0; g < GRP2; ++g) {
                const bool live = (t0 + g < ntile);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double zv = rdlane(zmine, g * 4 + r);
                    acc = fma(cur[g][r], live ? zv : 0.0, acc);
                }
            }
#pragma unroll
            for (int g = 0; g < GRP2; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = nxt[g][r];
        }
    }
    // r'_i = b_i - far column sums, published for the other tiles of S
    s_part[w][l] = acc;
    __syncthreads();
    if (tid < NB && c0 + tid < n) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += s_part[q][tid];
        st_bits(rstage + c0 + tid, (unsigned long long)__double_as_longlong(b[c0 + tid] - s));
    }
    // N'_S rows al..al+3 (independent of the chain; needed a link later)
    double nr[TPS][4];
#pragma unroll
    for (int c = 0; c < TPS; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            nr[c][r] = has_prev ? Nt[(int64_t)S * SBR * SBR + (int64_t)(al + r) * SBR + c * NB + l] : 0.0;
    // Y' entries: Uinv_SS^T[al + r][k] r'_S[k], k <= al + r, k = c*64 + l;
    // all r' polls in flight together, then the products
    double y[4] = {0.0, 0.0, 0.0, 0.0};
    {
        unsigned long long rb[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const int64_t kk = s0 + (int64_t)c * NB + l;
            rb[c] = ld_bits(rstage + (kk < n ? kk : n - 1));
        }
        double rv[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const int64_t kk = s0 + (int64_t)c * NB + l;
            rv[c] = (c <= loc && kk < n) ? settle(rb[c], rstage + kk, &ctl->err) : 0.0;
        }
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            if (c > loc) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                y[r] = fma(UinvT[(int64_t)S * SBR * SBR + (int64_t)(al + r) * SBR + c * NB + l], rv[c], y[r]);
        }
    }
    // the link: x_{S-1} (a complete super-block) arrives
    if (has_prev) {
        unsigned long long v[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) v[c] = ld_bits(stage + s0 - SBR + (int64_t)c * NB + l);
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const double xp = settle(v[c], stage + s0 - SBR + (int64_t)c * NB + l, &ctl->err);
#pragma unroll
            for (int r = 0; r < 4; ++r) y[r] = fma(-nr[c][r], xp, y[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) y[r] = wave_sum(y[r]);
    if (l < 4) {
        const int64_t e = c0 + 4 * w + l;
        const double xi = (l == 0) ? y[0] : (l == 1) ? y[1] : (l == 2) ? y[2] : y[3];
        if (e < n) {
            st_bits(stage + e, (unsigned long long)__double_as_longlong(xi));
            x[e] = xi;
        }
    }
    retire(ctl, stage, n, nblk, &s_last, rstage);
}

// Uinv (row-major) from UinvT (row-major) = transpose, one SBR x SBR block
// per blockIdx.y, 64x64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_sb(const double *__restrict__ src, double *dst)
{
    __shared__ double t[NB][NB + 1];
    const int S = blockIdx.y;
    const int tr = blockIdx.x / TPS, tc = blockIdx.x % TPS;
    const double *s = src + (int64_t)S * SBR * SBR;
    double *d = dst + (int64_t)S * SBR * SBR;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        t[a][c] = s[(int64_t)(tr * NB + a) * SBR + tc * NB + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        d[(int64_t)(tc * NB + a) * SBR + tr * NB + c] = t[c][a];
    }
}

// columns of an SBR x SBR column-major block set to the identity (r x r part)
__global__ void k_identity_sb(double *Y, int r)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)SBR * SBR) return;
    const int i = (int)(e % SBR), j = (int)(e / SBR);
    Y[e] = (i == j && i < r) ? 1.0 : 0.0;
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

int64_t trsv_sb_rows() { return SBR; }

size_t trsv_sb_bytes(int64_t n)
{
    const int64_t nsb = cdiv(n, SBR);
    return 4 * sizeof(double) * (size_t)nsb * SBR * SBR;
}

// Fills [Uinv | UinvT | N | N'] (each nsb blocks of SBR x SBR, row-major,
// FP64) for the upper factor U (stored FP64 or FP32) whose 64x64
// diagonal-block inverses are in Dinv.
template <typename T>
static int make_sb_t(const T *U, int64_t ldu, int64_t n, const double *Dinv, double *sb, hipStream_t st)
{
    const int64_t nsb = cdiv(n, SBR);
    const int64_t blk = (int64_t)SBR * SBR;
    double *Uinv = sb, *UinvT = sb + nsb * blk, *Nn = sb + 2 * nsb * blk, *Nt = sb + 3 * nsb * blk;
    if (hipMemsetAsync(sb, 0, trsv_sb_bytes(n), st) != hipSuccess) return GSYEIG_EHIP;
    for (int64_t S = 0; S < nsb; ++S) {
        const int64_t s0 = S * SBR;
        const int r = (int)((n - s0) < SBR ? (n - s0) : SBR);
        // UinvT block (row-major) == U_SS^-1 column-major: back-solve the identity
        double *X = UinvT + S * blk;
        hipLaunchKernelGGL(k_identity_sb, dim3((unsigned)cdiv(blk, 256)), dim3(256), 0, st, X, r);
        if (ok()) return GSYEIG_EHIP;
        int rc;
        if constexpr (sizeof(T) == 8)
            rc = launch_backsolve((const double *)U + s0 * ldu + s0, ldu, r, r, Dinv + (s0 / NB) * NB * NB, X,
                                  SBR, st);
        else
            rc = launch_backsolve_f32((const float *)U + s0 * ldu + s0, ldu, r, r, Dinv + (s0 / NB) * NB * NB,
                                      X, SBR, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_transpose_sb, dim3(TPS * TPS, (unsigned)nsb), dim3(256), 0, st, UinvT, Uinv);
    if (ok()) return GSYEIG_EHIP;
    for (int64_t S = 0; S < nsb; ++S) {
        const int64_t s0 = S * SBR;
        const int64_t r = std::min<int64_t>(SBR, n - s0);
        if (S + 1 < nsb) {  // N_S = Uinv_SS U_{S,S+1}
            const int64_t rn = std::min<int64_t>(SBR, n - s0 - SBR);
            GemmDesc d{};
            d.m = r; d.n = rn; d.k = r;
            d.A = Uinv + S * blk; d.lda = SBR; d.a_layout = 1;
            d.B = U + s0 * ldu + s0 + SBR; d.ldb = ldu; d.b_layout = 1; d.b_f32 = sizeof(T) == 4;
            d.C = Nn + S * blk; d.ldc = SBR; d.c_layout = 1;
            d.alpha = 1.0; d.beta = 0.0;
            int rc = launch_gemm_f64(d, st);
            if (rc) return rc;
        }
        if (S > 0) {  // N'_S = Uinv_SS^T U_{S-1,S}^T
            GemmDesc d{};
            d.m = r; d.n = SBR; d.k = r;
            d.A = UinvT + S * blk; d.lda = SBR; d.a_layout = 1;
            d.B = U + (s0 - SBR) * ldu + s0; d.ldb = ldu; d.b_layout = 0; d.b_f32 = sizeof(T) == 4;
            d.C = Nt + S * blk; d.ldc = SBR; d.c_layout = 1;
            d.alpha = 1.0; d.beta = 0.0;
            int rc = launch_gemm_f64(d, st);
            if (rc) return rc;
        }
    }
    return 0;
}

int launch_make_sb(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *sb,
                   hipStream_t st)
{
    return make_sb_t<double>(U, ldu, n, Dinv, sb, st);
}

int launch_make_sb_f32(const float *U, int64_t ldu, int64_t n, const double *Dinv, double *sb,
                       hipStream_t st)
{
    return make_sb_t<float>(U, ldu, n, Dinv, sb, st);
}

template <typename T>
static int trsv_sb_n_t(const T *U, int64_t ldu, int64_t n, const double *sb, const double *b, double *x,
                       double *rstage, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    const int64_t nsb = cdiv(n, SBR), blk = (int64_t)SBR * SBR;
    hipLaunchKernelGGL(k_trsv_sb_n<T>, dim3(nblk), dim3(1024), 0, st, U, ldu, n, nblk, sb,
                       sb + 2 * nsb * blk, b, x, rstage, ctl);
    return ok();
}

template <typename T>
static int trsv_sb_t_t(const T *U, int64_t ldu, int64_t n, const double *sb, const double *b, double *x,
                       double *rstage, PCtl *ctl, hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    const int64_t nsb = cdiv(n, SBR), blk = (int64_t)SBR * SBR;
    hipLaunchKernelGGL(k_trsv_sb_t<T>, dim3(nblk), dim3(1024), 0, st, U, ldu, n, nblk, sb + nsb * blk,
                       sb + 3 * nsb * blk, b, x, rstage, ctl);
    return ok();
}

int launch_trsv_sb_n(const double *U, int64_t ldu, int64_t n, const double *sb, const double *b,
                     double *x, double *rstage, PCtl *ctl, hipStream_t st)
{
    return trsv_sb_n_t<double>(U, ldu, n, sb, b, x, rstage, ctl, st);
}

int launch_trsv_sb_t(const double *U, int64_t ldu, int64_t n, const double *sb, const double *b,
                     double *x, double *rstage, PCtl *ctl, hipStream_t st)
{
    return trsv_sb_t_t<double>(U, ldu, n, sb, b, x, rstage, ctl, st);
}

int launch_trsv_sb_n_f32(const float *U, int64_t ldu, int64_t n, const double *sb, const double *b,
                         double *x, double *rstage, PCtl *ctl, hipStream_t st)
{
    return trsv_sb_n_t<float>(U, ldu, n, sb, b, x, rstage, ctl, st);
}

int launch_trsv_sb_t_f32(const float *U, int64_t ldu, int64_t n, const double *sb, const double *b,
                         double *x, double *rstage, PCtl *ctl, hipStream_t st)
{
    return trsv_sb_t_t<float>(U, ldu, n, sb, b, x, rstage, ctl, st);
}

// FP32 copy of an FP64 matrix (rows x cols, leading dimensions lds / ldd)
__global__ void k_to_f32(const double *__restrict__ src, int64_t lds, float *__restrict__ dst,
                         int64_t ldd, int64_t rows, int64_t cols)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = blockIdx.y;
    if (c < cols && r < rows) dst[r * ldd + c] = (float)src[r * lds + c];
}

int launch_to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows, int64_t cols,
                  hipStream_t st)
{
    for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
        const int64_t nr = std::min<int64_t>(65535, rows - r0);
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)cdiv(cols, 256), (unsigned)nr), dim3(256), 0, st,
                           src + r0 * lds, lds, dst + r0 * ldd, ldd, nr, cols);
        if (ok()) return GSYEIG_EHIP;
    }
    return 0;
}
