// k_trsv_w.hip -- KI1 / KI3 (Section 2.3, Table 1) with the factor written
// as U = D (I + W): D = blockdiag(U_SS) over 512-row super-blocks S and
// W_ST = U_SS^-1 U_ST (T > S), computed once per factorisation.  Then
//
//   KI1, x = U^-1 b:  c_S = Uinv_SS b_S  (no dependency: formed first),
//                     x_S = c_S - sum_{T > S} W_ST x_T             (from the bottom)
//   KI3, x = U^-T b:  y_S = b_S - sum_{T < S} W_TS^T y_T            (from the top),
//                     x_S = Uinv_SS^T y_S  (after y_S is known: off the chain)
//
// The diagonal blocks of I + W are identities, so a chain link only polls
// the neighbour super-block's 512 values and applies the link block
// (W_{S,S+1} rows, or W_{S-1,S}^T, loaded into registers beforehand); every
// other term is accumulated as its values arrive.  The bytes per sweep are
// those of the triangle (W takes the place of U's off-diagonal blocks).
//
// One 1024-thread workgroup owns each 64-row tile; waves own 4 rows (KI1)
// or 4 outputs (KI3), lanes own columns.  Tickets, staging, bounded waits
// and the reset are those of the other chained kernels (chain.h).  W may be
// stored FP64 or FP32 (mixed mode); Uinv blocks, vectors and arithmetic
// are FP64.
#include <algorithm>

#include "chain.h"

#define TPS 8          // tiles per super-block
#define SBR (TPS * NB) // super-block rows
#define GRP 8          // far tiles per poll round (a whole super-block)
#define LG 4           // tiles per round of the double-buffered KI1 sweep

namespace {

using namespace chain;

// ------------------------------------------------------------------ KI1
template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_w_n(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk,
                                                   const double *__restrict__ Uinv, const double *b, double *x,
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

    // c rows: Uinv_SS[rowl + r][k] b_S[k], k >= rowl (upper triangle), k = c*64 + l
    double y[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < TPS; ++c) {
        if (c < loc) continue;
        const int64_t kk = s0 + (int64_t)c * NB + l;
        const double bv = (kk < n) ? b[kk] : 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            y[r] = fma(Uinv[(int64_t)S * SBR * SBR + (int64_t)(rowl + r) * SBR + c * NB + l], bv, y[r]);
    }

    // Every tile right of the super-block, from the last one (j = nblk-1) to
    // the first of S+1 (the link), subtracted from y as its x values arrive:
    // rounds of LG tiles, double-buffered, so a round's W values are in
    // flight while the previous round waits for its x values.  The link
    // tiles are simply the last rounds, and their W values are resident by
    // the time x_{S+1} is published.  Each round's polls are issued before
    // the next round's loads (loads complete in order).
    const int NT = has_next ? nblk - (S + 1) * TPS : 0;
    if (NT > 0) {
        const T *Wr = W + (r0 + 4 * w) * ldw;  // rows of a tile before the last super-block exist
        const int64_t cmax = n - 1;
        const int jdum = (S + 1) * TPS;
        auto colof = [&](int t) {
            const int j = (t < NT) ? nblk - 1 - t : jdum;
            const int64_t cc = (int64_t)j * NB + l;
            return cc < cmax ? cc : cmax;
        };
        double cur[LG][4], nxt[LG][4];
#pragma unroll
        for (int g = 0; g < LG; ++g) {
            const int64_t cc = colof(g);
#pragma unroll
            for (int r = 0; r < 4; ++r) cur[g][r] = (double)Wr[(int64_t)r * ldw + cc];
        }
        // wave 0 alone polls a round's x values and hands them to the other
        // waves through LDS (two slots, one barrier per round): sixteen times
        // fewer polls on the staging lines every workgroup is waiting for
        __shared__ double s_xr[2][LG * NB];
        for (int t0 = 0, rnd = 0; t0 < NT; t0 += LG, ++rnd) {
            unsigned long long v[LG];
            if (w == 0) {
#pragma unroll
                for (int g = 0; g < LG; ++g) v[g] = ld_bits(stage + colof(t0 + g));
            }
            if (t0 + LG < NT) {
#pragma unroll
                for (int g = 0; g < LG; ++g) {
                    const int64_t cc = colof(t0 + LG + g);
#pragma unroll
                    for (int r = 0; r < 4; ++r) nxt[g][r] = (double)Wr[(int64_t)r * ldw + cc];
                }
            }
            double *sx = s_xr[rnd & 1];
            if (w == 0) {
#pragma unroll
                for (int g = 0; g < LG; ++g) {
                    const int t = t0 + g;
                    const int64_t col = (int64_t)(nblk - 1 - t) * NB + l;
                    const bool live = (t < NT) && (col < n);
                    sx[g * NB + l] = live ? settle(v[g], stage + colof(t), ctl) : 0.0;
                }
            }
            __syncthreads();
#pragma unroll
            for (int g = 0; g < LG; ++g) {
                const double xv = sx[g * NB + l];
#pragma unroll
                for (int r = 0; r < 4; ++r) y[r] = fma(-cur[g][r], xv, y[r]);
            }
#pragma unroll
            for (int g = 0; g < LG; ++g)
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = nxt[g][r];
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
    retire(ctl, stage, n, nblk, &s_last);
}

// ------------------------------------------------------------------ KI3
// KI3's right-hand side given as the SYMV tile partials instead of b
// (Pr == nullptr: b is used): the workgroup of block row K sums the row parts
// of K and the column parts of tiles (I, K), I < K, in the order of
// k_symv_reduce (bitwise the same b), before its far loop -- one launch less.
struct RowSums {
    const double *Pr, *Pc;
    int maxch, ch;
};

template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_w_t(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk,
                                                   const double *__restrict__ UinvT,
                                                   const double *__restrict__ WLt, const double *b, double *x,
                                                   PCtl *ctl, RowSums rs)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_part[16][NB];
    __shared__ double s_y[SBR];  // y values of a super-block, polled once per workgroup
    double *stage = ctl_stage(ctl);  // holds y
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

    __shared__ double s_rs[4][NB];
    if (rs.Pr) {  // uniform
        if (w < 4) {
            const int K = i, q = w;
            const int nch = (nblk - K + rs.ch - 1) / rs.ch;
            // unrolled so that several loads are in flight; the sums keep
            // k_symv_reduce's order
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
    }
    // far tiles: rows of super-blocks T <= S-2, i.e. tiles j < (S-1)*TPS
    double acc = 0.0;
    const int ntile = (S - 1) * TPS;
    if (ntile > 0) {
        auto rowof = [&](int t) { return (int64_t)((t < ntile) ? t : ntile - 1) * NB + 4 * w; };
        for (int t0 = 0; t0 < ntile; t0 += GRP) {
            double cur[GRP][4];
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const int64_t rr = rowof(t0 + g);
#pragma unroll
                for (int r = 0; r < 4; ++r) cur[g][r] = (double)W[(rr + r) * ldw + colc];
            }
            // lane p < 4 GRP polls value p&3 of tile p>>2 of the group; the
            // values reach every lane by readlane
            const int p = l & (4 * GRP - 1);
            const int64_t prow = rowof(t0 + (p >> 2)) + (p & 3);
            const unsigned long long pv = ld_bits(stage + prow);
            const double zmine = settle_lazy(pv, stage + prow, ctl);
#pragma unroll
            for (int g = 0; g < GRP; ++g) {
                const bool live = (t0 + g < ntile);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double zv = rdlane(zmine, g * 4 + r);
                    acc = fma(cur[g][r], live ? zv : 0.0, acc);
                }
            }
        }
    }
    // far column sums of this tile's 64 outputs, folded over the 16 waves at publication
    s_part[w][l] = acc;
    __syncthreads();
    // the link: y_{S-1} through the rows of W_{S-1,S}^T
    double lk[4] = {0.0, 0.0, 0.0, 0.0};
    if (has_prev) {
        double nr[TPS][4];
#pragma unroll
        for (int c = 0; c < TPS; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) nr[c][r] = WLt[(int64_t)S * SBR * SBR + (int64_t)(al + r) * SBR + c * NB + l];
        // y_{S-1}: polled by wave 0 alone, handed over through LDS
        if (w == 0) {
            unsigned long long v[TPS];
#pragma unroll
            for (int c = 0; c < TPS; ++c) v[c] = ld_bits(stage + s0 - SBR + (int64_t)c * NB + l);
#pragma unroll
            for (int c = 0; c < TPS; ++c)
                s_y[c * NB + l] = settle(v[c], stage + s0 - SBR + (int64_t)c * NB + l, ctl);
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            const double yp = s_y[c * NB + l];
#pragma unroll
            for (int r = 0; r < 4; ++r) lk[r] = fma(nr[c][r], yp, lk[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) lk[r] = wave_sum(lk[r]);
    }
    if (l < 4) {
        const int64_t e = c0 + 4 * w + l;
        double f = 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) f += s_part[q][4 * w + l];
        const double ye = f + ((l == 0) ? lk[0] : (l == 1) ? lk[1] : (l == 2) ? lk[2] : lk[3]);
        const int r = 4 * w + l;
        const double be = (e >= n) ? 0.0 : rs.Pr ? (s_rs[0][r] + s_rs[1][r]) + (s_rs[2][r] + s_rs[3][r]) : b[e];
        if (e < n) st_bits(stage + e, (unsigned long long)__double_as_longlong(be - ye));
    }
    // the product below must not be scheduled into the link above
    __syncthreads();
    // x rows of this tile: Uinv_SS^T[al + r][k] y_S[k], k <= al + r (chunks c <= loc);
    // y_S is published by the tiles of S (this one included), polled together
    {
        // polled by wave 0 alone, handed over through LDS (the link's slot
        // is free: every wave has passed the barrier above since reading it)
        if (w == 0) {
            unsigned long long rb[TPS];
#pragma unroll
            for (int c = 0; c < TPS; ++c) {
                const int64_t kk = s0 + (int64_t)c * NB + l;
                rb[c] = ld_bits(stage + (kk < n ? kk : n - 1));
            }
#pragma unroll
            for (int c = 0; c < TPS; ++c) {
                const int64_t kk = s0 + (int64_t)c * NB + l;
                s_y[c * NB + l] = (c <= loc && kk < n) ? settle(rb[c], stage + kk, ctl) : 0.0;
            }
        }
        __syncthreads();
        double rv[TPS];
#pragma unroll
        for (int c = 0; c < TPS; ++c) rv[c] = s_y[c * NB + l];
        double xo[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < TPS; ++c) {
            if (c > loc) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                xo[r] = fma(UinvT[(int64_t)S * SBR * SBR + (int64_t)(al + r) * SBR + c * NB + l], rv[c], xo[r]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) xo[r] = wave_sum(xo[r]);
        if (l < 4) {
            const int64_t e = c0 + 4 * w + l;
            const double xi = (l == 0) ? xo[0] : (l == 1) ? xo[1] : (l == 2) ? xo[2] : xo[3];
            if (e < n) x[e] = xi;
        }
    }
    retire(ctl, stage, n, nblk, &s_last);
}

// WLt_S = (W_{S-1,S})^T for S >= 1 (blockIdx.y = S - 1): 64x64 tiles through
// LDS; columns of S beyond n are zero.
template <typename T>
__global__ __launch_bounds__(256) void k_link_transpose(const T *__restrict__ W, int64_t ldw, int64_t n,
                                                        double *WLt)
{
    __shared__ double t[NB][NB + 1];
    const int S = blockIdx.y + 1;
    const int tr = blockIdx.x / TPS, tc = blockIdx.x % TPS;  // tr: rows of S-1, tc: columns of S
    const int64_t s0 = (int64_t)S * SBR;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        const int64_t row = s0 - SBR + tr * NB + a, cl = s0 + tc * NB + c;
        t[a][c] = (cl < n) ? (double)W[row * ldw + cl] : 0.0;
    }
    __syncthreads();
    double *d = WLt + (int64_t)S * SBR * SBR;
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
        const int a = e / NB, c = e % NB;
        d[(int64_t)(tc * NB + a) * SBR + tr * NB + c] = t[c][a];
    }
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

// Uinv_SS (row-major) and its transpose for every 512-row diagonal
// super-block of U (stored FP64 or FP32), from the 64x64 block inverses in
// Dinv: the identity back-solved block by block (MFMA updates), then
// transposed.  Blocks beyond n are zero.
template <typename T>
int sb_inverses_t(const T *U, int64_t ldu, int64_t n, const double *Dinv, double *Uinv, double *UinvT,
                         hipStream_t st)
{
    const int64_t nsb = cdiv(n, SBR);
    const int64_t blk = (int64_t)SBR * SBR;
    if (hipMemsetAsync(Uinv, 0, sizeof(double) * (size_t)(nsb * blk), st) != hipSuccess) return GSYEIG_EHIP;
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
    return ok();
}

template <typename T>
int make_w_t(const T *U, int64_t ldu, int64_t n, const double *Dinv, double *sbw, T *W, int64_t ldw,
             hipStream_t st)
{
    const int64_t nsb = cdiv(n, SBR);
    const int64_t blk = (int64_t)SBR * SBR;
    double *Uinv = sbw, *UinvT = sbw + nsb * blk, *WLt = sbw + 2 * nsb * blk;
    int rc;
    if ((rc = sb_inverses_t<T>(U, ldu, n, Dinv, Uinv, UinvT, st))) return rc;
    if (hipMemsetAsync(WLt, 0, sizeof(double) * (size_t)(nsb * blk), st) != hipSuccess) return GSYEIG_EHIP;
    for (int64_t S = 0; S < nsb; ++S) {  // W_{S, >S} = Uinv_SS U_{S, >S}
        const int64_t s0 = S * SBR, s1 = s0 + SBR;
        if (s1 >= n) break;
        const int64_t r = std::min<int64_t>(SBR, n - s0);
        GemmDesc d{};
        d.m = r; d.n = n - s1; d.k = r;
        d.A = Uinv + S * blk; d.lda = SBR; d.a_layout = 1;
        d.B = U + s0 * ldu + s1; d.ldb = ldu; d.b_layout = 1; d.b_f32 = sizeof(T) == 4;
        d.C = W + s0 * ldw + s1; d.ldc = ldw; d.c_layout = 1; d.c_f32 = sizeof(T) == 4;
        d.alpha = 1.0; d.beta = 0.0;
        if ((rc = launch_gemm(d, st))) return rc;
    }
    if (nsb > 1) {
        hipLaunchKernelGGL(k_link_transpose<T>, dim3(TPS * TPS, (unsigned)(nsb - 1)), dim3(256), 0, st, W, ldw, n,
                           WLt);
        if (ok()) return GSYEIG_EHIP;
    }
    return 0;
}

}  // namespace

int64_t trsv_sb_rows() { return SBR; }

int launch_sb_inverses(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *Uinv, double *UinvT,
                       hipStream_t st)
{
    return sb_inverses_t<double>(U, ldu, n, Dinv, Uinv, UinvT, st);
}

int launch_sb_inverses_f32(const float *U, int64_t ldu, int64_t n, const double *Dinv, double *Uinv,
                           double *UinvT, hipStream_t st)
{
    return sb_inverses_t<float>(U, ldu, n, Dinv, Uinv, UinvT, st);
}

size_t trsv_w_side_bytes(int64_t n)
{
    const int64_t nsb = cdiv(n, SBR);
    return 3 * sizeof(double) * (size_t)nsb * SBR * SBR;
}

int launch_make_w(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *sbw, double *W, int64_t ldw,
                  hipStream_t st)
{
    return make_w_t<double>(U, ldu, n, Dinv, sbw, W, ldw, st);
}

int launch_make_w_f32(const float *U, int64_t ldu, int64_t n, const double *Dinv, double *sbw, float *W,
                      int64_t ldw, hipStream_t st)
{
    return make_w_t<float>(U, ldu, n, Dinv, sbw, W, ldw, st);
}

template <typename T>
static int trsv_w_n_t(const T *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                      hipStream_t st)
{
    const int nblk = (int)cdiv(n, NB);
    hipLaunchKernelGGL((k_trsv_w_n<T>), dim3(nblk), dim3(1024), 0, st, W, ldw, n, nblk, sbw, b, x, ctl);
    return ok();
}

template <typename T>
static int trsv_w_t_t(const T *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                      hipStream_t st, RowSums rs = RowSums{})
{
    const int nblk = (int)cdiv(n, NB);
    const int64_t nsb = cdiv(n, SBR), blk = (int64_t)SBR * SBR;
    hipLaunchKernelGGL((k_trsv_w_t<T>), dim3(nblk), dim3(1024), 0, st, W, ldw, n, nblk, sbw + nsb * blk,
                       sbw + 2 * nsb * blk, b, x, ctl, rs);
    return ok();
}

int launch_trsv_w_n(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                    PCtl *ctl, hipStream_t st)
{
    return trsv_w_n_t<double>(W, ldw, n, sbw, b, x, ctl, st);
}

int launch_trsv_w_t(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                    PCtl *ctl, hipStream_t st)
{
    return trsv_w_t_t<double>(W, ldw, n, sbw, b, x, ctl, st);
}

int launch_trsv_w_n_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                        PCtl *ctl, hipStream_t st)
{
    return trsv_w_n_t<float>(W, ldw, n, sbw, b, x, ctl, st);
}

int launch_trsv_w_t_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                        PCtl *ctl, hipStream_t st)
{
    return trsv_w_t_t<float>(W, ldw, n, sbw, b, x, ctl, st);
}

// KI3 with the right-hand side as SYMV tile partials (KI2's reduction done
// by the sweep's own workgroups)
int launch_trsv_w_t_rows(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *Pr,
                         const double *Pc, int maxch, int ch, double *x, PCtl *ctl, hipStream_t st)
{
    return trsv_w_t_t<double>(W, ldw, n, sbw, nullptr, x, ctl, st, RowSums{Pr, Pc, maxch, ch});
}

int launch_trsv_w_t_rows_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *Pr,
                             const double *Pc, int maxch, int ch, double *x, PCtl *ctl, hipStream_t st)
{
    return trsv_w_t_t<float>(W, ldw, n, sbw, nullptr, x, ctl, st, RowSums{Pr, Pc, maxch, ch});
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
