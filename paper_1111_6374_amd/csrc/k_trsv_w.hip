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
// KI2 fused into the KI1 sweep (optional, SYMV = true): once a workgroup has
// published its 64 values, its four 256-thread quarters take 64x64 tiles
// (I, J >= I) of A's upper triangle from a queue ordered by block row from
// the bottom (the order in which the sweep publishes x), wait (bounded) for
// x_I and x_J on the staging vector, and apply each tile both ways --
// y_I += A_IJ x_J, and y_J += A_IJ^T x_I for J > I -- into per-tile
// partials that k_symv_reduce sums in a fixed order.  The SYMV stream
// thereby runs in the bandwidth the latency-bound sweep leaves idle.  The
// waits are safe only if every workgroup is resident: the fused form is
// launched cooperatively.
struct SymvFuse {
    const void *A; int64_t lda;
    const int2 *items;   // (I, J) tiles in queue order
    int ntiles;
    double *Pr, *Pc;     // row partials [I][J - I][64], column partials [J][I][64]
};

constexpr int FUSE_GRAB = 16;  // tiles per queue ticket: 4 per quarter

template <typename TA>
__device__ __forceinline__ void symv_one_tile(const SymvFuse &sf, int64_t n, int nblk, double *stage, PCtl *ctl,
                                              double (*s_sp)[4][NB], int t)
{
    const TA *A = (const TA *)sf.A;
    const int tid = threadIdx.x;
    const int qd = tid >> 8, qt = tid & 255, ql = qt & 63, qw = qt >> 6;
    const int c = 16 * qw + (ql & 15), rg = ql >> 4;
    const bool have = t < sf.ntiles;
    int I = 0, J = 0;
    if (have) {
        const int2 it = sf.items[t];
        I = it.x;
        J = it.y;
    }
    const int64_t r0 = (int64_t)I * NB, col = (int64_t)J * NB + c;
    const bool colok = have && col < n;
    double a[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = r0 + rg + 4 * q;
        a[q] = (colok && row < n) ? (double)A[row * sf.lda + col] : 0.0;
    }
    const double *pj = stage + (colok ? col : 0);
    const unsigned long long vj = ld_bits(pj);
    unsigned long long vi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = r0 + rg + 4 * q;
        vi[q] = ld_bits(stage + ((have && row < n) ? row : 0));
    }
    const double xj = colok ? settle(vj, pj, &ctl->err) : 0.0;
    double acc[16], cs = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = r0 + rg + 4 * q;
        const double xi = (have && row < n) ? settle(vi[q], stage + row, &ctl->err) : 0.0;
        acc[q] = a[q] * xj;
        cs = fma(a[q], xi, cs);
    }
    // column part (J > I): sum over the tile's 64 rows
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (have && J > I && rg == 0) sf.Pc[((int64_t)J * nblk + I) * NB + c] = cs;
    // row part: sum over the 16 columns of this lane group, then over the 4 waves
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double v = acc[q];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        acc[q] = v;
    }
    if ((ql & 15) == 0) {
#pragma unroll
        for (int q = 0; q < 16; ++q) s_sp[qd][qw][rg + 4 * q] = acc[q];
    }
    __syncthreads();
    if (have && qt < NB)
        sf.Pr[((int64_t)I * nblk + (J - I)) * NB + qt] =
            (s_sp[qd][0][qt] + s_sp[qd][1][qt]) + (s_sp[qd][2][qt] + s_sp[qd][3][qt]);
    __syncthreads();
}

// Tickets of FUSE_GRAB tiles; the next ticket is taken while the current
// tiles are processed, so the queue's atomic is off the critical path.
template <typename TA>
__device__ __forceinline__ void symv_tiles_phase(const SymvFuse &sf, int64_t n, int nblk, double *stage, PCtl *ctl,
                                                 double (*s_sp)[4][NB], int *s_tk)
{
    const int tid = threadIdx.x, qd = tid >> 8;
    if (tid == 0) s_tk[0] = (int)atomicAdd(&ctl->pad, (unsigned)FUSE_GRAB);
    __syncthreads();
    int cur = s_tk[0];
    for (int round = 0; cur < sf.ntiles; ++round) {
        if (tid == 0) s_tk[(round + 1) & 1] = (int)atomicAdd(&ctl->pad, (unsigned)FUSE_GRAB);
#pragma unroll 1
        for (int u = 0; u < FUSE_GRAB / 4; ++u) symv_one_tile<TA>(sf, n, nblk, stage, ctl, s_sp, cur + 4 * qd + u);
        cur = s_tk[(round + 1) & 1];  // written before the last __syncthreads of the tiles
    }
}

template <typename T, typename TA, bool SYMV>
__global__ __launch_bounds__(1024) void k_trsv_w_n(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk,
                                                   const double *__restrict__ Uinv, const double *b, double *x,
                                                   PCtl *ctl, SymvFuse sf)
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
                    sx[g * NB + l] = live ? settle(v[g], stage + colof(t), &ctl->err) : 0.0;
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
    if constexpr (SYMV) {
        __shared__ double s_sp[4][4][NB];
        __shared__ int s_tk[2];
        symv_tiles_phase<TA>(sf, n, nblk, stage, ctl, s_sp, s_tk);
    }
    retire(ctl, stage, n, nblk, &s_last);
}

// ------------------------------------------------------------------ KI3
// KI2 fused into the KI3 sweep (optional, SYMV = true; FP64): the sweep's
// right-hand side A x is not an input.  Whenever the next group of far
// values (or, before the link, the tiles its own rows need) is not yet
// available, a workgroup applies 64x64 tiles of A's upper triangle, taken
// from a queue ordered by block row from the top (the order in which the
// sweep needs the rows), to the complete KI1 result.  Partial sums are
// written once each as data-carrying values into buffers that hold the
// sentinel between launches; the workgroup of row block K sums the N
// partials of its 64 rows (bounded waits) and restores the sentinels.  The
// chain's demand for A x is front-loaded exactly when most workgroups are
// still waiting for their turn.  Cooperative launch (the waits need every
// workgroup resident).
struct FuseT {
    const double *A; int64_t lda;
    const int2 *items;   // (I, J >= I) tiles, block rows from the top
    int ntiles;
    double *Pr, *Pc;     // sentinel-initialised row / column partials
    const double *xin;   // the complete KI1 result
};

// One queue round: each 256-thread quarter applies one tile.  WG-uniform.
__device__ __forceinline__ void ki3_symv_round(const FuseT &ft, int64_t n, int nblk, PCtl *ctl,
                                               double (*s_sp)[4][NB], int *s_q)
{
    const int tid = threadIdx.x;
    const int qd = tid >> 8, qt = tid & 255, ql = qt & 63, qw = qt >> 6;
    const int c = 16 * qw + (ql & 15), rg = ql >> 4;
    if (tid == 0) s_q[0] = (int)atomicAdd(&ctl->pad, 4u);
    __syncthreads();
    const int t = s_q[0] + qd;
    if (s_q[0] + 4 >= ft.ntiles) s_q[1] = 1;  // queue exhausted from now on (benign race: all write 1)
    const bool have = t < ft.ntiles;
    int I = 0, J = 0;
    if (have) {
        const int2 it = ft.items[t];
        I = it.x;
        J = it.y;
    }
    const int64_t r0 = (int64_t)I * NB, col = (int64_t)J * NB + c;
    const bool colok = have && col < n;
    double a[16], xi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t row = r0 + rg + 4 * q;
        const bool rok = have && row < n;
        a[q] = (colok && rok) ? ft.A[row * ft.lda + col] : 0.0;
        xi[q] = rok ? ft.xin[row] : 0.0;
    }
    const double xj = colok ? ft.xin[col] : 0.0;
    double cs = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) cs = fma(a[q], xi[q], cs);
    cs += __shfl_xor(cs, 16);
    cs += __shfl_xor(cs, 32);
    if (have && J > I && rg == 0)
        st_bits(ft.Pc + ((int64_t)J * nblk + I) * NB + c, (unsigned long long)__double_as_longlong(cs));
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        double v = a[q] * xj;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if ((ql & 15) == 0) s_sp[qd][qw][rg + 4 * q] = v;
    }
    __syncthreads();
    if (have && qt < NB) {
        const double v = (s_sp[qd][0][qt] + s_sp[qd][1][qt]) + (s_sp[qd][2][qt] + s_sp[qd][3][qt]);
        st_bits(ft.Pr + ((int64_t)I * nblk + (J - I)) * NB + qt, (unsigned long long)__double_as_longlong(v));
    }
    __syncthreads();
}

// KI3's right-hand side given as the SYMV tile partials instead of b
// (Pr == nullptr: b is used): the workgroup of block row K sums the row parts
// of K and the column parts of tiles (I, K), I < K, in the order of
// k_symv_reduce (bitwise the same b), before its far loop -- one launch less.
struct RowSums {
    const double *Pr, *Pc;
    int maxch, ch;
};

template <typename T, bool SYMV>
__global__ __launch_bounds__(1024) void k_trsv_w_t(const T *__restrict__ W, int64_t ldw, int64_t n, int nblk,
                                                   const double *__restrict__ UinvT,
                                                   const double *__restrict__ WLt, const double *b, double *x,
                                                   PCtl *ctl, FuseT ft, RowSums rs)
{
    __shared__ int s_blk, s_last;
    __shared__ double s_part[16][NB];
    __shared__ double s_sp[SYMV ? 4 : 1][4][NB];
    __shared__ double s_b[SYMV ? 16 : 1][NB];
    __shared__ int s_q[4];   // ticket, queue exhausted, ready flag
    __shared__ double s_y[SBR];  // y values of a super-block, polled once per workgroup
    double *stage = ctl_stage(ctl);  // holds y
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    if (tid == 0) {
        s_blk = take_ticket(ctl, nblk);
        s_q[1] = 0;
    }
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
            if constexpr (SYMV) {
                // while the group's values are not yet published, work the queue
                for (;;) {
                    if (w == 0) {
                        const int p = l & (4 * GRP - 1);
                        const int64_t prow = (int64_t)((t0 + (p >> 2) < ntile) ? t0 + (p >> 2) : ntile - 1) * NB +
                                             (p & 3);
                        const bool ok = ld_bits(stage + prow) != STAGE_SENTINEL;
                        const unsigned long long all = __ballot(ok);
                        if (l == 0) s_q[2] = (all == ~0ull) ? 1 : 0;
                    }
                    __syncthreads();
                    const int rdy = s_q[2], ex = s_q[1];
                    __syncthreads();
                    if (rdy || ex) break;
                    ki3_symv_round(ft, n, nblk, ctl, s_sp, s_q);
                }
            }
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
            const double zmine = settle_lazy(pv, stage + prow, &ctl->err);
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
    if constexpr (SYMV) {
        // the rows of this tile need the tiles of block rows 0..i: work the
        // queue until those have all been taken, then sum the N partials of
        // the tile's 64 rows (waiting for any still in flight)
        const int64_t N = nblk;
        const int64_t need = (int64_t)(i + 1) * N - (int64_t)i * (i + 1) / 2;
        for (;;) {
            if (tid == 0) s_q[2] = (int)__hip_atomic_load(&ctl->pad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int64_t taken = s_q[2];
            const int ex = s_q[1];
            __syncthreads();
            if (taken >= need || ex) break;
            ki3_symv_round(ft, n, nblk, ctl, s_sp, s_q);
        }
        double sb = 0.0;
        const int64_t nr = N - i;   // row partials of block row i
        for (int64_t q = w; q < N; q += 16) {
            double *pp = (q < nr) ? ft.Pr + ((int64_t)i * nblk + q) * NB + l
                                  : ft.Pc + ((int64_t)i * nblk + (q - nr)) * NB + l;
            sb += settle(ld_bits(pp), pp, &ctl->err);
            st_bits(pp, STAGE_SENTINEL);
        }
        s_b[w][l] = sb;
        __syncthreads();
    }
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
                s_y[c * NB + l] = settle(v[c], stage + s0 - SBR + (int64_t)c * NB + l, &ctl->err);
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
        double be;
        if constexpr (SYMV) {
            be = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) be += s_b[q][4 * w + l];
        } else {
            const int r = 4 * w + l;
            be = (e >= n) ? 0.0 : rs.Pr ? (s_rs[0][r] + s_rs[1][r]) + (s_rs[2][r] + s_rs[3][r]) : b[e];
        }
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
                s_y[c * NB + l] = (c <= loc && kk < n) ? settle(rb[c], stage + kk, &ctl->err) : 0.0;
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
    if constexpr (SYMV) {
        for (;;) {
            __syncthreads();
            const int ex = s_q[1];
            __syncthreads();
            if (ex) break;
            ki3_symv_round(ft, n, nblk, ctl, s_sp, s_q);
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
    hipLaunchKernelGGL((k_trsv_w_n<T, T, false>), dim3(nblk), dim3(1024), 0, st, W, ldw, n, nblk, sbw, b, x, ctl,
                       SymvFuse{});
    return ok();
}

template <typename T>
static int trsv_w_t_t(const T *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                      hipStream_t st, RowSums rs = RowSums{})
{
    const int nblk = (int)cdiv(n, NB);
    const int64_t nsb = cdiv(n, SBR), blk = (int64_t)SBR * SBR;
    hipLaunchKernelGGL((k_trsv_w_t<T, false>), dim3(nblk), dim3(1024), 0, st, W, ldw, n, nblk, sbw + nsb * blk,
                       sbw + 2 * nsb * blk, b, x, ctl, FuseT{}, rs);
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

// KI1 with KI2 fused (FP64 W and A): x = U^-1 b and the tile partials of
// A x, cooperative launch.  Returns GSYEIG_EHIP when the grid cannot be
// co-resident (the caller then runs the two kernels apart).
int fused_symv_fits(int64_t n)
{
    static int max_blocks = -1;
    if (max_blocks < 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_trsv_w_n<double, double, true>,
                                                         1024, 0) != hipSuccess)
            max_blocks = 0;
        else
            max_blocks = per_cu * cus;
    }
    return cdiv(n, NB) <= max_blocks;
}

int fused_ki3_fits(int64_t n)
{
    static int max_blocks = -1;
    if (max_blocks < 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_trsv_w_t<double, true>, 1024, 0) !=
                hipSuccess)
            max_blocks = 0;
        else
            max_blocks = per_cu * cus;
    }
    return cdiv(n, NB) <= max_blocks;
}

// KI2 and KI3 together: x = U^-T (A xin) (FP64 W and A), cooperative launch;
// Pr, Pc must hold the sentinel (they are left holding it).
int launch_trsv_w_t_symv(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *A, int64_t lda,
                         const double *xin, double *x, PCtl *ctl, const int2 *items, int ntiles, double *Pr,
                         double *Pc, hipStream_t st)
{
    if (!fused_ki3_fits(n)) return GSYEIG_EHIP;
    int nblk = (int)cdiv(n, NB);
    const int64_t nsb = cdiv(n, SBR), blk = (int64_t)SBR * SBR;
    const double *UinvT = sbw + nsb * blk, *WLt = sbw + 2 * nsb * blk;
    const double *bnull = nullptr;
    FuseT ft{A, lda, items, ntiles, Pr, Pc, xin};
    RowSums rs{};
    void *args[] = {(void *)&W,     (void *)&ldw,   (void *)&n, (void *)&nblk, (void *)&UinvT, (void *)&WLt,
                    (void *)&bnull, (void *)&x,     (void *)&ctl, (void *)&ft, (void *)&rs};
    if (hipLaunchCooperativeKernel((const void *)k_trsv_w_t<double, true>, dim3(nblk), dim3(1024), args, 0, st) !=
        hipSuccess)
        return GSYEIG_EHIP;
    return ok();
}

int launch_trsv_w_n_symv(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                         PCtl *ctl, const double *A, int64_t lda, const int2 *items, int ntiles, double *Pr,
                         double *Pc, hipStream_t st)
{
    if (!fused_symv_fits(n)) return GSYEIG_EHIP;
    int nblk = (int)cdiv(n, NB);
    SymvFuse sf{A, lda, items, ntiles, Pr, Pc};
    void *args[] = {(void *)&W, (void *)&ldw, (void *)&n, (void *)&nblk, (void *)&sbw, (void *)&b, (void *)&x,
                    (void *)&ctl, (void *)&sf};
    if (hipLaunchCooperativeKernel((const void *)k_trsv_w_n<double, double, true>, dim3(nblk), dim3(1024), args, 0,
                                   st) != hipSuccess)
        return GSYEIG_EHIP;
    return ok();
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
