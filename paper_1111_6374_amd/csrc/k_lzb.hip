// k_lzb.hip -- the Lanczos phase of a batch of instances in one launch.
//
// One 1024-thread workgroup carries one instance through its whole Lanczos
// iteration (Section 2.3; keys KI1-KI5 of Table 1): every step applies
// C = U^-T A U^-1 to w_k -- the sweep with U, the product with A, the sweep
// with U^T, all vectors held in LDS -- then the three-term recurrence with
// the omega estimates of partial re-orthogonalisation (Simon 1984), two
// Gram-Schmidt passes against the basis on the steps those estimates flag,
// and, every few steps, the convergence test of the innermost wanted Ritz
// values of T_m (Sturm bisection; inverse iteration for the last
// components).  Workgroups take instances from a device-side counter over a
// largest-first order, so a batch of uneven sizes is one launch, and no
// workgroup ever waits on another.
//
// Operands (rows contiguous: element (r, c) of a matrix M at M[r * ld + c]):
//  * U: the Cholesky factor, upper triangle (c >= r) read only off the
//    64 x 64 diagonal blocks, whose FP64 inverses Dinv (row-major, 4096
//    doubles per block, zero beyond n) stand for them; a row's entries
//    from column n up to the next multiple of 4 must be zero (or absent:
//    n a multiple of the 16-byte group);
//  * A: symmetric, upper triangle read.
// U and A are FP32 (mixed mode) or FP64; vectors and sums are FP64.
//
// Thread layouts: in the sweep with U (row dots, back-substitution) a wave
// owns four rows of the current 64-row tile and its lanes stride along
// them; in the product with A and the sweep with U^T every thread owns four
// columns (16-byte groups) and walks down the rows, so each load
// instruction reads consecutive bytes of one row.  All sums are taken in a
// fixed order, so results do not depend on timing.
#include "internal.h"
#include "tridiag_dev.h"

namespace {

constexpr int NT = 1024;            // threads of a workgroup
constexpr int NW = NT / 64;         // its wavefronts
constexpr int NMX = LZB_NMAX;       // largest n
constexpr int CPT = NMX / NT;       // columns (rows) owned per thread
constexpr int QC = 16;              // innermost wanted values of a pre-check

struct Lds {
    double wk[NMX];       // w_k
    double wp[NMX];       // w_{k-1}; the Gram-Schmidt coefficients while they run
    double x[NMX];        // KI1: right-hand side, then U^-1 w_k
    double z[NMX];        // C w_k, then the residual vector
    double red[NW][64];   // partials of the 64 x 64 diagonal solves
    double t64[64];       // a tile's right-hand side
    double s16[NW];       // workgroup reductions
    int inst;
};

__device__ __forceinline__ double wsum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// workgroup sum (fixed order), returned to every thread
__device__ double bsum(double v, double *s16)
{
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s16[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t += s16[q];
    return t;
}

__device__ double bmax(double v, double *s16)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s16[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NW; ++q) t = fmax(t, s16[q]);
    return t;
}

// the start vector's generator (SplitMix64 of seed and index), the one the
// single-instance solver uses
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// The operands' addresses come from the descriptor in memory, so the
// compiler cannot tell they are global and would emit FLAT accesses, which
// also count against the LDS wait counter (every LDS read would then wait
// for all loads in flight).  Casting to the global address space keeps them
// global loads.
#define GAS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GAS T *gp(const T *p)
{
    return (const GAS T *)p;
}
template <typename T>
__device__ __forceinline__ GAS T *gpw(T *p)
{
    return (GAS T *)p;
}

template <typename T>
__device__ __forceinline__ T ldr(const T *p)
{
    return *gp(p);
}
template <typename T>
__device__ __forceinline__ double ld(const T *p)
{
    return (double)ldr(p);
}

// 16-byte groups: VW consecutive elements (4 FP32, 2 FP64) at a 16-byte
// aligned address.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
template <typename T> struct Vec;
template <> struct Vec<float> {
    using type = f4v;
    static constexpr int n = 4;
};
template <> struct Vec<double> {
    using type = d2v;
    static constexpr int n = 2;
};

// Matrix rows are read with buffer loads: the matrix's base and extent sit
// in a scalar resource, the row's byte offset is a scalar and a thread adds
// only its 32-bit column offset.  A per-thread 64-bit address per column
// group, live across the loops, does not fit the register budget of a
// 1024-thread workgroup; spilled, each of its reloads waits for every load
// in flight, and the stages' loads no longer overlap.  The matrix's bytes
// (n rows of ld elements) must stay below 2^31.
typedef unsigned u4v __attribute__((ext_vector_type(4)));
struct Mat {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t pitch;  // bytes per row
};
template <typename T>
__device__ __forceinline__ Mat mat(const T *p, int64_t ld, int64_t n)
{
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    Mat m;
    m.pitch = __builtin_amdgcn_readfirstlane((uint32_t)(ld * (int64_t)sizeof(T)));
    const uint32_t bytes = __builtin_amdgcn_readfirstlane((uint32_t)(n * ld * (int64_t)sizeof(T)));
    // word 3: 32-bit data format, the raw layout of CDNA buffer resources
    m.rs = __builtin_amdgcn_make_buffer_rsrc((void *)((uint64_t)hi << 32 | lo), (short)0, (int)bytes, 0x00020000);
    return m;
}
// VW elements of row r from column c (16-byte aligned), or zeros where ok
// is false: the column offset then lies past the resource's extent, and a
// buffer load out of range returns zeros without touching memory.  Every
// lane issues the load, so no branch splits a stage, and the wait for one
// stage's data leaves the next stage's loads in flight (a load skipped on
// some path would make that wait count every load).
template <typename T>
__device__ __forceinline__ typename Vec<T>::type ldrow(const Mat &m, int r, int c, bool ok)
{
    const unsigned voff = ok ? (unsigned)c * (unsigned)sizeof(T) : 0x80000000u;
    const u4v v = __builtin_amdgcn_raw_buffer_load_b128(m.rs, voff, (unsigned)r * m.pitch, 0);
    return __builtin_bit_cast(typename Vec<T>::type, v);
}

// Every load of the three operator passes reads matrix entries only; the
// chain of the solves is in the arithmetic.  So each pass streams its
// matrix in stages, issuing stage i + 1's loads (even across a tile
// boundary, before the tile's barriers) before the arithmetic of stage i.

// x := U^-1 x (x in LDS) by back-substitution over 64-row tiles: the rows of
// tile i take their dot products with the solved tail (a wave per four rows,
// each lane VW consecutive columns per load), then x_i = Dinv_i t.
template <typename T>
__device__ void sweep_u(const Mat &U, const double *__restrict__ Dinv, int64_t n, Lds &L)
{
    using VT = typename Vec<T>::type;
    constexpr int VW = Vec<T>::n, SPAN = 64 * VW, UB = 2;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nn = (int)n;
    const int nt = (nn + 63) / 64;
    // stage (tile t, first column c): rows 64 t + 4 w + j (clamped to the
    // tile), columns c + SPAN e .. + VW - 1; zero past n, and all zero
    // unless live (the stages past a tile's end and before tile 0 are
    // issued too, as zeros, so that no branch splits the pipeline)
    auto stage = [&](int t, int c, VT u[UB][4], bool live) {
        const int rt = nn - 64 * t < 64 ? nn - 64 * t : 64;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = 64 * t + ((4 * w + j) < rt ? 4 * w + j : rt - 1);
#pragma unroll
            for (int e = 0; e < UB; ++e) {
                const int ce = c + SPAN * e;
                u[e][j] = ldrow<T>(U, r, ce, live && ce < nn);
            }
        }
    };
    // the stages of tile t start at column 64 (t + 1) + VW lane, UB * SPAN apart
    auto nstages = [&](int t) {
        const int len = nn - 64 * (t + 1);
        return len > 0 ? (len + UB * SPAN - 1) / (UB * SPAN) : 1;
    };
    auto dot = [&](const VT u[UB][4], int c, double acc[4]) {
#pragma unroll
        for (int e = 0; e < UB; ++e)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                // past n, U's row padding and x are zero
                const double xc = L.x[c + SPAN * e + v];
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[j] = fma((double)u[e][j][v], xc, acc[j]);
            }
    };
    VT ua[UB][4], ub[UB][4];
    stage(nt - 1, 64 * nt + VW * lane, ua, true);
    for (int ti = nt - 1; ti >= 0; --ti) {
        const int r0 = ti * 64;
        const int rows = (nn - r0) < 64 ? (nn - r0) : 64;
        const double *Di = Dinv + (int64_t)ti * 4096;
        double dv[4], acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dv[j] = gp(Di)[(4 * w + j) * 64 + lane];
            acc[j] = 0.0;
        }
        // stage 0 is in ua; stages alternate between ua and ub
        const int ns = nstages(ti);
        const int cb = r0 + 64 + VW * lane;
        for (int st = 0;; st += 2) {
            // past the tile's last stage the columns are past n: zeros
            stage(ti, cb + (st + 1) * UB * SPAN, ub, true);
            dot(ua, cb + st * UB * SPAN, acc);
            if (st + 1 >= ns) break;
            stage(ti, cb + (st + 2) * UB * SPAN, ua, true);
            dot(ub, cb + (st + 1) * UB * SPAN, acc);
            if (st + 2 >= ns) break;
        }
        // the next tile's first stage, in flight across this tile's barriers
        stage(ti > 0 ? ti - 1 : 0, r0 + VW * lane, ua, ti > 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = wsum(acc[j]);
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * w + j;
                L.t64[r] = (r < rows) ? L.x[r0 + r] - acc[j] : 0.0;
            }
        }
        __syncthreads();
        const double tl = L.t64[lane];
        double xo[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) xo[j] = wsum(dv[j] * tl);
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * w + j < rows) L.x[r0 + 4 * w + j] = xo[j];
        }
        __syncthreads();
    }
}

// Owned columns: thread t holds the CPT columns VW t + NT VW q + v (q <
// CPT / VW, v < VW), so each 16-byte load covers a thread's group of VW.
template <typename T>
__device__ __forceinline__ int owned_col(int tid, int q)
{
    return Vec<T>::n * tid + NT * Vec<T>::n * q;
}

// y = A x for the owned columns from A's upper triangle, four rows per
// stage: an entry A(r, c), c >= r, adds A(r, c) x_r to the owner's y_c and,
// right of the diagonal, A(r, c) x_c to row r's sum.  A wave reduces its
// lanes' row sums for the stage's rows (halving the set at lane distances
// 32 and 16, then adding across the rest) into one scratch row per wave,
// P (NW x n); the 16 rows are added in a fixed order at the end.  Reading
// one triangle also makes the operator exactly symmetric: a matrix that is
// symmetric only to FP64 rounding can differ from its transpose by an FP32
// ulp once rounded to FP32, which the Lanczos recurrence does not tolerate.
template <typename T>
__device__ void symv_upper(const Mat &A, int64_t n, const double *xv, double *P, double y[CPT])
{
    using VT = typename Vec<T>::type;
    constexpr int VW = Vec<T>::n, NQ = CPT / VW, RG = 4;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nn = (int)n;
    double xq[CPT];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < VW; ++v) {
            const int c = owned_col<T>(tid, q) + v;
            y[q * VW + v] = 0.0;
            xq[q * VW + v] = (c < nn) ? xv[c] : 0.0;
        }
    // rows r0 .. r0 + RG - 1 at the owned column groups that reach the
    // diagonal; zero elsewhere and past row n - 1
    auto stage = [&](int r0, VT a[RG][NQ]) {
#pragma unroll
        for (int e = 0; e < RG; ++e) {
            const int r = r0 + e;
            const int rr = r < nn ? r : nn - 1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int c = owned_col<T>(tid, q);
                a[e][q] = ldrow<T>(A, rr, c, r < nn && c < nn && c + VW - 1 >= r);
            }
        }
    };
    double pacc = 0.0;
    auto group = [&](const VT a[RG][NQ], int r0) {
        double pr[RG];
#pragma unroll
        for (int e = 0; e < RG; ++e) {
            const int r = r0 + e;
            const double xr = (r < nn) ? xv[r] : 0.0;
            pr[e] = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int v = 0; v < VW; ++v) {
                    const int c = owned_col<T>(tid, q) + v;
                    // entries left of the diagonal or past n do not count
                    const double av = (c >= r && c < nn) ? (double)a[e][q][v] : 0.0;
                    y[q * VW + v] = fma(av, xr, y[q * VW + v]);
                    if (c > r) pr[e] = fma(av, xq[q * VW + v], pr[e]);
                }
        }
        const bool b5 = lane & 32, b4 = lane & 16;
        double h2[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const double snd = b5 ? pr[i] : pr[i + 2];
            h2[i] = (b5 ? pr[i + 2] : pr[i]) + __shfl_xor(snd, 32);
        }
        double h1 = (b4 ? h2[1] : h2[0]) + __shfl_xor(b4 ? h2[0] : h2[1], 16);
        h1 += __shfl_xor(h1, 8);
        h1 += __shfl_xor(h1, 4);
        h1 += __shfl_xor(h1, 2);
        h1 += __shfl_xor(h1, 1);
        // row r0 + e's sum is in the lanes 16 e .. 16 e + 15; lane l keeps
        // row 64 floor(r0 / 64) + l and the wave stores its 64 rows at once
        const double hv = __shfl(h1, 16 * (lane & 3));
        if ((lane >> 2) == ((r0 & 63) >> 2)) pacc = hv;
        if ((r0 & 63) == 64 - RG || r0 + RG >= nn) {
            const int rb = r0 & ~63;
            if (rb + lane < nn) gpw(P)[w * nn + rb + lane] = pacc;
        }
    };
    // every stage is issued (as zeros past row n - 1), so that no branch
    // splits the pipeline
    VT ga[RG][NQ], gb[RG][NQ];
    stage(0, ga);
    for (int r0 = 0;; r0 += 2 * RG) {
        stage(r0 + RG, gb);
        group(ga, r0);
        if (r0 + RG >= nn) break;
        stage(r0 + 2 * RG, ga);
        group(gb, r0 + RG);
        if (r0 + 2 * RG >= nn) break;
    }
    __syncthreads();
    double ps[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) ps[k] = 0.0;
#pragma unroll 2
    for (int u = 0; u < NW; ++u) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < VW; ++v) {
                const int c = owned_col<T>(tid, q) + v;
                if (c < nn) ps[q * VW + v] += gp(P)[u * nn + c];
            }
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) y[k] += ps[k];
}

// z = U^-T y (y in the owners' registers): forward substitution over 64-row
// tiles; tile i's owners hand their sums to the workgroup, z_i = Dinv_i^T t,
// then every owner of a later column subtracts tile i's rows times z_i,
// eight rows per stage.
template <typename T>
__device__ void sweep_ut(const Mat &U, const double *__restrict__ Dinv, int64_t n, double y[CPT], Lds &L)
{
    using VT = typename Vec<T>::type;
    constexpr int VW = Vec<T>::n, NQ = CPT / VW, RR = (sizeof(T) == 4) ? 8 : 4;
    constexpr int NG = 64 / RR;  // stages per tile (even)
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nn = (int)n;
    const int nt = (nn + 63) / 64;
    // stage (tile t, rows 64 t + RR g ..): the owned column groups right of
    // the tile; zero for rows past n - 1 (their z is 0) and for g past the
    // tile's last stage (issued too, so that no branch splits the pipeline)
    auto stage = [&](int t, int g, VT u[RR][NQ]) {
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            const int r = 64 * t + RR * g + e;
            const int rr = r < nn ? r : nn - 1;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int c = owned_col<T>(tid, q);
                u[e][q] = ldrow<T>(U, rr, c, g < NG && r < nn && c >= 64 * t + 64 && c < nn);
            }
        }
    };
    auto panel = [&](const VT u[RR][NQ], int zrow) {
#pragma unroll
        for (int e = 0; e < RR; ++e) {
            const double zr = L.z[zrow + e];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
#pragma unroll
                for (int v = 0; v < VW; ++v) y[q * VW + v] = fma(-(double)u[e][q][v], zr, y[q * VW + v]);
        }
    };
    VT pa[RR][NQ], pb[RR][NQ];
    for (int ti = 0; ti < nt; ++ti) {
        const int r0 = ti * 64;
        // the tile's first stage, in flight across the diagonal solve
        stage(ti, 0, pa);
        const double *Di = Dinv + (int64_t)ti * 4096;
        double dv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) dv[j] = gp(Di)[(4 * w + j) * 64 + lane];
        // the owners of the tile's columns hand over their sums
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int c = owned_col<T>(tid, q);
            if (c >= r0 && c < r0 + 64) {
#pragma unroll
                for (int v = 0; v < VW; ++v) L.t64[c - r0 + v] = (c + v < nn) ? y[q * VW + v] : 0.0;
            }
        }
        __syncthreads();
        double p = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) p = fma(dv[j], L.t64[4 * w + j], p);
        L.red[w][lane] = p;
        __syncthreads();
        if (w == 0) {
            double sum = 0.0;
#pragma unroll
            for (int u = 0; u < NW; ++u) sum += L.red[u][lane];
            L.z[r0 + lane] = sum;
        }
        __syncthreads();
#pragma unroll 1
        for (int g = 0; g < NG; g += 2) {
            stage(ti, g + 1, pb);
            panel(pa, r0 + RR * g);
            stage(ti, g + 2, pa);
            panel(pb, r0 + RR * (g + 1));
        }
    }
    __syncthreads();
}

// The convergence pre-check of the single-instance solver on the q
// innermost wanted Ritz values of T_m: their values and the two extremes by
// bisection (one wave per value), the last components of their vectors by
// two inverse-iteration solves from a random start (one wave per value),
// then the count of |beta_m| |e_m^T s_i| <= tol ||T||.  Returns the count;
// *ratio = the largest |beta_m| |e_m^T s_i| / (tol ||T||).
__device__ __noinline__ int precheck(const double *alpha, const double *beta, int64_t m, int64_t first, int qq, int which,
                        double tol, double *chk, int64_t mmax, double *ratio, Lds &L)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double *thq = chk, *lastc = chk + 32, *scr = chk + 64;
    for (int i = w; i < qq + 2; i += NW) {
        int64_t idx;
        if (i < qq) idx = first + i;
        else if (i == qq) idx = (which == 0) ? m - 1 : 0;
        else idx = (which == 0) ? 0 : m - 1;
        const double v = tdg::bisect_index(alpha, beta, m, idx);
        if (lane == 0) thq[i] = v;
    }
    __syncthreads();
    if (w < qq) {
        const int j = w;
        const double tn = fmax(fmax(fabs(thq[0]), fabs(thq[qq - 1])), fabs(thq[qq]));
        const double pivtiny = tdg::EPS * fmax(tn, 0x1p-1000);
        const double pert = 10.0 * tdg::EPS * fmax(tn, 0x1p-1000);
        int q0 = j;
        while (q0 > 0 && thq[q0] - thq[q0 - 1] < pert) --q0;
        const double lam = thq[j] + (double)(j - q0) * pert;
        double *f = scr + (int64_t)j * 6 * mmax;
        double *x = f + 5 * m;
        // f and x live in global memory and pass between the wave's lanes:
        // each hand-over waits for the stores (a workgroup-scope fence)
        tdg::tri_lu(alpha, beta, m, lam, pivtiny, f);
        for (int64_t t = lane; t < m; t += 64)
            x[t] = 2.0 * ((double)(tdg::mix64(0x5DEECE66Dull * (uint64_t)(j + 1) + (uint64_t)t) >> 11) * 0x1p-53) - 1.0;
        __threadfence_block();
        for (int it = 0; it < 2; ++it) {
            tdg::tri_solve(f, m, x);
            __threadfence_block();
            double s = 0.0;
            for (int64_t t = lane; t < m; t += 64) s = fma(x[t], x[t], s);
            s = wsum(s);
            const double inv = (s > 0.0) ? 1.0 / sqrt(s) : 0.0;
            for (int64_t t = lane; t < m; t += 64) x[t] *= inv;
            __threadfence_block();
        }
        if (lane == 0) lastc[j] = fabs(x[m - 1]);
    }
    __syncthreads();
    const double tn = fmax(fmax(fmax(fabs(thq[0]), fabs(thq[qq - 1])), fabs(thq[qq])), fabs(thq[qq + 1]));
    const double bm = fabs(beta[m - 1]);
    int c = 0;
    double mr = 0.0;
    for (int i = 0; i < qq; ++i) {
        c += (bm * lastc[i] <= tol * tn);
        mr = fmax(mr, bm * lastc[i] / fmax(tol * tn, 0x1p-1000));
    }
    *ratio = mr;
    __syncthreads();
    (void)L;
    return c;
}

template <typename T>
__device__ void run_instance(LzbDesc &d, Lds &L)
{
    const int tid = threadIdx.x;
    const uint64_t t0 = wall_clock64();
    const int64_t n = d.n, mmax = d.mmax, every = d.every, s = d.s, ldv = d.ldv;
    const Mat U = mat((const T *)d.U, d.ldu, n);
    const Mat A = mat((const T *)d.A, d.lda, n);
    double *V = d.V, *alpha = d.alpha, *beta = d.beta, *om = d.om;
    const int64_t ldom = d.ldom;
    double *P = d.chk;                         // NW x n row sums of the product with A
    double *chk = d.chk + (int64_t)NW * n;     // pre-check scratch
    const double eps1 = 0.5 * sqrt((double)n) * 0x1p-53;
    constexpr double thr = 1.0536712127723509e-08;  // sqrt(u), u = 2^-53
    int64_t k = d.k, next_check = d.next_check, prev_m = d.prev_m;
    double prev_rho = d.prev_rho, anorm = d.anorm;
    int forced = d.forced, nre = d.reorth_steps, status = 0;
    if (k == 0) {
        double ss = 0.0;
        for (int64_t i = tid; i < n; i += NT) {
            const double v = 2.0 * ((double)(splitmix(d.seed, (uint64_t)i) >> 11) * 0x1p-53) - 1.0;
            L.wk[i] = v;
            ss = fma(v, v, ss);
        }
        const double nrm = sqrt(bsum(ss, L.s16));
        for (int64_t i = tid; i < n; i += NT) {
            L.wk[i] = L.wk[i] / nrm;
            V[i] = L.wk[i];
            L.wp[i] = 0.0;
        }
        if (tid == 0) om[0] = 1.0;
        anorm = 0.0;
        forced = 0;
        nre = 0;
    } else {
        for (int64_t i = tid; i < n; i += NT) {
            L.wk[i] = V[k * ldv + i];
            L.wp[i] = V[(k - 1) * ldv + i];
        }
    }
    __syncthreads();
    while (k < mmax) {
        // KI1-KI3: z = U^-T A U^-1 w_k
        for (int64_t i = tid; i < n; i += NT) L.x[i] = L.wk[i];
        if (tid < 4 && n + tid < NMX) L.x[n + tid] = 0.0;
        __syncthreads();
        sweep_u<T>(U, d.Dinv, n, L);
        double y[CPT];
        symv_upper<T>(A, n, L.x, P, y);
        sweep_ut<T>(U, d.Dinv, n, y, L);
        // KI4: alpha_k, beta_k, the omega recurrence, w_{k+1}
        double *omC = om + (k % 3) * ldom, *omN = om + ((k + 1) % 3) * ldom;
        const double *omP = om + ((k + 2) % 3) * ldom;
        const double bkm1 = (k > 0) ? beta[k - 1] : 0.0;
        double zr[CPT], dd = 0.0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int64_t i = tid + (int64_t)NT * q;
            zr[q] = 0.0;
            if (i < n) {
                double zi = L.z[i];
                if (k > 0) zi = fma(-bkm1, L.wp[i], zi);
                zr[q] = zi;
                dd = fma(L.wk[i], zi, dd);
            }
        }
        const double ak = bsum(dd, L.s16);
        double ss = 0.0;
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int64_t i = tid + (int64_t)NT * q;
            if (i < n) {
                zr[q] = fma(-ak, L.wk[i], zr[q]);
                ss = fma(zr[q], zr[q], ss);
            }
        }
        double bk = sqrt(bsum(ss, L.s16));
        const double an = fmax(anorm, fabs(ak) + bk + bkm1);
        const double tau = eps1 * an;
        const double inv = (bk > 0.0) ? 1.0 / bk : 0.0;
        double mx = 0.0;
        for (int64_t j = tid; j < k; j += NT) {
            const GAS double *bg = gp(beta), *cg = gp(omC);
            double num = bg[j] * cg[j + 1] + (gp(alpha)[j] - ak) * cg[j] - bkm1 * gp(omP)[j];
            if (j > 0) num += bg[j - 1] * cg[j - 1];
            const double o = (num + copysign(tau, num)) * inv;
            gpw(omN)[j] = o;
            mx = fmax(mx, fabs(o));
        }
        mx = bmax(mx, L.s16);
        const int f = forced || !(mx <= thr) || (bk * thr < tau);
        if (f) {
            // two classical Gram-Schmidt passes against w_0 .. w_k
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int64_t i = tid + (int64_t)NT * q;
                if (i < n) L.z[i] = zr[q];
            }
            __syncthreads();
            const int lane = tid & 63, wv = tid >> 6;
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t j = wv; j <= k; j += NW) {
                    const GAS double *Vj = gp(V) + j * ldv;
                    double h = 0.0;
                    for (int64_t i = lane; i < n; i += 64) h = fma(Vj[i], L.z[i], h);
                    h = wsum(h);
                    if (lane == 0) L.wp[j] = h;
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < CPT; ++q) {
                    const int64_t i = tid + (int64_t)NT * q;
                    if (i < n) {
                        double v = L.z[i];
                        for (int64_t j = 0; j <= k; ++j) v = fma(-L.wp[j], gp(V)[j * ldv + i], v);
                        zr[q] = v;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < CPT; ++q) {
                    const int64_t i = tid + (int64_t)NT * q;
                    if (i < n) L.z[i] = zr[q];
                }
                __syncthreads();
            }
            ss = 0.0;
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int64_t i = tid + (int64_t)NT * q;
                if (i < n) ss = fma(zr[q], zr[q], ss);
            }
            const double bk0 = bk;
            bk = sqrt(bsum(ss, L.s16));
            for (int64_t j = tid; j < k; j += NT) omN[j] = eps1;
            nre += 1;
            // projections on an orthonormal basis never lengthen z: if they
            // did, the basis has lost orthogonality the estimates did not
            // see; stop this instance (the host solves it again per instance)
            if (!(bk <= bk0 * 1.001)) {
                status = 4;
                break;
            }
        }
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int64_t i = tid + (int64_t)NT * q;
            if (i < n) {
                const double wn = zr[q] / bk;
                gpw(V)[(k + 1) * ldv + i] = wn;
                L.wp[i] = L.wk[i];
                L.wk[i] = wn;
            }
        }
        if (tid == 0) {
            alpha[k] = ak;
            beta[k] = bk;
            omN[k] = f ? eps1 : tau * inv;
            omN[k + 1] = 1.0;
        }
        anorm = an;
        forced = f && !forced;
        __syncthreads();
        k += 1;
        const int64_t m = k;
        if (m >= d.nvec && (m >= next_check || m == mmax)) {
            next_check = m + every;
            if (m == mmax) {
                status = 3;
                break;
            }
            const int qq = (int)(s < QC ? s : QC);
            const int64_t first = d.which ? m - s : s - qq;
            double ratio;
            const int c = precheck(alpha, beta, m, first, qq, d.which, d.tol, chk, mmax, &ratio, L);
            if (c < qq) {
                const double rho = log10(fmax(ratio, 1.0));
                int64_t interval = 2 * every;
                if (prev_m >= 0 && prev_rho > rho) {
                    const double remaining = rho * (double)(m - prev_m) / (prev_rho - rho);
                    const int64_t rem = (int64_t)(0.6 * remaining);
                    interval = rem < every ? every : rem;
                    if (interval > 4 * every) interval = 4 * every;
                }
                prev_m = m;
                prev_rho = rho;
                next_check = m + interval;
                continue;
            }
            status = (qq == s) ? 1 : 2;
            break;
        }
    }
    if (k >= mmax && status == 0) status = 3;
    if (tid == 0) {
        d.k = k;
        d.next_check = next_check;
        d.prev_m = prev_m;
        d.prev_rho = prev_rho;
        d.anorm = anorm;
        d.forced = forced;
        d.reorth_steps = nre;
        d.status = status;
        d.ticks += (int64_t)(wall_clock64() - t0);
    }
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(1024) void k_lzb(LzbDesc *desc, const int *order, int count, unsigned *next)
{
    __shared__ Lds L;
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned q = __hip_atomic_fetch_add(next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            L.inst = (q < (unsigned)count) ? order[q] : -1;
        }
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(L.inst);
        __syncthreads();
        if (i < 0) break;
        run_instance<T>(desc[i], L);
    }
}

}  // namespace

int64_t lzb_scratch_doubles(int64_t n, int64_t mmax)
{
    return (int64_t)NW * n + 64 + (int64_t)QC * 6 * mmax;
}

int launch_lzb(LzbDesc *desc, const int *order, int count, unsigned *next, int f32, hipStream_t st)
{
    if (count <= 0) return 0;
    static int resident[2] = {0, 0};
    int &res = resident[f32 ? 1 : 0];
    if (!res) {
        int per_cu = 0, dev = 0, cus = 0;
        const void *fn = f32 ? (const void *)k_lzb<float> : (const void *)k_lzb<double>;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, NT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1, cus = 256;
        res = per_cu * cus;
    }
    const int grid = count < res ? count : res;
    if (hipMemsetAsync(next, 0, sizeof(unsigned), st) != hipSuccess) return GSYEIG_EHIP;
    if (f32)
        hipLaunchKernelGGL(k_lzb<float>, dim3((unsigned)grid), dim3(NT), 0, st, desc, order, count, next);
    else
        hipLaunchKernelGGL(k_lzb<double>, dim3((unsigned)grid), dim3(NT), 0, st, desc, order, count, next);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}
