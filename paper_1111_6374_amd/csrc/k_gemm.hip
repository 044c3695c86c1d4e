// k_gemm.hip -- dense tile contraction on CDNA4 matrix cores, FP64 or FP32.
//
// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j) over logical indices,
// with each operand's storage chosen by a layout code (column-major,
// row-major, or symmetric-from-lower-triangle) and a storage type (FP64 or
// FP32; values are converted to the compute type as they are loaded).  Used
// where the path is a dense contraction: the Cholesky panel and trailing
// SYRK update (Eq. 2), the Ritz vectors Y = V_m S (key KI5), the block
// back-substitution (Eq. 4), the block operator of the mixed-precision
// refinement and the FP64 residual check.
//
// Compute types: FP64 on v_mfma_f64_16x16x4_f64, FP32 on
// v_mfma_f32_16x16x4_f32 with FP32 accumulation (the mixed-precision
// trailing updates and block sweeps).
//
// Tiling: one 256-thread workgroup owns a 64x64 tile of C; its four wave64s
// each own a 32x32 quadrant = 2x2 MFMA blocks of 16x16.  K is staged through
// LDS 16 at a time, the next slab prefetched into registers while the
// current one is multiplied.  With split-K, blockIdx.z owns one K chunk and
// writes its partial tile to scratch; a second kernel adds the chunks in a
// fixed order (reproducible) and applies alpha/beta.
#include <stdint.h>

#include "internal.h"

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

template <typename T> struct Acc;
template <> struct Acc<double> { using type = dbl4; static constexpr int pad = 2; };
template <> struct Acc<float> { using type = flt4; static constexpr int pad = 16; };

template <typename TS, int L>
__device__ __forceinline__ TS load_op(const TS *p, int64_t ld, int64_t i, int64_t j, const double *diag)
{
    if constexpr (L == 0) return p[j * ld + i];
    else if constexpr (L == 1) return p[i * ld + j];
    else {
        if (i == j) return (TS)diag[i];
        return (i > j) ? p[i * ld + j] : p[j * ld + i];
    }
}

struct Args {
    int64_t m, n, k;
    const void *A; int64_t lda;
    const void *B; int64_t ldb;
    void *C; int64_t ldc; int c_row;
    double alpha, beta;
    const double *a_diag;
    int upper_only;
    int64_t kchunk;   // split-K chunk length (k when not split)
    double *part;     // split-K partial tiles, m x n column-major per chunk
};

// D layout of a 16x16 MFMA block: lane holds column (lane & 15); rows
// (lane >> 4) + 4 r for FP64 and 4 (lane >> 4) + r for FP32, r = 0..3.
template <typename TC>
__device__ __forceinline__ int d_row(int lk, int r)
{
    if constexpr (sizeof(TC) == 8) return lk + 4 * r;
    else return 4 * lk + r;
}

// WT = 1: 64x64 tiles, each wave a 32x32 quadrant (2x2 MFMA blocks);
// WT = 2: 128x128 tiles, each wave a 64x64 quadrant (4x4 blocks, the
// accumulators in the matrix cores' accumulation registers): twice the
// products per LDS fragment and per byte staged, for large m and n.
template <typename TC, typename TA, typename TB, typename TCS, int AL, int BL, int WT>
__global__ __launch_bounds__(256) void k_gemm(Args g)
{
    using V4 = typename Acc<TC>::type;
    constexpr int PAD = Acc<TC>::pad;
    constexpr int TMX = TM * WT, TNX = TN * WT;   // tile
    constexpr int NP = TMX * TK / 256;            // A (and B) values per thread per slab
    const TA *Ap = (const TA *)g.A;
    const TB *Bp = (const TB *)g.B;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int64_t tm0 = (int64_t)blockIdx.x * TMX;
    const int64_t tn0 = (int64_t)blockIdx.y * TNX;
    if (g.upper_only && tm0 > tn0 + TNX - 1) return;  // tile strictly below the diagonal
    const int64_t kbeg = (int64_t)blockIdx.z * g.kchunk;
    const int64_t kend = (kbeg + g.kchunk < g.k) ? kbeg + g.kchunk : g.k;

    __shared__ TC As[TK][TMX + PAD];
    __shared__ TC Bs[TK][TNX + PAD];

    // The next slab is fetched while the current one is multiplied: loads
    // come from clamped in-bounds indices (no predicated load) and stay in
    // their storage type until stash, which converts them and zeroes the
    // out-of-range ones -- nothing waits for the loads before the products.
    TA ra[NP];
    TB rb[NP];
    unsigned am = 0, bm = 0;
    // element p of this thread: A (AL = 0: contiguous rows) or B (BL = 1:
    // contiguous columns) along the tile edge, else along K
    auto a_idx = [&](int p, int &ii, int &kk) {
        if constexpr (AL == 0) { ii = tid % TMX; kk = tid / TMX + (256 / TMX) * p; }
        else { kk = tid & 15; ii = (tid >> 4) + 16 * p; }
    };
    auto b_idx = [&](int p, int &kk, int &jj) {
        if constexpr (BL == 1) { jj = tid % TNX; kk = tid / TNX + (256 / TNX) * p; }
        else { kk = tid & 15; jj = (tid >> 4) + 16 * p; }
    };
    auto fetch = [&](int64_t k0) {
        am = bm = 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            int ii, kk;
            a_idx(p, ii, kk);
            const int64_t gi = tm0 + ii, gk = k0 + kk;
            const bool ok = gi < g.m && gk < kend;
            am |= (unsigned)ok << p;
            if constexpr (AL == 2) {
                ra[p] = ok ? load_op<TA, AL>(Ap, g.lda, gi, gk, g.a_diag) : (TA)0;
            } else {
                ra[p] = load_op<TA, AL>(Ap, g.lda, gi < g.m ? gi : g.m - 1, gk < kend ? gk : kend - 1, nullptr);
            }
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            int kk, jj;
            b_idx(p, kk, jj);
            const int64_t gk = k0 + kk, gj = tn0 + jj;
            bm |= (unsigned)(gk < kend && gj < g.n) << p;
            rb[p] = load_op<TB, BL>(Bp, g.ldb, gk < kend ? gk : kend - 1, gj < g.n ? gj : g.n - 1, nullptr);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            int ii, kk;
            a_idx(p, ii, kk);
            As[kk][ii] = ((am >> p) & 1u) ? (TC)ra[p] : (TC)0;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            int kk, jj;
            b_idx(p, kk, jj);
            Bs[kk][jj] = ((bm >> p) & 1u) ? (TC)rb[p] : (TC)0;
        }
    };

    constexpr int NBK = 2 * WT;  // MFMA blocks per wave along each edge
    const int wm = wave & 1, wn = wave >> 1;
    V4 acc[NBK][NBK];
#pragma unroll
    for (int a = 0; a < NBK; ++a)
#pragma unroll
        for (int b = 0; b < NBK; ++b) acc[a][b] = V4{0, 0, 0, 0};

    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) fetch(kbeg);
    for (int64_t k0 = kbeg; k0 < kend; k0 += TK) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + TK < kend) fetch(k0 + TK);
#pragma unroll
        for (int kq = 0; kq < TK / 4; ++kq) {
            const int kr = kq * 4 + lk;
            TC av[NBK], bv[NBK];
#pragma unroll
            for (int a = 0; a < NBK; ++a) av[a] = As[kr][wm * 32 * WT + a * 16 + li];
#pragma unroll
            for (int b = 0; b < NBK; ++b) bv[b] = Bs[kr][wn * 32 * WT + b * 16 + li];
#pragma unroll
            for (int a = 0; a < NBK; ++a)
#pragma unroll
                for (int b = 0; b < NBK; ++b) {
                    if constexpr (sizeof(TC) == 8)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
                    else
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
                }
        }
    }

    TCS *Cp = (TCS *)g.C;
#pragma unroll
    for (int a = 0; a < NBK; ++a)
#pragma unroll
        for (int b = 0; b < NBK; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = tm0 + wm * 32 * WT + a * 16 + d_row<TC>(lk, r);
                const int64_t j = tn0 + wn * 32 * WT + b * 16 + li;
                if (i >= g.m || j >= g.n) continue;
                if (g.part) {  // split-K partial: plain sum, alpha/beta applied by the reduction
                    g.part[((int64_t)blockIdx.z * g.n + j) * g.m + i] = (double)acc[a][b][r];
                    continue;
                }
                if (g.upper_only && i > j) continue;
                TCS *cp = g.c_row ? &Cp[i * g.ldc + j] : &Cp[j * g.ldc + i];
                double v = g.alpha * (double)acc[a][b][r];
                if (g.beta != 0.0) v += g.beta * (double)*cp;
                *cp = (TCS)v;
            }
}

// ---------------------------------------------------------------- skinny
// C (m x n, column-major FP64) = alpha A B + beta C for n <= 32 columns: the
// shapes of the block operator (n rows times a block of b = 16 or 32
// columns; K = n for the symmetric product, 512 for the super-block
// updates).  One 256-thread workgroup owns 128 rows and all BN columns, so
// every element of A is read once.  K is staged through LDS in slabs of
// 32 KB of A (64 FP32 or 32 FP64 values deep), A kept in its storage type
// and converted as it enters the matrix cores; the next slab is loaded into
// registers with 16-byte vector loads while the current one is multiplied.
// Tiles that overhang m or K (and unaligned operands) load element-wise.
// A is FP64 or FP32, column- (AL = 0) or row-major (AL = 1); B is FP64
// column-major.
constexpr int SK_TM = 128;

struct SkArgs {
    int64_t m, n, k;
    const void *A; int64_t lda;
    const double *B; int64_t ldb;
    double *C; int64_t ldc;
    double alpha, beta;
    int vec;   // operands aligned for 16-byte loads
    int64_t sa, sb, sc;   // batch strides (elements); blockIdx.y = product
};

template <typename TC, typename TA, int AL, int BN>
__global__ __launch_bounds__(256) void k_gemm_skinny(SkArgs g)
{
    using V4 = typename Acc<TC>::type;
    constexpr int TK = 128 / (int)sizeof(TA) * 2;   // 64 (FP32 A) or 32 (FP64 A)
    constexpr int VA = 16 / (int)sizeof(TA);        // A values per 16-byte load
    constexpr int NA = SK_TM * TK / 256;            // A values per thread per slab (32 or 16)
    constexpr int NAV = NA / VA;                    // 16-byte loads of A per thread (8)
    constexpr int NBV = TK * BN / 256;               // B values per thread per slab
    constexpr int PADA = (sizeof(TA) == 8) ? 2 : 4;
    constexpr int NBLK = BN / 16;
    const TA *Ap = (const TA *)g.A + (int64_t)blockIdx.y * g.sa;
    g.B += (int64_t)blockIdx.y * g.sb;
    g.C += (int64_t)blockIdx.y * g.sc;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t tm0 = (int64_t)blockIdx.x * SK_TM;
    __shared__ TA As[TK][SK_TM + PADA];
    __shared__ TC Bs[TK][BN + 2];

    // A: vector v of thread t covers VA consecutive values along A's
    // contiguous index.  AL = 1 (row-major): row ii, k kk..kk+VA-1;
    // AL = 0 (column-major): k kk, rows ii..ii+VA-1.
    auto a_pos = [&](int v, int &ii, int &kk) {
        if constexpr (AL == 1) {
            constexpr int PR = TK / VA;                 // vectors per row
            const int e = tid + 256 * v;
            ii = e / PR;
            kk = (e % PR) * VA;
        } else {
            constexpr int PC = SK_TM / VA;              // vectors per column
            const int e = tid + 256 * v;
            kk = e / PC;
            ii = (e % PC) * VA;
        }
    };
    // B: thread t covers NBV consecutive k of column jb
    constexpr int BPC = TK / NBV;                        // threads per column
    const int jb = tid / BPC, kb = (tid % BPC) * NBV;

    TA ra[NA];
    double rb[NBV];
    auto fetch = [&](int64_t k0) {
        // B first: its few loads complete before the A slab, which then
        // stays in flight through the products of the current slab
        // uniform branch again: a column beyond n is read from column n - 1
        // (zeroed in stash), so no load is predicated; the values stay raw
        // until stash, so the loads remain in flight during the products
        const bool bfull = __builtin_amdgcn_readfirstlane((int)(g.vec && k0 + TK <= g.k));
        if (bfull) {
            const double *bsrc = g.B + (int64_t)(jb < g.n ? jb : g.n - 1) * g.ldb + k0 + kb;
#pragma unroll
            for (int u = 0; u < NBV; u += 2) {
                const double2 q = *(const double2 *)(bsrc + u);
                rb[u] = q.x;
                rb[u + 1] = q.y;
            }
        } else {
            const double *bsrc = g.B + (int64_t)jb * g.ldb + k0 + kb;
#pragma unroll
            for (int u = 0; u < NBV; ++u)
                rb[u] = (jb < g.n && k0 + kb + u < g.k) ? bsrc[u] : 0.0;
        }
        // one uniform branch around the whole slab, so that the vector loads
        // of the common (interior, aligned) case form one block and are all
        // in flight together
        const bool full = __builtin_amdgcn_readfirstlane((int)(g.vec && tm0 + SK_TM <= g.m && k0 + TK <= g.k));
        if (full) {
#pragma unroll
            for (int v = 0; v < NAV; ++v) {
                int ii, kk;
                a_pos(v, ii, kk);
                const int64_t gi = tm0 + ii, gk = k0 + kk;
                const TA *src = (AL == 1) ? Ap + gi * g.lda + gk : Ap + gk * g.lda + gi;
                if constexpr (sizeof(TA) == 4) {
                    const float4 q = *(const float4 *)src;
                    ra[v * 4 + 0] = q.x; ra[v * 4 + 1] = q.y; ra[v * 4 + 2] = q.z; ra[v * 4 + 3] = q.w;
                } else {
                    const double2 q = *(const double2 *)src;
                    ra[v * 2 + 0] = q.x; ra[v * 2 + 1] = q.y;
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < NAV; ++v) {
                int ii, kk;
                a_pos(v, ii, kk);
                const int64_t gi = tm0 + ii, gk = k0 + kk;
#pragma unroll
                for (int u = 0; u < VA; ++u) {
                    const int64_t ei = gi + ((AL == 1) ? 0 : u), ek = gk + ((AL == 1) ? u : 0);
                    ra[v * VA + u] = (ei < g.m && ek < g.k) ? Ap[(AL == 1) ? ei * g.lda + ek : ek * g.lda + ei]
                                                            : (TA)0;
                }
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int v = 0; v < NAV; ++v) {
            int ii, kk;
            a_pos(v, ii, kk);
#pragma unroll
            for (int u = 0; u < VA; ++u) {
                if constexpr (AL == 1) As[kk + u][ii] = ra[v * VA + u];
                else As[kk][ii + u] = ra[v * VA + u];
            }
        }
#pragma unroll
        for (int u = 0; u < NBV; ++u) Bs[kb + u][jb] = (jb < g.n) ? (TC)rb[u] : (TC)0;
    };

    V4 acc[2][NBLK];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NBLK; ++b) acc[a][b] = V4{0, 0, 0, 0};
    const int li = lane & 15, lk = lane >> 4;
    if (g.k > 0) fetch(0);
    for (int64_t k0 = 0; k0 < g.k; k0 += TK) {
        __syncthreads();
        stash();
        __syncthreads();
        if (k0 + TK < g.k) fetch(k0 + TK);
#pragma unroll
        for (int kq = 0; kq < TK / 4; ++kq) {
            const int kr = kq * 4 + lk;
            TC av[2], bv[NBLK];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = (TC)As[kr][wave * 32 + a * 16 + li];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) bv[b] = Bs[kr][b * 16 + li];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < NBLK; ++b) {
                    if constexpr (sizeof(TC) == 8)
                        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
                    else
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
                }
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NBLK; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = tm0 + wave * 32 + a * 16 + d_row<TC>(lk, r);
                const int64_t j = b * 16 + li;
                if (i >= g.m || j >= g.n) continue;
                double *cp = &g.C[j * g.ldc + i];
                double v = g.alpha * (double)acc[a][b][r];
                if (g.beta != 0.0) v += g.beta * *cp;
                *cp = v;
            }
}

template <typename TC, typename TA, int AL>
int run_skinny_bn(const SkArgs &a, int64_t batch, hipStream_t st)
{
    dim3 grid((unsigned)cdiv(a.m, SK_TM), (unsigned)batch);
    if (a.n <= 16) hipLaunchKernelGGL((k_gemm_skinny<TC, TA, AL, 16>), grid, dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_gemm_skinny<TC, TA, AL, 32>), grid, dim3(256), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

template <typename TC>
int run_skinny(SkArgs a, int a_f32, int al, int64_t batch, hipStream_t st)
{
    const int64_t va = a_f32 ? 4 : 2;
    a.vec = ((uintptr_t)a.A % 16 == 0) && (a.lda % va == 0) && ((uintptr_t)a.B % 16 == 0) && (a.ldb % 2 == 0) &&
            (batch == 1 || (a.sa % va == 0 && a.sb % 2 == 0));
    if (a_f32) return al ? run_skinny_bn<TC, float, 1>(a, batch, st) : run_skinny_bn<TC, float, 0>(a, batch, st);
    return al ? run_skinny_bn<TC, double, 1>(a, batch, st) : run_skinny_bn<TC, double, 0>(a, batch, st);
}

template <typename TCS>
__global__ void k_splitk_reduce(const double *__restrict__ part, int nz, int64_t m, int64_t n, void *C,
                                int64_t ldc, int c_row, double alpha, double beta, int upper_only)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * n) return;
    const int64_t i = t % m, j = t / m;
    if (upper_only && i > j) return;
    double s = 0.0;
    for (int z = 0; z < nz; ++z) s += part[(int64_t)z * m * n + t];
    TCS *Cp = (TCS *)C;
    TCS *cp = c_row ? &Cp[i * ldc + j] : &Cp[j * ldc + i];
    double v = alpha * s;
    if (beta != 0.0) v += beta * (double)*cp;
    *cp = (TCS)v;
}

// Tile choice: 128x128 where both edges are large (>= g_big_min) and the
// grid still fills the GPU; 0 disables the large tiles.
int64_t g_big_min = 2048;

template <typename TC, typename TA, typename TB, typename TCS, int AL, int BL>
int run(const Args &a, int nz, hipStream_t st)
{
    if (g_big_min > 0 && a.m >= g_big_min && a.n >= g_big_min) {
        dim3 grid((unsigned)cdiv(a.m, 2 * TM), (unsigned)cdiv(a.n, 2 * TN), (unsigned)nz);
        hipLaunchKernelGGL((k_gemm<TC, TA, TB, TCS, AL, BL, 2>), grid, dim3(256), 0, st, a);
    } else {
        dim3 grid((unsigned)cdiv(a.m, TM), (unsigned)cdiv(a.n, TN), (unsigned)nz);
        hipLaunchKernelGGL((k_gemm<TC, TA, TB, TCS, AL, BL, 1>), grid, dim3(256), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

template <typename TC, typename TA, typename TB, typename TCS>
int run_layout(const Args &a, int al, int bl, int nz, hipStream_t st)
{
    switch (al * 2 + bl) {
        case 0: return run<TC, TA, TB, TCS, 0, 0>(a, nz, st);
        case 1: return run<TC, TA, TB, TCS, 0, 1>(a, nz, st);
        case 2: return run<TC, TA, TB, TCS, 1, 0>(a, nz, st);
        case 3: return run<TC, TA, TB, TCS, 1, 1>(a, nz, st);
        case 4:
            if constexpr (sizeof(TA) == 8) return run<TC, TA, TB, TCS, 2, 0>(a, nz, st);
            else return GSYEIG_EHIP;
        case 5:
            if constexpr (sizeof(TA) == 8) return run<TC, TA, TB, TCS, 2, 1>(a, nz, st);
            else return GSYEIG_EHIP;
        default: return GSYEIG_EHIP;
    }
}

template <typename TC, typename TCS>
int run_types(const Args &a, const GemmDesc &d, int nz, hipStream_t st)
{
    const int ta = d.a_f32, tb = d.b_f32;
    if (!ta && !tb) return run_layout<TC, double, double, TCS>(a, d.a_layout, d.b_layout, nz, st);
    if (!ta && tb) return run_layout<TC, double, float, TCS>(a, d.a_layout, d.b_layout, nz, st);
    if (ta && !tb) return run_layout<TC, float, double, TCS>(a, d.a_layout, d.b_layout, nz, st);
    return run_layout<TC, float, float, TCS>(a, d.a_layout, d.b_layout, nz, st);
}

}  // namespace

int launch_gemm(const GemmDesc &d, hipStream_t st)
{
    if (d.m <= 0 || d.n <= 0) return 0;
    if (d.a_layout == 2 && d.a_f32) return GSYEIG_EHIP;
    const int64_t batch = d.batch > 1 ? d.batch : 1;
    // a block of at most 32 FP64 columns times a tall A: the skinny kernel
    if (d.n <= 32 && d.m >= SK_TM && d.a_layout != 2 && !d.b_f32 && !d.c_f32 && d.b_layout == 0 &&
        d.c_layout == 0 && !d.upper_only && d.splitk <= 1) {
        SkArgs a{d.m, d.n, d.k > 0 ? d.k : 0, d.A, d.lda, (const double *)d.B, d.ldb, (double *)d.C, d.ldc,
                 d.alpha, d.beta, 0, d.stride_a, d.stride_b, d.stride_c};
        return d.f32 ? run_skinny<float>(a, d.a_f32, d.a_layout, batch, st)
                     : run_skinny<double>(a, d.a_f32, d.a_layout, batch, st);
    }
    if (batch > 1) {  // other shapes: one launch per product
        GemmDesc e = d;
        e.batch = 1;
        const size_t ea = d.a_f32 ? 4 : 8, eb = d.b_f32 ? 4 : 8, ec = d.c_f32 ? 4 : 8;
        for (int64_t q = 0; q < batch; ++q) {
            e.A = (const char *)d.A + ea * (size_t)(q * d.stride_a);
            e.B = (const char *)d.B + eb * (size_t)(q * d.stride_b);
            e.C = (char *)d.C + ec * (size_t)(q * d.stride_c);
            const int rc = launch_gemm(e, st);
            if (rc) return rc;
        }
        return 0;
    }
    Args a{d.m, d.n, d.k > 0 ? d.k : 0, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.c_layout == 1,
           d.alpha, d.beta, d.a_diag, d.upper_only, 0, nullptr};
    int nz = 1;
    if (d.splitk > 1 && d.part && a.k > 0) {
        const int64_t kc = cdiv(cdiv(a.k, d.splitk), TK) * TK;
        nz = (int)cdiv(a.k, kc);
        a.kchunk = kc;
        a.part = d.part;
    } else {
        a.kchunk = a.k;
    }
    if (nz == 1) {
        a.part = nullptr;
        a.kchunk = a.k;
    }
    int rc;
    if (d.f32) {
        // FP32 compute: C stored FP64 or FP32
        rc = d.c_f32 ? run_types<float, float>(a, d, nz, st) : run_types<float, double>(a, d, nz, st);
    } else {
        rc = d.c_f32 ? run_types<double, float>(a, d, nz, st) : run_types<double, double>(a, d, nz, st);
    }
    if (rc || nz == 1) return rc;
    const int64_t tot = d.m * d.n;
    if (d.c_f32)
        hipLaunchKernelGGL(k_splitk_reduce<float>, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, st, d.part, nz,
                           d.m, d.n, d.C, d.ldc, (int)(d.c_layout == 1), d.alpha, d.beta, d.upper_only);
    else
        hipLaunchKernelGGL(k_splitk_reduce<double>, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, st, d.part, nz,
                           d.m, d.n, d.C, d.ldc, (int)(d.c_layout == 1), d.alpha, d.beta, d.upper_only);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

int launch_gemm_f64(const GemmDesc &d, hipStream_t st) { return launch_gemm(d, st); }

void gemm_set_big_min(int64_t m) { g_big_min = m; }
int64_t gemm_big_min() { return g_big_min; }

int64_t gemm_splitk_parts(const GemmDesc &d)
{
    if (d.splitk <= 1 || d.k <= 0) return 1;
    const int64_t kc = cdiv(cdiv(d.k, d.splitk), TK) * TK;
    return cdiv(d.k, kc);
}
