// blz.hip -- block Lanczos on the implicit operator C = U^-T A U^-1 with
// full re-orthogonalisation and thick restart (Sec. 2.3, variant KI, keys
// KI1-KI5 of Table 1 applied to blocks of b vectors).
//
// A step takes the newest basis block Q_j (n x b) to W = C Q_j -- two block
// triangular solves and one symmetric product on the matrix cores (TRSM,
// SYMM) -- then removes V^T W from W by classical Gram-Schmidt twice (GEMMs
// over the whole basis V) and factors the rest as W = Q_{j+1} R_{j+1}
// (Cholesky QR, the first of three passes shifted so that it cannot break
// down).  The Gram-Schmidt coefficients of the two passes, summed, are the
// column block j of H = V^T C V; H is symmetric, so only its upper triangle
// is kept and mirrored before the projected eigen-solve.  In exact arithmetic
// H is block tridiagonal (plus, after a restart, an arrow of couplings to the
// kept Ritz vectors); taking every computed coefficient makes it the
// projection of C on the computed basis, whatever orthogonality was lost.
//
// Convergence: with the Ritz pairs (theta_i, V s_i) of H, C V s_i - theta_i
// V s_i = Q_{j+1} R_{j+1} (last b entries of s_i), so the residual norm is
// ||R_{j+1} s_i,last||.  When the basis is full, the kept Ritz vectors
// nearest the wanted end replace it (Sec. 2.3: the best approximations
// restart the procedure) and the newest block Q_{j+1} continues it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

#define TRY(expr)                \
    do {                         \
        int _rc = (expr);        \
        if (_rc) return _rc;     \
    } while (0)

namespace {

constexpr int BMAX = 64;  // largest block

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

// Cholesky G + shift I = R^T R of a b x b Gram matrix (column-major, b <=
// 64), shift = shift_rel * trace(G).  Writes R (upper, zeros below) and
// R^-1, both column-major b x b, and, when Rprev is given, Racc = R Rprev
// (else Racc = R).  *flag = 1 when a pivot is not positive or has lost more
// than 24 digits of its diagonal entry (the columns were numerically
// dependent); the factorisation then continues on a floored pivot.
__global__ __launch_bounds__(256) void k_chol_small(const double *__restrict__ G, int b, double shift_rel,
                                                    double *__restrict__ R, double *__restrict__ Rinv,
                                                    const double *__restrict__ Rprev, double *__restrict__ Racc,
                                                    int *__restrict__ flag)
{
    __shared__ double L[BMAX][BMAX + 1];
    __shared__ double Iv[BMAX][BMAX + 1];
    __shared__ double g0[BMAX];
    __shared__ double s_tr;
    __shared__ int s_bad;
    const int t = threadIdx.x;
    for (int e = t; e < b * b; e += 256) {
        const int i = e % b, j = e / b;
        L[i][j] = G[(int64_t)j * b + i];
    }
    __syncthreads();
    if (t == 0) {
        double s = 0.0;
        for (int i = 0; i < b; ++i) s += L[i][i];
        s_tr = s;
        s_bad = (s > 0.0 && s < INFINITY) ? 0 : 1;
    }
    __syncthreads();
    if (t < b) {
        g0[t] = L[t][t];
        L[t][t] += shift_rel * s_tr;
    }
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        if (t == 0) {
            double p = L[k][k];
            const double fl = 1e-24 * g0[k] + 1e-300;
            if (!(p > fl)) {
                s_bad = 1;
                p = fl;
            }
            L[k][k] = sqrt(p);
        }
        __syncthreads();
        const double d = L[k][k];
        for (int j = k + 1 + t; j < b; j += 256) L[k][j] /= d;
        __syncthreads();
        for (int e = t; e < b * b; e += 256) {
            const int i = e % b, j = e / b;
            if (i > k && i <= j) L[i][j] -= L[k][i] * L[k][j];
        }
        __syncthreads();
    }
    // R^-1 by columns (upper triangular back substitution)
    if (t < b) {
        const int j = t;
        for (int i = b - 1; i >= 0; --i) {
            double v;
            if (i > j) v = 0.0;
            else {
                v = (i == j) ? 1.0 : 0.0;
                for (int k = i + 1; k <= j; ++k) v -= L[i][k] * Iv[k][j];
                v /= L[i][i];
            }
            Iv[i][j] = v;
        }
    }
    __syncthreads();
    for (int e = t; e < b * b; e += 256) {
        const int i = e % b, j = e / b;
        R[(int64_t)j * b + i] = (i <= j) ? L[i][j] : 0.0;
        Rinv[(int64_t)j * b + i] = Iv[i][j];
        double a;
        if (Rprev) {
            a = 0.0;
            for (int k = i; k <= j; ++k) a += L[i][k] * Rprev[(int64_t)j * b + k];
            if (i > j) a = 0.0;
        } else {
            a = (i <= j) ? L[i][j] : 0.0;
        }
        Racc[(int64_t)j * b + i] = a;
    }
    if (t == 0 && s_bad) *flag = 1;
}

// Hw (N x N, ld N) = the symmetric matrix whose upper triangle is H's
__global__ void k_mirror_upper(const double *__restrict__ H, int64_t ldh, int64_t N, double *__restrict__ Hw)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * N) return;
    const int64_t i = e % N, j = e / N;
    Hw[e] = (i <= j) ? H[j * ldh + i] : H[i * ldh + j];
}

__global__ void k_set_diag(double *__restrict__ H, int64_t ldh, const double *__restrict__ d, int64_t k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) H[i * ldh + i] = d[i];
}

// H[0:m, 0:b] += h[0:m, 0:b]
__global__ void k_add_cols(double *__restrict__ H, int64_t ldh, const double *__restrict__ h, int64_t ldhh,
                           int64_t m, int64_t b)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * b) return;
    const int64_t i = e % m, j = e / m;
    H[j * ldh + i] += h[j * ldhh + i];
}

// Residual norms ||R s_i,last|| of the Ritz pairs i0 .. i0+cnt-1 (S: N x nq,
// ld N, its last b rows are the last components); a pair has converged when
// its residual is at most tol times the largest |theta| seen (w[0], w[nq-1]
// and the opposite extreme w[nq]).  Writes the count and the largest
// residual / (tol ||T||).
__global__ __launch_bounds__(256) void k_blk_resid(const double *__restrict__ Racc, int b,
                                                   const double *__restrict__ S, int64_t N, int64_t i0,
                                                   int64_t cnt, const double *__restrict__ w, int64_t nq,
                                                   double tol, int *__restrict__ nconv,
                                                   double *__restrict__ ratio)
{
    __shared__ int s_cnt[256];
    __shared__ double s_max[256];
    const int t = threadIdx.x;
    const double tn = fmax(fmax(fabs(w[0]), fabs(w[nq - 1])), fabs(w[nq]));
    const double thr = tol * tn;
    int c = 0;
    double mx = 0.0;
    for (int64_t q = t; q < cnt; q += 256) {
        const double *sl = S + (i0 + q) * N + (N - b);
        double r2 = 0.0;
        for (int a = 0; a < b; ++a) {
            double v = 0.0;
            for (int k = a; k < b; ++k) v = fma(Racc[(int64_t)k * b + a], sl[k], v);
            r2 = fma(v, v, r2);
        }
        const double r = sqrt(r2);
        c += (r <= thr) ? 1 : 0;
        mx = fmax(mx, thr > 0.0 ? r / thr : INFINITY);
    }
    s_cnt[t] = c;
    s_max[t] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            s_cnt[t] += s_cnt[t + h];
            s_max[t] = fmax(s_max[t], s_max[t + h]);
        }
        __syncthreads();
    }
    if (t == 0) {
        *nconv = s_cnt[0];
        if (ratio) *ratio = s_max[0];
    }
}

// ------------------------------------------------------------ host pieces
// C (m x nn, column-major) = alpha X^T Y + beta C; X: n x m, Y: n x nn (FP64,
// split-K over n through `part`)
int gemm_tn(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t m, int64_t nn,
            double *C, int64_t ldc, double alpha, double beta, double *part, int64_t part_elems, hipStream_t st)
{
    GemmDesc d{};
    d.m = m; d.n = nn; d.k = n;
    d.A = X; d.lda = ldx; d.a_layout = 1;
    d.B = Y; d.ldb = ldy; d.b_layout = 0;
    d.C = C; d.ldc = ldc; d.c_layout = 0;
    d.alpha = alpha; d.beta = beta;
    const int64_t tiles = cdiv(m, 64) * cdiv(nn, 64);
    int64_t sk = std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 512), cdiv(1024, tiles)));
    while (sk > 1 && sk * m * nn > part_elems) sk /= 2;
    d.splitk = (int)sk;
    d.part = part;
    return launch_gemm(d, st);
}

// C (n x nn) = alpha X Q + beta C; X: n x m, Q: m x nn (FP64)
int gemm_nn(const double *X, int64_t ldx, const double *Q, int64_t ldq, int64_t n, int64_t m, int64_t nn,
            double *C, int64_t ldc, double alpha, double beta, hipStream_t st)
{
    if (m == 0) return 0;
    GemmDesc d{};
    d.m = n; d.n = nn; d.k = m;
    d.A = X; d.lda = ldx; d.a_layout = 0;
    d.B = Q; d.ldb = ldq; d.b_layout = 0;
    d.C = C; d.ldc = ldc; d.c_layout = 0;
    d.alpha = alpha; d.beta = beta;
    return launch_gemm(d, st);
}

struct Dims {
    int64_t b, keep, mmax, nq;
};

Dims dims(int64_t n, int64_t s, int64_t nvec, const gsyeig_opts *o)
{
    Dims d{};
    d.b = o->block;
    const int64_t cap = std::min<int64_t>(syev_small_max(), n - d.b);
    d.keep = (o->keep > 0) ? o->keep : std::max<int64_t>(nvec, std::min<int64_t>(2 * s, cap / 2));
    d.keep = std::max<int64_t>(d.keep, nvec);
    d.mmax = (o->basis > 0) ? o->basis : std::max<int64_t>(d.keep + 4 * d.b, 5 * s);
    d.mmax = std::min<int64_t>(d.mmax, cap);
    d.nq = d.keep;
    return d;
}

struct Bump {
    char *base;
    size_t off;
    template <typename T> T *take(size_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

struct Bufs {
    double *H, *Hw, *S, *w, *sy, *hc, *G, *R[3], *Rinv, *Racc[2], *part, *Wb, *t1, *t2, *Vtmp, *scal;
    int *flag;
    int64_t part_elems;
};

size_t layout(int64_t n, const Dims &d, Bufs *b, char *base)
{
    Bump m{base, 0};
    const int64_t ldv = cdiv(n, 64) * 64, M = d.mmax, B = d.b;
    Bufs x{};
    x.H = m.take<double>((size_t)M * M);
    x.Hw = m.take<double>((size_t)M * M);
    x.S = m.take<double>((size_t)M * d.nq);
    x.w = m.take<double>((size_t)d.nq + 8);
    x.sy = m.take<double>(syev_small_scratch(M, d.nq) / sizeof(double) + 8);
    x.hc = m.take<double>((size_t)(M + B) * B);
    x.G = m.take<double>((size_t)B * B);
    for (int i = 0; i < 3; ++i) x.R[i] = m.take<double>((size_t)B * B);
    x.Rinv = m.take<double>((size_t)B * B);
    x.Racc[0] = m.take<double>((size_t)B * B);
    x.Racc[1] = m.take<double>((size_t)B * B);
    x.part_elems = std::max<int64_t>((int64_t)1 << 22, 8 * (M + B) * B);
    x.part = m.take<double>((size_t)x.part_elems);
    x.Wb = m.take<double>((size_t)ldv * B);
    x.t1 = m.take<double>((size_t)ldv * B);
    x.t2 = m.take<double>((size_t)ldv * B);
    x.Vtmp = m.take<double>((size_t)ldv * d.keep);
    x.scal = m.take<double>(64);
    x.flag = m.take<int>(64);
    if (b) *b = x;
    return m.off + 4096;
}

// Y = C X for a block of b columns (X preserved).  sample: hipEvents around
// the three products (KI1, KI2, KI3), harvested by sample_harvest.
int block_apply(gsyeig_ctx *ctx, const BlkOp &op, int64_t n, const double *X, int64_t ldx, double *Y,
                int64_t ldy, int64_t b, const Bufs &w, int64_t ldw, bool sample)
{
    hipStream_t st = ctx->stream;
    sample = sample && ctx->npev + 4 <= 64;
    hipEvent_t *e = ctx->pev + ctx->npev;
    if (sample) HIP_TRY(hipEventRecord(e[0], st));
    if (op.W) {
        TRY(launch_trsm_w(0, op.W, op.w_f32, op.ldw, n, op.sb, const_cast<double *>(X), ldx, w.t2, ldw, b, op.f32,
                          st));
    } else {
        TRY(launch_blk_copy(X, ldx, w.t1, ldw, n, b, st));
        TRY(launch_trsm_sb(0, op.U, op.u_f32, op.ldu, n, op.sb, w.t1, ldw, w.t2, ldw, b, op.f32, st));
    }
    if (sample) HIP_TRY(hipEventRecord(e[1], st));
    GemmDesc d{};
    d.m = n; d.n = b; d.k = n;
    d.A = op.A; d.lda = op.lda; d.a_layout = 1; d.a_f32 = op.a_f32;
    d.B = w.t2; d.ldb = ldw; d.b_layout = 0;
    d.C = w.t1; d.ldc = ldw; d.c_layout = 0;
    d.alpha = 1.0; d.beta = 0.0;
    d.f32 = op.f32;
    TRY(launch_gemm(d, st));
    if (sample) HIP_TRY(hipEventRecord(e[2], st));
    if (op.W)
        TRY(launch_trsm_w(1, op.W, op.w_f32, op.ldw, n, op.sb, w.t1, ldw, Y, ldy, b, op.f32, st));
    else
        TRY(launch_trsm_sb(1, op.U, op.u_f32, op.ldu, n, op.sb, w.t1, ldw, Y, ldy, b, op.f32, st));
    if (sample) {
        HIP_TRY(hipEventRecord(e[3], st));
        ctx->npev += 4;
    }
    return 0;
}

int sample_harvest(gsyeig_ctx *ctx)
{
    for (int i = 0; i + 3 < ctx->npev; i += 4) {
        float t[3];
        for (int k = 0; k < 3; ++k) HIP_TRY(hipEventElapsedTime(&t[k], ctx->pev[i + k], ctx->pev[i + k + 1]));
        for (int k = 0; k < 3; ++k) ctx->prof_ms[k] += t[k];
        ctx->prof_samples += 1;
    }
    ctx->npev = 0;
    return 0;
}

// W (n x b, ld ldw) <- the Q of W = Q R by Cholesky QR in three passes, the
// first shifted; *Racc = R3 R2 R1.  Returns the Racc buffer used.
int chol_qr(int64_t n, int64_t b, double *W, int64_t ldw, const Bufs &w, int *flag, double **Racc_out,
            hipStream_t st)
{
    const double shift_rel = 11.0 * (double)(n * b + b * (b + 1)) * 1.1102230246251565e-16;
    const double *prev = nullptr;
    int cur = 0;
    for (int pass = 0; pass < 3; ++pass) {
        TRY(gemm_tn(W, ldw, W, ldw, n, b, b, w.G, b, 1.0, 0.0, w.part, w.part_elems, st));
        hipLaunchKernelGGL(k_chol_small, dim3(1), dim3(256), 0, st, w.G, (int)b, pass == 0 ? shift_rel : 0.0,
                           w.R[pass], w.Rinv, prev, w.Racc[cur], flag);
        TRY(ok());
        TRY(gemm_nn(W, ldw, w.Rinv, b, n, b, b, w.t1, ldw, 1.0, 0.0, st));
        TRY(launch_blk_copy(w.t1, ldw, W, ldw, n, b, st));
        prev = w.Racc[cur];
        cur ^= 1;
    }
    *Racc_out = w.Racc[cur ^ 1];
    return 0;
}

void fill_random_block(double *W, int64_t ldw, int64_t n, int64_t b, uint64_t seed, int64_t c0, hipStream_t st,
                       int *rc)
{
    for (int64_t c = 0; c < b && *rc == 0; ++c)
        *rc = launch_fill_splitmix(W + c * ldw, n, seed + 0x9E3779B97F4A7C15ull * (uint64_t)(c0 + c + 1), st);
}

}  // namespace

size_t blz_bytes(int64_t n, int64_t s, int64_t nvec, const gsyeig_opts *o)
{
    const Dims d = dims(n, s, nvec, o);
    return layout(n, d, nullptr, nullptr) + sizeof(double) * (size_t)cdiv(n, 64) * 64 * (size_t)(d.mmax + d.b);
}

int blz_check_dims(int64_t n, int64_t s, int64_t nvec, const gsyeig_opts *o)
{
    if (o->block < 2 || o->block > BMAX) return -8;
    const Dims d = dims(n, s, nvec, o);
    if (d.keep < nvec || d.keep + d.b > d.mmax || d.mmax > n - d.b) return -8;
    return 0;
}

int blz_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t nvec, const BlkOp &op, const gsyeig_opts *o,
              double *theta_out, double *Y, int64_t ldy, BlzResult *res)
{
    TRY(blz_check_dims(n, s, nvec, o));
    const Dims d = dims(n, s, nvec, o);
    const int64_t b = d.b, ldv = cdiv(n, 64) * 64, ldh = d.mmax;
    hipStream_t st = ctx->stream;
    void *p;
    TRY(ws_get(ctx, WS_V, sizeof(double) * (size_t)ldv * (size_t)(d.mmax + b), &p));
    double *V = (double *)p;
    TRY(ws_get(ctx, WS_BLZ, layout(n, d, nullptr, nullptr), &p));
    Bufs w;
    layout(n, d, &w, (char *)p);
    int *nconv_d = w.flag + 1, *flag_d = w.flag;
    double *ratio_d = w.scal;
    int *hflag = (int *)ctx->host_pinned;
    const int64_t wanted0 = o->which ? d.nq - s : 0;
    const int64_t max_ops = (o->max_steps > 0) ? o->max_steps : 50 * (100 * s + 2000);
    const int64_t stride = std::max<int64_t>(8 * b, (d.mmax - d.keep) / 2);
    // with FP32 accumulation the operator itself carries rounding of order
    // u_32 ||C||: Ritz residuals stall there, so the tolerance is no finer
    // than 64 u_32 (the FP64 refinement takes the pairs the rest of the way)
    const double tol = op.f32 ? std::max(o->tol, 64.0 * 5.9604644775390625e-8) : o->tol;
    memset(res, 0, sizeof(*res));
    const int64_t pe = o->profile_every;
    ctx->npev = 0;
    ctx->prof_samples = 0;
    ctx->prof_ms[0] = ctx->prof_ms[1] = ctx->prof_ms[2] = 0.0;

    HIP_TRY(hipEventRecord(ctx->ev[6], st));
    HIP_TRY(hipMemsetAsync(w.H, 0, sizeof(double) * (size_t)ldh * ldh, st));
    HIP_TRY(hipMemsetAsync(w.flag, 0, 64 * sizeof(int), st));
    // first block: v0 (if given) and SplitMix64 columns, orthonormalised
    int rc = 0;
    fill_random_block(V, ldv, n, b, o->seed, 0, st, &rc);
    TRY(rc);
    if (o->v0) TRY(launch_copy(o->v0, V, n, st));
    double *Racc = nullptr;
    TRY(chol_qr(n, b, V, ldv, w, flag_d, &Racc, st));

    int64_t c0 = 0, N = b, ops = 0, last_check = 0, nconv = 0;
    bool have_rr = false;
    for (;;) {
        // ---- one block step: W = C Q_j, CGS2 against V[:, 0:N], W = Q R
        double *Qj = V + c0 * ldv;
        const bool sample = pe > 0 && (ops / b) % pe == pe - 1;
        TRY(block_apply(ctx, op, n, Qj, ldv, w.Wb, ldv, b, w, ldv, sample));
        ops += b;
        double *Hc = w.H + c0 * ldh;
        TRY(gemm_tn(V, ldv, w.Wb, ldv, n, N, b, Hc, ldh, 1.0, 0.0, w.part, w.part_elems, st));
        TRY(gemm_nn(V, ldv, Hc, ldh, n, N, b, w.Wb, ldv, -1.0, 1.0, st));
        TRY(gemm_tn(V, ldv, w.Wb, ldv, n, N, b, w.hc, N, 1.0, 0.0, w.part, w.part_elems, st));
        TRY(gemm_nn(V, ldv, w.hc, N, n, N, b, w.Wb, ldv, -1.0, 1.0, st));
        hipLaunchKernelGGL(k_add_cols, dim3((unsigned)cdiv(N * b, 256)), dim3(256), 0, st, Hc, ldh, w.hc, N, N, b);
        TRY(ok());
        TRY(chol_qr(n, b, w.Wb, ldv, w, flag_d, &Racc, st));
        HIP_TRY(hipMemcpyAsync(hflag, flag_d, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        TRY(sample_harvest(ctx));
        if (*hflag) {
            // breakdown: C Q_j lies (numerically) in span(V); continue from
            // random directions orthogonal to V, with no coupling
            res->breakdowns += 1;
            HIP_TRY(hipMemsetAsync(flag_d, 0, sizeof(int), st));
            fill_random_block(w.Wb, ldv, n, b, o->seed ^ 0xB10C, ops, st, &rc);
            TRY(rc);
            for (int pass = 0; pass < 2; ++pass) {
                TRY(gemm_tn(V, ldv, w.Wb, ldv, n, N, b, w.hc, N, 1.0, 0.0, w.part, w.part_elems, st));
                TRY(gemm_nn(V, ldv, w.hc, N, n, N, b, w.Wb, ldv, -1.0, 1.0, st));
            }
            TRY(chol_qr(n, b, w.Wb, ldv, w, flag_d, &Racc, st));
            HIP_TRY(hipMemsetAsync(Racc, 0, sizeof(double) * (size_t)(b * b), st));
            HIP_TRY(hipMemcpyAsync(hflag, flag_d, sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            if (*hflag) break;  // no room left: stop with what the basis holds
        }
        TRY(launch_blk_copy(w.Wb, ldv, V + N * ldv, ldv, n, b, st));

        // ---- Rayleigh-Ritz on H[0:N, 0:N] when due
        const bool full = N + b > d.mmax;
        const bool stop = ops >= max_ops;
        if (N >= d.nq && (full || stop || N - last_check >= stride)) {
            last_check = N;
            hipLaunchKernelGGL(k_mirror_upper, dim3((unsigned)cdiv(N * N, 256)), dim3(256), 0, st, w.H, ldh, N,
                               w.Hw);
            TRY(ok());
            HIP_TRY(hipEventRecord(ctx->ev[2], st));
            TRY((ctx->syev_site = 1, syev_small(ctx, N, w.Hw, d.nq, o->which, w.w, w.S, w.sy, st)));
            HIP_TRY(hipEventRecord(ctx->ev[3], st));
            hipLaunchKernelGGL(k_blk_resid, dim3(1), dim3(256), 0, st, Racc, (int)b, w.S, N, wanted0, s, w.w,
                               d.nq, tol, nconv_d, ratio_d);
            TRY(ok());
            HIP_TRY(hipMemcpyAsync(hflag, nconv_d, sizeof(int), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            nconv = *hflag;
            have_rr = true;
            float tq;
            HIP_TRY(hipEventElapsedTime(&tq, ctx->ev[2], ctx->ev[3]));
            res->t_rr_ms += tq;
            res->rr_count += 1;
            if (nconv >= s || stop) break;
            if (full) {
                // thick restart: V[:, 0:keep] = V S_keep, then Q_{j+1}
                res->restarts += 1;
                const int64_t koff = o->which ? d.nq - d.keep : 0;
                TRY(gemm_nn(V, ldv, w.S + koff * N, N, n, N, d.keep, w.Vtmp, ldv, 1.0, 0.0, st));
                TRY(launch_blk_copy(w.Wb, ldv, V + d.keep * ldv, ldv, n, b, st));  // Q_{j+1} (also at V[:, N])
                TRY(launch_blk_copy(w.Vtmp, ldv, V, ldv, n, d.keep, st));
                HIP_TRY(hipMemsetAsync(w.H, 0, sizeof(double) * (size_t)ldh * ldh, st));
                hipLaunchKernelGGL(k_set_diag, dim3((unsigned)cdiv(d.keep, 256)), dim3(256), 0, st, w.H, ldh,
                                   w.w + koff, d.keep);
                TRY(ok());
                c0 = d.keep;
                N = d.keep + b;
                last_check = N;
                have_rr = false;
                continue;
            }
        } else if (stop) {
            break;
        }
        c0 = N;
        N += b;
        have_rr = false;
    }
    if (!have_rr) {
        if (N < d.nq) return GSYEIG_ENOCONV;
        hipLaunchKernelGGL(k_mirror_upper, dim3((unsigned)cdiv(N * N, 256)), dim3(256), 0, st, w.H, ldh, N, w.Hw);
        TRY(ok());
        TRY((ctx->syev_site = 1, syev_small(ctx, N, w.Hw, d.nq, o->which, w.w, w.S, w.sy, st)));
    }
    HIP_TRY(hipEventRecord(ctx->ev[7], st));
    // Ritz vectors Y = V S for the nvec pairs nearest the wanted end
    const int64_t off = o->which ? d.nq - nvec : 0;
    TRY(gemm_nn(V, ldv, w.S + off * N, N, n, N, nvec, Y, ldy, 1.0, 0.0, st));
    TRY(launch_copy(w.w + off, theta_out, nvec, st));
    HIP_TRY(hipEventRecord(ctx->ev[5], st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipEventElapsedTime(&res->t_loop_ms, ctx->ev[6], ctx->ev[7]));
    HIP_TRY(hipEventElapsedTime(&res->t_ritz_ms, ctx->ev[7], ctx->ev[5]));
    res->steps = ops;
    res->nconv = nconv;
    res->basis = d.mmax;
    res->keep = d.keep;
    return 0;
}
