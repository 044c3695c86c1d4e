// gsyeig_api.hip -- host driver and C ABI (see include/gsyeig.h).
//
// The driver only sequences kernels on the context's stream and moves a few
// scalars (info codes, the converged count, check results) to the host.
// Every arithmetic step of the path runs in the kernels of this library.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <numeric>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"

// ------------------------------------------------------------------ workspace
int ws_get(gsyeig_ctx *ctx, int slot, size_t bytes, void **out)
{
    if (bytes == 0) bytes = 256;
    if (ctx->ws_bytes[slot] >= bytes) {
        *out = ctx->ws[slot];
        return 0;
    }
    if (ctx->ws[slot]) {
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        HIP_TRY(hipFree(ctx->ws[slot]));
        ctx->ws[slot] = nullptr;
        ctx->ws_bytes[slot] = 0;
        if (slot == WS_SYMVMAP) ctx->symv_map_n = -1;
    }
    const size_t sz = (bytes + 4095) & ~(size_t)4095;
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        return GSYEIG_ENOMEM;
    }
    ctx->ws[slot] = p;
    ctx->ws_bytes[slot] = sz;
    *out = p;
    return 0;
}

// counters, then two staging vectors of `rows` entries (solved values x and,
// for the super-block solves, the partial right-hand sides r')
static size_t ctl_bytes(int64_t rows) { return PCTL_STAGE_OFFSET + 2 * sizeof(double) * (size_t)rows; }
static double *ctl_rstage(gsyeig_ctx *ctx, PCtl *c) { return ctl_stage(c) + ctx->ctl_rows; }

// zero counters, the context's spin bound, staging entries all
// STAGE_SENTINEL (all-ones bytes)
static int ctl_init(gsyeig_ctx *ctx, PCtl *c, int64_t rows)
{
    HIP_TRY(hipMemsetAsync(c, 0, PCTL_STAGE_OFFSET, ctx->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&c->spin, (int)ctx->spin_limit, 1, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctl_stage(c), 0xFF, 2 * sizeof(double) * (size_t)rows, ctx->stream));
    return 0;
}

// Forget expired waits of earlier work (stream-ordered): a synchronous
// entry point then reports only the waits of its own kernels.
static int ctl_clear_err(gsyeig_ctx *ctx)
{
    HIP_TRY(hipMemsetAsync(&ctx->ctl_n->err, 0, sizeof(unsigned), ctx->stream));
    HIP_TRY(hipMemsetAsync(&ctx->ctl_t->err, 0, sizeof(unsigned), ctx->stream));
    HIP_TRY(hipMemsetAsync(&ctx->ctl_lz->err, 0, sizeof(unsigned), ctx->stream));
    return 0;
}

// the fused Lanczos step's queue: counters zero, the context's spin bound
static int lzctl_init(gsyeig_ctx *ctx)
{
    HIP_TRY(hipMemsetAsync(ctx->ctl_lz, 0, sizeof(LzCtl), ctx->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&ctx->ctl_lz->spin, (int)ctx->spin_limit, 1, ctx->stream));
    return 0;
}

int ctl_reserve(gsyeig_ctx *ctx, int64_t rows)
{
    if (rows <= ctx->ctl_rows) return 0;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (ctx->ctl_n) HIP_TRY(hipFree(ctx->ctl_n));
    if (ctx->ctl_t) HIP_TRY(hipFree(ctx->ctl_t));
    ctx->ctl_n = ctx->ctl_t = nullptr;
    ctx->ctl_rows = 0;
    const int64_t cap = std::max<int64_t>(cdiv(rows, NB) * NB, 65536);
    HIP_TRY(hipMalloc((void **)&ctx->ctl_n, ctl_bytes(cap)));
    HIP_TRY(hipMalloc((void **)&ctx->ctl_t, ctl_bytes(cap)));
    int rc;
    if ((rc = ctl_init(ctx, ctx->ctl_n, cap)) || (rc = ctl_init(ctx, ctx->ctl_t, cap))) return rc;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->ctl_rows = cap;
    return 0;
}

// Reads and clears the persistent kernels' sticky wait-expiry flags.
static int ctl_check(gsyeig_ctx *ctx)
{
    unsigned *h = (unsigned *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, &ctx->ctl_n->err, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(h + 1, &ctx->ctl_t->err, sizeof(unsigned), hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipMemcpyAsync(h + 2, &ctx->ctl_lz->err, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (h[0] || h[1] || h[2]) {
        // a wait expired: restart the control blocks and the queue sweeps'
        // partial buffers from a clean state
        ctx->trsvq_n = -1;
        int rc;
        if ((rc = ctl_init(ctx, ctx->ctl_n, ctx->ctl_rows)) || (rc = ctl_init(ctx, ctx->ctl_t, ctx->ctl_rows)) ||
            (rc = lzctl_init(ctx)))
            return rc;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return GSYEIG_ESPIN;
    }
    return 0;
}

#define TRY(expr)                \
    do {                         \
        int _rc = (expr);        \
        if (_rc) return _rc;     \
    } while (0)

static void opts_fill_defaults(gsyeig_opts *o)
{
    memset(o, 0, sizeof(*o));
    o->prec = GSYEIG_FP64;
    o->block = 1;
    o->which = 0;
    o->invert = 0;
    o->tol = 1e-12;
    o->max_steps = 0;  // 0 = default_max_steps(n, s)
    o->check_every = 25;
    o->seed = 6374;
    o->v0 = nullptr;
    o->profile_every = 0;
    o->eta_tol = 1e-10;
    o->refine_iters = 10;
    o->refine_inner = 20;
    o->guard = 0;
    o->reorth = 2;
}

// width of the mixed-mode refinement block: s wanted + guard vectors
static int64_t mixed_block(int64_t n, int64_t s, const gsyeig_opts *o)
{
    const int64_t g = (o->guard > 0) ? o->guard : std::max<int64_t>(8, cdiv(s, 4));
    return std::min<int64_t>(n, std::min<int64_t>(s + g, syev_small_max() / 2));
}

// Default cap on the Lanczos steps: 100 s + 2000, raised to 10 sqrt(n s)
// for small s on large n (the steps a clustered spectrum needs grow like
// sqrt(n s): about 4.5 sqrt(n s) for 80 % of the values in [0, 1]).
static int64_t default_max_steps(int64_t n, int64_t s)
{
    const int64_t by_s = 100 * s + 2000;
    const int64_t by_ns = (int64_t)(10.0 * sqrt((double)n * (double)s));
    return std::min<int64_t>(n, std::max<int64_t>(by_s, by_ns));
}

static int64_t eff_max_steps(int64_t n, int64_t s, const gsyeig_opts *o)
{
    int64_t m = (o && o->max_steps > 0) ? o->max_steps : default_max_steps(n, s);
    m = std::min<int64_t>(m, n);
    return std::max<int64_t>(m, std::min<int64_t>(s, n));
}

static int64_t round_ld(int64_t n) { return cdiv(n, 64) * 64; }

// rows of the outer blocks of the Cholesky factorisation (rank of the
// deferred trailing updates); a multiple of the 64-row diagonal blocks
constexpr int64_t POTRF_OUTER = 256;

// ------------------------------------------------------------------ steps
// Block data of the factor used by the solves, one WS_DINV allocation:
// [Dinv_i | M_i = Dinv_i U_{i,i+1} | M'_i = Dinv_i^T U_{i-1,i}^T], 64x64 each.
static size_t tri_aux_bytes(int64_t n) { return 3 * sizeof(double) * (size_t)cdiv(n, NB) * NB * NB; }
static const double *aux_m(const double *Dinv, int64_t n) { return Dinv + cdiv(n, NB) * NB * NB; }

static int dinv_from_u(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, double **Dinv);

// Side data of the factor for the solves: M blocks always; for the
// super-block solves the super-block inverses, the link blocks and
// W = blockdiag(U_SS)^-1 U_offdiag (WS_SB, WS_W).
static int prepare_solves(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, double *Dinv)
{
    TRY(launch_make_m(U, ldu, n, Dinv, Dinv + cdiv(n, NB) * NB * NB, ctx->stream));
    if (ctx->trsv_block == 64) return 0;
    void *p, *q;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    TRY(ws_get(ctx, WS_W, sizeof(double) * (size_t)round_ld(n) * (size_t)n, &q));
    return launch_make_w(U, ldu, n, Dinv, (double *)p, (double *)q, round_ld(n), ctx->stream);
}

static int dinv_from_u(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, double **Dinv)
{
    void *p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    *Dinv = (double *)p;
    TRY(launch_diag_inv(U, ldu, n, *Dinv, ctx->stream));
    return prepare_solves(ctx, n, U, ldu, *Dinv);
}

// The super-block sweeps on U = D (I + W) (W FP64 or FP32): the work-queue
// kernels (default) or one workgroup per tile (gsyeig_set_trsv_sweep).
// KI3 takes b, or (b == nullptr) the SYMV tile partials Pr / Pc.
static bool queue_n(const gsyeig_ctx *ctx) { return ctx->trsv_sweep == 0 || ctx->trsv_sweep == 3; }
static bool queue_t(const gsyeig_ctx *ctx) { return ctx->trsv_sweep == 0 || ctx->trsv_sweep == 2; }

static int sweep_n(gsyeig_ctx *ctx, int64_t n, const void *W, int w_f32, int64_t ldw, const double *sb,
                   const double *b, double *x)
{
    if (queue_n(ctx)) {
        TrsvQ q;
        TRY(trsvq_prepare(ctx, n, &q));
        return w_f32 ? launch_trsvq_n_f32((const float *)W, ldw, n, sb, b, x, ctx->ctl_n, q, ctx->stream)
                     : launch_trsvq_n((const double *)W, ldw, n, sb, b, x, ctx->ctl_n, q, ctx->stream);
    }
    return w_f32 ? launch_trsv_w_n_f32((const float *)W, ldw, n, sb, b, x, ctx->ctl_n, ctx->stream)
                 : launch_trsv_w_n((const double *)W, ldw, n, sb, b, x, ctx->ctl_n, ctx->stream);
}

static int sweep_t(gsyeig_ctx *ctx, int64_t n, const void *W, int w_f32, int64_t ldw, const double *sb,
                   const double *b, const double *Pr, const double *Pc, int maxch, int ch, double *x)
{
    if (queue_t(ctx)) {
        TrsvQ q;
        TRY(trsvq_prepare(ctx, n, &q));
        return w_f32 ? launch_trsvq_t_f32((const float *)W, ldw, n, sb, b, Pr, Pc, maxch, ch, x, ctx->ctl_t, q,
                                          ctx->stream)
                     : launch_trsvq_t((const double *)W, ldw, n, sb, b, Pr, Pc, maxch, ch, x, ctx->ctl_t, q,
                                      ctx->stream);
    }
    if (b) return w_f32 ? launch_trsv_w_t_f32((const float *)W, ldw, n, sb, b, x, ctx->ctl_t, ctx->stream)
                        : launch_trsv_w_t((const double *)W, ldw, n, sb, b, x, ctx->ctl_t, ctx->stream);
    return w_f32 ? launch_trsv_w_t_rows_f32((const float *)W, ldw, n, sb, Pr, Pc, maxch, ch, x, ctx->ctl_t, ctx->stream)
                 : launch_trsv_w_t_rows((const double *)W, ldw, n, sb, Pr, Pc, maxch, ch, x, ctx->ctl_t, ctx->stream);
}

static int solve_n(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, const double *Dinv,
                   const double *b, double *x)
{
    if (ctx->trsv_block == 64)
        return launch_trsv_n(U, ldu, n, Dinv, aux_m(Dinv, n), b, x, ctx->ctl_n, ctx->stream);
    if (b == x) {  // each tile reads b across its super-block: solve from a copy
        void *p;
        TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)n, &p));
        TRY(launch_copy(b, (double *)p, n, ctx->stream));
        b = (const double *)p;
    }
    return sweep_n(ctx, n, ctx->ws[WS_W], 0, round_ld(n), (const double *)ctx->ws[WS_SB], b, x);
}

static int solve_t(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, const double *Dinv,
                   const double *b, double *x)
{
    if (ctx->trsv_block == 64)
        return launch_trsv_t(U, ldu, n, Dinv, aux_m(Dinv, n), b, x, ctx->ctl_t, ctx->stream);
    return sweep_t(ctx, n, ctx->ws[WS_W], 0, round_ld(n), (const double *)ctx->ws[WS_SB], b, nullptr, nullptr, 0, 0,
                   x);
}

// Super-block inverses of an FP64 factor for the block solves: built with
// the factor's side data by the super-block sweeps, else built here.
static int block_sb_fp64(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, const double *Dinv,
                         const double **sb)
{
    void *p;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    if (ctx->trsv_block == 64) {
        const int64_t SB = trsv_sb_rows();
        TRY(launch_sb_inverses(U, ldu, n, Dinv, (double *)p, (double *)p + cdiv(n, SB) * SB * SB, ctx->stream));
    }
    *sb = (const double *)p;
    return 0;
}

// Sampled kernel timing: events recorded around KI1/KI2/KI3 on the stream;
// harvested (elapsed times summed) at the next synchronisation point.
static int prof_harvest(gsyeig_ctx *ctx)
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

// The implicit operator C = U^-T A U^-1 of KI1-KI3: FP64 A and U, or (mixed
// mode) FP32 copies of both with FP64 super-block inverses.
struct LzOp {
    int f32;
    const double *A; int64_t lda;
    const double *U; int64_t ldu;
    const double *Dinv;
    const float *A32; int64_t lda32;
    const float *U32; int64_t ldu32;
    const float *W32; int64_t ldw32;
    const double *sb;   // super-block inverses and link blocks of U~
    const double *C; int64_t ldc;  // variant KE: the explicit C (the operator is one SYMV)
};

static LzOp op_fp64(const double *A, int64_t lda, const double *U, int64_t ldu, const double *Dinv)
{
    LzOp op{};
    op.A = A; op.lda = lda; op.U = U; op.ldu = ldu; op.Dinv = Dinv;
    return op;
}

// KI1-KI3 into z (z may alias w); tmp is an n-vector of scratch.
static int apply_op(gsyeig_ctx *ctx, int64_t n, const LzOp &op, const double *w, double *z, double *tmp,
                    bool sample = false)
{
    sample = sample && ctx->npev + 4 <= 64;
    hipEvent_t *e = ctx->pev + ctx->npev;
    if (sample) HIP_TRY(hipEventRecord(e[0], ctx->stream));
    if (op.C) {  // variant KE: z = C w (KI1 and KI3 are empty in the samples)
        if (sample) HIP_TRY(hipEventRecord(e[1], ctx->stream));
        TRY(launch_symv(ctx, n, op.C, op.ldc, w, w == z ? tmp : z));
        if (w == z) TRY(launch_copy(tmp, z, n, ctx->stream));
        if (sample) {
            HIP_TRY(hipEventRecord(e[2], ctx->stream));
            HIP_TRY(hipEventRecord(e[3], ctx->stream));
            ctx->npev += 4;
        }
        return 0;
    }
    if (op.f32)
        TRY(sweep_n(ctx, n, op.W32, 1, op.ldw32, op.sb, w, tmp));
    else
        TRY(solve_n(ctx, n, op.U, op.ldu, op.Dinv, w, tmp));
    if (sample) HIP_TRY(hipEventRecord(e[1], ctx->stream));
    if (op.f32 || ctx->trsv_block != 64) {
        // KI2's tile pass, then KI3 on U = D (I + W) summing the partials of
        // its own rows (no separate reduction launch)
        double *Pr, *Pc;
        int maxch, ch;
        if (op.f32)
            TRY(launch_symv_partials_f32(ctx, n, op.A32, op.lda32, tmp, &Pr, &Pc, &maxch, &ch));
        else
            TRY(launch_symv_partials(ctx, n, op.A, op.lda, tmp, &Pr, &Pc, &maxch, &ch));
        if (sample) HIP_TRY(hipEventRecord(e[2], ctx->stream));
        if (op.f32)
            TRY(sweep_t(ctx, n, op.W32, 1, op.ldw32, op.sb, nullptr, Pr, Pc, maxch, ch, z));
        else
            TRY(sweep_t(ctx, n, ctx->ws[WS_W], 0, round_ld(n), (const double *)ctx->ws[WS_SB], nullptr, Pr, Pc, maxch,
                        ch, z));
    } else {
        TRY(launch_symv(ctx, n, op.A, op.lda, tmp, z));
        if (sample) HIP_TRY(hipEventRecord(e[2], ctx->stream));
        TRY(solve_t(ctx, n, op.U, op.ldu, op.Dinv, z, z));
    }
    if (sample) {
        HIP_TRY(hipEventRecord(e[3], ctx->stream));
        ctx->npev += 4;
    }
    return 0;
}

static int potrf_core(gsyeig_ctx *ctx, int64_t n, double *B, int64_t ldb, double *Dinv, int *info_d);

// Makes the nw columns of S (m x nw, column-major) orthonormal by Cholesky
// QR applied twice: G = S^T S = R^T R, S <- S R^-1 (FP64 GEMMs on the matrix
// cores, small Cholesky and triangular inverse by the GS1 kernels).  Used
// on inverse-iteration eigenvectors of T_m, whose mutual overlaps are tiny
// except inside clusters of close eigenvalues; there any orthonormal basis
// of the computed vectors is as good.  *info_d != 0 if G was not positive
// definite or if two columns overlapped by more than 0.5 (the caller then
// falls back to sequential Gram-Schmidt with extra inverse-iteration solves).
int orthonormalise_cols(gsyeig_ctx *ctx, int64_t m, int64_t nw, double *S, int64_t lds, int *info_d)
{
    const int64_t nwr = cdiv(nw, NB) * NB;
    const int64_t sk = std::max<int64_t>(1, std::min<int64_t>(32, cdiv(m, 1024)));
    const size_t need = sizeof(double) * ((size_t)nw * nw * 2 + (size_t)nwr * NB + (size_t)m * nw +
                                          (size_t)sk * nw * nw + 64);
    void *p;
    TRY(ws_get(ctx, WS_RITZ, need, &p));
    double *G = (double *)p, *Ri = G + nw * nw, *Dv = Ri + nw * nw, *T = Dv + nwr * NB, *part = T + m * nw;
    HIP_TRY(hipMemsetAsync(info_d, 0, sizeof(int), ctx->stream));
    int *info2 = info_d + 1;
    for (int pass = 0; pass < 2; ++pass) {
        GemmDesc g{};
        g.m = nw; g.n = nw; g.k = m;
        g.A = S; g.lda = lds; g.a_layout = 1;   // A(i, t) = S(t, i)
        g.B = S; g.ldb = lds; g.b_layout = 0;
        g.C = G; g.ldc = nw; g.c_layout = 1;    // symmetric: either layout
        g.alpha = 1.0; g.beta = 0.0;
        g.splitk = (int)sk; g.part = part;
        TRY(launch_gemm(g, ctx->stream));
        // Inverse-iteration vectors (random start per index) overlap by about
        // u ||T|| / gap; inside a tight cluster they are independent mixtures
        // of the cluster's eigenvectors, of which any orthonormal basis is as
        // accurate, and the two passes make them orthonormal.  Only vectors
        // that came out nearly parallel (overlap beyond 0.5) need the
        // sequential treatment (extra solves inside the cluster).
        if (pass == 0) TRY(launch_flag_offdiag(G, nw, 0.5, info_d, ctx->stream));
        TRY(potrf_core(ctx, nw, G, nw, Dv, info2));
        TRY(launch_accum_info(info2, info_d, ctx->stream));
        // Ri = R^-1 (column-major; R is G's upper triangle, row-major)
        TRY(launch_identity(Ri, nw, nw, ctx->stream));
        TRY(launch_backsolve(G, nw, nw, nw, Dv, Ri, nw, ctx->stream));
        GemmDesc u{};
        u.m = m; u.n = nw; u.k = nw;
        u.A = S; u.lda = lds; u.a_layout = 0;
        u.B = Ri; u.ldb = nw; u.b_layout = 0;
        u.C = T; u.ldc = m; u.c_layout = 0;
        u.alpha = 1.0; u.beta = 0.0;
        TRY(launch_gemm(u, ctx->stream));
        TRY(launch_blk_copy(T, m, S, lds, m, nw, ctx->stream));
    }
    return 0;
}

// Ritz coefficients in an orthonormal basis of span(V_m) when V_m is only
// semi-orthogonal (partial re-orthogonalisation): with V_m^T V_m = R^T R,
// W = V_m R^-1 is orthonormal and W^T C W equals T_m up to O(u ||C||)
// (Simon 1984), so the Ritz vectors are W S = V_m (R^-1 S).  Taking V_m S
// instead would leave residuals of up to sqrt(u) ||C||: the Gram-Schmidt
// coefficients of the orthogonalised steps are not part of T_m.  On return
// S holds R^-1 S; *info_d != 0 if V_m^T V_m was not positive definite.
static int semiorth_coeffs(gsyeig_ctx *ctx, int64_t n, int64_t m, const double *V, int64_t ldv, double *S,
                           int64_t nvec, int *info_d)
{
    GemmDesc g{};
    g.m = m; g.n = m; g.k = n;
    g.A = V; g.lda = ldv; g.a_layout = 1;   // A(i, t) = V(t, i)
    g.B = V; g.ldb = ldv; g.b_layout = 0;
    g.c_layout = 1;                         // upper triangle, row-major, as potrf_core reads it
    g.ldc = m;
    g.alpha = 1.0; g.beta = 0.0;
    g.upper_only = 1;
    const int64_t tiles = cdiv(m, 64) * cdiv(m, 64);
    g.splitk = (int)std::max<int64_t>(1, std::min<int64_t>({32, 512 / tiles, cdiv(n, 1024)}));
    const int64_t parts = (g.splitk > 1) ? gemm_splitk_parts(g) : 0;
    const int64_t mr = cdiv(m, NB) * NB;
    void *p;
    TRY(ws_get(ctx, WS_PROG, sizeof(double) * ((size_t)m * m * (1 + parts) + (size_t)mr * NB + 64), &p));
    double *G = (double *)p, *Dv = G + m * m, *part = Dv + mr * NB;
    g.C = G;
    g.part = parts ? part : nullptr;
    if (!parts) g.splitk = 1;
    TRY(launch_gemm(g, ctx->stream));
    TRY(potrf_core(ctx, m, G, m, Dv, info_d));
    return launch_backsolve(G, m, m, nvec, Dv, S, m, ctx->stream);
}

// KI5's vectors once theta holds the nvec wanted Ritz values of T_m: S
// (m x nvec) by inverse iteration, made orthonormal (sequential
// Gram-Schmidt in clusters if Cholesky QR cannot), R^-1 S for a
// semi-orthogonal basis (reorth 2), Y = V_m S, theta_out = theta.
// oinfo_d[2] != 0 afterwards if V_m^T V_m was not positive definite.
static int lz_ritz_vectors(gsyeig_ctx *ctx, int64_t n, int64_t m, int64_t nvec, int reorth, const double *alpha,
                           const double *beta, const double *V, int64_t ldv, const double *theta, double *lastc,
                           double *tri, double *theta_out, double *Y, int64_t ldy, int *oinfo_d)
{
    void *p;
    TRY(ws_get(ctx, WS_S, sizeof(double) * (size_t)m * (size_t)nvec, &p));
    double *S = (double *)p;
    int *h = (int *)ctx->host_pinned + 3;
    TRY(launch_tri_vectors(alpha, beta, m, nvec, theta, S, m, tri, 0, lastc, ctx->stream));
    TRY(orthonormalise_cols(ctx, m, nvec, S, m, oinfo_d));
    HIP_TRY(hipMemcpyAsync(h, oinfo_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (*h != 0) {  // near-parallel vectors or Gram not positive definite: sequential Gram-Schmidt in clusters
        ctx->n_fallback += 1;
        ctx->fallback_why = 1;
        TRY(launch_tri_vectors(alpha, beta, m, nvec, theta, S, m, tri, 1, lastc, ctx->stream));
    }
    if (reorth == 2) TRY(semiorth_coeffs(ctx, n, m, V, ldv, S, nvec, oinfo_d + 2));
    else HIP_TRY(hipMemsetAsync(oinfo_d + 2, 0, sizeof(int), ctx->stream));
    GemmDesc d{};
    d.m = n; d.n = nvec; d.k = m;
    d.A = V; d.lda = ldv; d.a_layout = 0;
    d.B = S; d.ldb = m; d.b_layout = 0;
    d.C = Y; d.ldc = ldy; d.c_layout = 0;
    d.alpha = 1.0; d.beta = 0.0;
    TRY(launch_gemm_f64(d, ctx->stream));
    return launch_copy(theta, theta_out, nvec, ctx->stream);
}

struct LzBufs {
    double *z, *tmp, *red, *red2, *h, *normpart, *z0part;
    int *flag;       // [0] Gram-Schmidt pass needed, [1] count of such steps, [2] next step forced (device)
    int reorth;      // 0: always two passes; 1: second pass when needed; 2: partial (omega estimates)
    double *om;      // reorth 2: three omega vectors of length ldom, and the ||T|| estimate after them
    int64_t ldom;
    double *slots;   // reorth 2: the published partial sums of the fused step (sentinel-initialised)
};

static int lz_bufs(gsyeig_ctx *ctx, int64_t n, int64_t kmax, LzBufs *b)
{
    void *p;
    TRY(ws_get(ctx, WS_TMP1, sizeof(double) * (size_t)n, &p));
    b->z = (double *)p;
    TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)n, &p));
    b->tmp = (double *)p;
    const size_t red = (size_t)lz_red_parts(n) * (size_t)(kmax + 8) + (size_t)lz_norm_parts(n) +
                       (size_t)lz_z0_parts(n) + 1024 + 64;
    TRY(ws_get(ctx, WS_RED, sizeof(double) * red, &p));
    b->red = (double *)p;
    b->normpart = b->red + 1024;
    b->z0part = b->normpart + lz_norm_parts(n);
    b->flag = (int *)(b->z0part + lz_z0_parts(n));
    b->red2 = b->z0part + lz_z0_parts(n) + 64;
    b->reorth = 1;
    b->om = nullptr;
    b->slots = nullptr;
    b->ldom = 0;
    TRY(ws_get(ctx, WS_RED2, sizeof(double) * (size_t)(kmax + 8), &p));
    b->h = (double *)p;
    return 0;
}

// One Lanczos step k (KI1-KI4): w_k = V[:, k] -> w_{k+1} = V[:, k+1].
static int lz_step(gsyeig_ctx *ctx, int64_t n, const LzOp &op, double *V, int64_t ldv, double *alpha,
                   double *beta, int64_t k, const LzBufs &b, bool sample = false)
{
    const double *wk = V + k * ldv;
    const double *wp = (k > 0) ? V + (k - 1) * ldv : wk;
    TRY(apply_op(ctx, n, op, wk, b.z, b.tmp, sample));
    if (b.reorth == 2) {
        // both passes only on the steps where the omega estimates of w_j^T w_{k+1}
        // exceed sqrt(u), and on the step after each of them
        // (two launches: alpha_k, the omega recurrence, beta_k and w_{k+1};
        // the two passes, only on the steps that ask for them)
        double *om_c = b.om + (k % 3) * b.ldom, *om_n = b.om + ((k + 1) % 3) * b.ldom;
        const double *om_p = b.om + ((k + 2) % 3) * b.ldom;
        return launch_lz_post(b.z, wp, wk, V + (k + 1) * ldv, alpha, beta, k, n, V, ldv, om_p, om_c, om_n,
                              b.om + 3 * b.ldom, b.flag, b.slots, b.slots + lz_post_slots(), b.ldom, ctx->ctl_lz,
                              ctx->stream);
    }
    if (b.reorth) {
        // second pass only where the first lost more than 1/sqrt(2) of the norm
        TRY(launch_lz_alpha(b.z, wp, wk, alpha, beta, k, n, b.red, ctx->stream, b.z0part));
        TRY(launch_cgs_pass(V, ldv, n, k + 1, b.z, b.red2, b.h, b.normpart, ctx->stream));
        TRY(launch_reorth_flag(b.z0part, n, b.normpart, b.flag, ctx->stream));
        TRY(launch_cgs_pass(V, ldv, n, k + 1, b.z, b.red2, b.h, b.normpart, ctx->stream, b.flag));
    } else {
        TRY(launch_lz_alpha(b.z, wp, wk, alpha, beta, k, n, b.red, ctx->stream));
        TRY(launch_cgs_pass(V, ldv, n, k + 1, b.z, b.red2, b.h, nullptr, ctx->stream));
        TRY(launch_cgs_pass(V, ldv, n, k + 1, b.z, b.red2, b.h, b.normpart, ctx->stream));
    }
    TRY(launch_lz_normalize(b.z, V + (k + 1) * ldv, beta, k, n, b.normpart, ctx->stream));
    return 0;
}

// KI1-KI5 with convergence checks.  The nvec >= s extreme Ritz pairs are
// extracted (ascending; values -> theta_out, vectors -> Y); the run stops
// when the s wanted ones among them (the first s for which = 0, the last s
// for which = 1) meet tol.
struct LzResult {
    int64_t steps;
    int64_t nconv;
    int64_t reorth_steps;
    float t_loop_ms, t_ritz_ms;
};

static int lz_solve_body(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t nvec, const LzOp &op,
                         const gsyeig_opts *o, double *theta_out, double *Y, int64_t ldy, LzResult *res)
{
    const int64_t mmax = std::max<int64_t>(eff_max_steps(n, s, o), std::min<int64_t>(nvec, n));
    const int64_t w0 = o->which ? nvec - s : 0;
    const int64_t ldv = round_ld(n);
    void *p;
    TRY(ws_get(ctx, WS_V, sizeof(double) * (size_t)ldv * (size_t)(mmax + 1), &p));
    double *V = (double *)p;
    // T: alpha (mmax), beta (mmax), theta (nvec+1), lastcomp (nvec), pre-check (2 x 32)
    TRY(ws_get(ctx, WS_T, sizeof(double) * (size_t)(2 * mmax + 2 * nvec + 16 + 64), &p));
    double *alpha = (double *)p, *beta = alpha + mmax, *theta = beta + mmax, *lastc = theta + nvec + 1;
    double *theta_q = lastc + nvec + 8, *lastc_q = theta_q + 32;
    // pre-check: the q innermost wanted Ritz values converge last; only when
    // they all meet tol is the full set of s checked
    const int64_t q = std::min<int64_t>(s, 16);
    TRY(ws_get(ctx, WS_TRI, sizeof(double) * (size_t)nvec * 7 * (size_t)mmax, &p));
    double *tri = (double *)p;
    LzBufs b;
    TRY(lz_bufs(ctx, n, mmax, &b));
    b.reorth = (int)o->reorth;
    if (b.reorth == 2) {
        b.ldom = mmax + 8;
        const size_t sent = (size_t)lz_post_slots() + (size_t)lz_cgs_doubles(n, b.ldom);
        TRY(ws_get(ctx, WS_PRO, sizeof(double) * ((size_t)(3 * b.ldom + 8) + sent), &p));
        b.om = (double *)p;
        b.slots = b.om + 3 * b.ldom + 8;
        TRY(launch_pro_init(b.om, b.om + 3 * b.ldom, b.flag, ctx->stream));
        HIP_TRY(hipMemsetAsync(b.slots, 0xFF, sizeof(double) * sent, ctx->stream));
    } else {
        HIP_TRY(hipMemsetAsync(b.flag, 0, 4 * sizeof(int), ctx->stream));
    }
    TRY(ctl_reserve(ctx, n));
    int *nconv_d = (int *)ctx->dscal;
    int *nconv_h = (int *)ctx->host_pinned;

    HIP_TRY(hipEventRecord(ctx->ev[6], ctx->stream));
    // w_0
    if (o->v0) {
        TRY(launch_normalize_into(o->v0, V, n, b.red, nullptr, ctx->stream));
    } else {
        TRY(launch_fill_splitmix(b.z, n, o->seed, ctx->stream));
        TRY(launch_normalize_into(b.z, V, n, b.red, nullptr, ctx->stream));
    }
    const int64_t every = std::max<int64_t>(1, o->check_every);
    int64_t m = 0, nconv = 0;
    bool checked_at_m = false;
    // check schedule: every `every` steps near convergence; further apart
    // (up to 4x) while the slowest innermost wanted pair is predicted to
    // need many more steps (its residual ratio extrapolated linearly in
    // log scale from the last two pre-checks)
    int64_t next_check = every;
    int64_t prev_m = -1;
    double prev_rho = 0.0;
    double *ratio_d = (double *)ctx->dscal + 32;
    ctx->npev = 0;
    ctx->prof_samples = 0;
    ctx->prof_ms[0] = ctx->prof_ms[1] = ctx->prof_ms[2] = 0.0;
    const int64_t pe = o->profile_every;
    for (int64_t k = 0; k < mmax; ++k) {
        const bool sample = pe > 0 && (k % pe) == pe - 1;
        TRY(lz_step(ctx, n, op, V, ldv, alpha, beta, k, b, sample));
        m = k + 1;
        checked_at_m = false;
        if (m >= nvec && (m >= next_check || m == mmax)) {
            next_check = m + every;
            if (m < mmax) {
                const int64_t qq = std::min<int64_t>(q, s);
                const int64_t first = o->which ? m - s : s - qq;
                TRY(launch_tri_bisect_range(alpha, beta, m, first, qq, o->which, theta_q, ctx->stream));
                TRY(launch_tri_vectors(alpha, beta, m, qq, theta_q, nullptr, 0, tri, 0, lastc_q, ctx->stream));
                TRY(launch_conv_count(theta_q, lastc_q, beta + (m - 1), qq, 0, qq, 1, o->tol, nconv_d, ctx->stream,
                                      ratio_d));
                HIP_TRY(hipMemcpyAsync(nconv_h, nconv_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
                HIP_TRY(hipMemcpyAsync((double *)ctx->host_pinned + 8, ratio_d, sizeof(double),
                                       hipMemcpyDeviceToHost, ctx->stream));
                HIP_TRY(hipStreamSynchronize(ctx->stream));
                TRY(prof_harvest(ctx));
                const double ratio = ((double *)ctx->host_pinned)[8];
                if (*nconv_h < qq) {
                    const double rho = log10(std::max(ratio, 1.0));
                    int64_t interval = 2 * every;
                    if (prev_m >= 0 && prev_rho > rho) {
                        const double remaining = rho * (double)(m - prev_m) / (prev_rho - rho);
                        interval = std::min<int64_t>(4 * every, std::max<int64_t>(every, (int64_t)(0.6 * remaining)));
                    }
                    prev_m = m;
                    prev_rho = rho;
                    next_check = m + interval;
                    continue;
                }
                if (qq == s) {  // the pre-check covered every wanted pair
                    nconv = s;
                    checked_at_m = false;
                    break;
                }
            }
            TRY(launch_tri_bisect(alpha, beta, m, nvec, o->which, theta, ctx->stream));
            TRY(launch_tri_vectors(alpha, beta, m, nvec, theta, nullptr, 0, tri, 0, lastc, ctx->stream));
            TRY(launch_conv_count(theta, lastc, beta + (m - 1), nvec, w0, s, 0, o->tol, nconv_d, ctx->stream));
            HIP_TRY(hipMemcpyAsync(nconv_h, nconv_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
            HIP_TRY(hipStreamSynchronize(ctx->stream));
            TRY(prof_harvest(ctx));
            nconv = *nconv_h;
            checked_at_m = true;
            if (nconv >= s) break;
        }
    }
    if (!checked_at_m) {
        TRY(launch_tri_bisect(alpha, beta, m, nvec, o->which, theta, ctx->stream));
    }
    HIP_TRY(hipEventRecord(ctx->ev[7], ctx->stream));
    int *oinfo_d = (int *)ctx->dscal + 24;
    TRY(lz_ritz_vectors(ctx, n, m, nvec, b.reorth, alpha, beta, V, ldv, theta, lastc, tri, theta_out, Y, ldy,
                        oinfo_d));
    HIP_TRY(hipMemcpyAsync(nconv_h + 1, b.flag + 1, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(nconv_h + 2, oinfo_d + 2, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[5], ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    res->reorth_steps = (b.reorth == 0) ? m : nconv_h[1];
    TRY(prof_harvest(ctx));
    HIP_TRY(hipEventElapsedTime(&res->t_loop_ms, ctx->ev[6], ctx->ev[7]));
    HIP_TRY(hipEventElapsedTime(&res->t_ritz_ms, ctx->ev[7], ctx->ev[5]));
    res->steps = m;
    res->nconv = nconv;
    if (b.reorth == 2 && nconv_h[2] != 0) {  // basis lost semi-orthogonality: the Ritz vectors are not valid
        res->nconv = 0;
        return GSYEIG_ENOCONV;
    }
    return 0;
}

// lz_solve_body with the chained sweeps' wait record: cleared before the
// first sweep, read on every exit, so that an expired wait is reported
// (GSYEIG_ESPIN, ahead of GSYEIG_ENOCONV) by the call whose kernels it hit.
static int lz_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t nvec, const LzOp &op,
                    const gsyeig_opts *o, double *theta_out, double *Y, int64_t ldy, LzResult *res)
{
    TRY(ctl_reserve(ctx, n));
    TRY(ctl_clear_err(ctx));
    const int rc = lz_solve_body(ctx, n, s, nvec, op, o, theta_out, Y, ldy, res);
    const int crc = ctl_check(ctx);
    if (crc == GSYEIG_ESPIN && (rc == 0 || rc == GSYEIG_ENOCONV)) return GSYEIG_ESPIN;
    return rc ? rc : crc;
}

// Blocked right-looking Cholesky B = U^T U of the upper triangle in place
// (FP64), diagonal-block inverses into Dinv (cdiv(n, 64) blocks of 64x64).
static int potrf_core(gsyeig_ctx *ctx, int64_t n, double *B, int64_t ldb, double *Dinv, int *info_d)
{
    HIP_TRY(hipMemsetAsync(info_d, 0, sizeof(int), ctx->stream));
    const int64_t nblk = cdiv(n, NB);
    for (int64_t kb = 0; kb < nblk; ++kb) {
        TRY(launch_potrf_diag(B, ldb, n, kb, Dinv, info_d, ctx->stream));
        const int64_t r0 = kb * NB;
        const int64_t r = std::min<int64_t>(NB, n - r0);
        const int64_t c0 = r0 + r;
        const int64_t m2 = n - c0;
        if (m2 <= 0) break;
        // panel: U_{k, >k} = U_kk^-T B_{k, >k}   (Dinv_kk^T times the row panel)
        GemmDesc pd{};
        pd.m = r; pd.n = m2; pd.k = r;
        pd.A = Dinv + kb * NB * NB; pd.lda = NB; pd.a_layout = 0;   // A(i,k) = Dinv[k][i]
        pd.B = B + r0 * ldb + c0; pd.ldb = ldb; pd.b_layout = 1;
        pd.C = B + r0 * ldb + c0; pd.ldc = ldb; pd.c_layout = 1;
        pd.alpha = 1.0; pd.beta = 0.0;
        TRY(launch_gemm_f64(pd, ctx->stream));
        // trailing update of the upper triangle, B_>k,>k -= P^T P, in two
        // levels: the rows of this outer block of POTRF_OUTER rows at once
        // (the next diagonal blocks need them), the rows below it by one
        // rank-POTRF_OUTER product when the outer block is done -- the
        // trailing matrix is then read and written once per POTRF_OUTER
        // columns instead of once per 64
        const int64_t K0 = (r0 / POTRF_OUTER) * POTRF_OUTER;
        const int64_t Kend = std::min<int64_t>(n, K0 + POTRF_OUTER);
        if (Kend > c0) {
            GemmDesc sd{};
            sd.m = Kend - c0; sd.n = m2; sd.k = r;
            sd.A = B + r0 * ldb + c0; sd.lda = ldb; sd.a_layout = 0;    // A(i,k) = P[k][i]
            sd.B = B + r0 * ldb + c0; sd.ldb = ldb; sd.b_layout = 1;    // B(k,j) = P[k][j]
            sd.C = B + c0 * ldb + c0; sd.ldc = ldb; sd.c_layout = 1;
            sd.alpha = -1.0; sd.beta = 1.0;
            sd.upper_only = 1;
            TRY(launch_gemm_f64(sd, ctx->stream));
        } else if (n > Kend) {
            GemmDesc bd{};
            bd.m = n - Kend; bd.n = n - Kend; bd.k = Kend - K0;
            bd.A = B + K0 * ldb + Kend; bd.lda = ldb; bd.a_layout = 0;
            bd.B = B + K0 * ldb + Kend; bd.ldb = ldb; bd.b_layout = 1;
            bd.C = B + Kend * ldb + Kend; bd.ldc = ldb; bd.c_layout = 1;
            bd.alpha = -1.0; bd.beta = 1.0;
            bd.upper_only = 1;
            TRY(launch_gemm_f64(bd, ctx->stream));
        }
    }
    return 0;
}

// GS1: B = U^T U in place (upper triangle), Dinv blocks into WS_DINV.
static int potrf_enqueue(gsyeig_ctx *ctx, int64_t n, double *B, int64_t ldb, double **Dinv_out,
                         int *info_d)
{
    void *p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    *Dinv_out = Dinv;
    TRY(potrf_core(ctx, n, B, ldb, Dinv, info_d));
    return prepare_solves(ctx, n, B, ldb, Dinv);
}

// GS1 in mixed precision: W = fl32(upper(B)) (B untouched), 64x64 diagonal
// blocks factored in FP64, panel and trailing SYRK as FP32 MFMA products
// with FP32 accumulation on the FP32 matrix; U~ (FP32) is left in W's upper
// triangle with zeros below.  Dinv then holds the FP64 inverses of the
// stored FP32 diagonal blocks.
static int potrf_mixed_enqueue(gsyeig_ctx *ctx, int64_t n, const double *B, int64_t ldb, float *W,
                               int64_t ldw, double *Dinv, int *info_d)
{
    HIP_TRY(hipMemsetAsync(info_d, 0, sizeof(int), ctx->stream));
    TRY(launch_upper_to_f32(B, ldb, W, ldw, n, ctx->stream));
    const int64_t nblk = cdiv(n, NB);
    for (int64_t kb = 0; kb < nblk; ++kb) {
        TRY(launch_potrf_diag_f32(W, ldw, n, kb, Dinv, info_d, ctx->stream));
        const int64_t r0 = kb * NB;
        const int64_t r = std::min<int64_t>(NB, n - r0);
        const int64_t c0 = r0 + r;
        const int64_t m2 = n - c0;
        if (m2 <= 0) break;
        GemmDesc pd{};
        pd.m = r; pd.n = m2; pd.k = r;
        pd.A = Dinv + kb * NB * NB; pd.lda = NB; pd.a_layout = 0;
        pd.B = W + r0 * ldw + c0; pd.ldb = ldw; pd.b_layout = 1; pd.b_f32 = 1;
        pd.C = W + r0 * ldw + c0; pd.ldc = ldw; pd.c_layout = 1; pd.c_f32 = 1;
        pd.alpha = 1.0; pd.beta = 0.0;
        pd.f32 = 1;
        TRY(launch_gemm(pd, ctx->stream));
        // two-level trailing update as in potrf_core
        const int64_t K0 = (r0 / POTRF_OUTER) * POTRF_OUTER;
        const int64_t Kend = std::min<int64_t>(n, K0 + POTRF_OUTER);
        GemmDesc sd{};
        if (Kend > c0) {
            sd.m = Kend - c0; sd.n = m2; sd.k = r;
            sd.A = W + r0 * ldw + c0; sd.B = W + r0 * ldw + c0; sd.C = W + c0 * ldw + c0;
        } else if (n > Kend) {
            sd.m = n - Kend; sd.n = n - Kend; sd.k = Kend - K0;
            sd.A = W + K0 * ldw + Kend; sd.B = W + K0 * ldw + Kend; sd.C = W + Kend * ldw + Kend;
        } else {
            continue;
        }
        sd.lda = ldw; sd.a_layout = 0; sd.a_f32 = 1;
        sd.ldb = ldw; sd.b_layout = 1; sd.b_f32 = 1;
        sd.ldc = ldw; sd.c_layout = 1; sd.c_f32 = 1;
        sd.alpha = -1.0; sd.beta = 1.0;
        sd.upper_only = 1;
        sd.f32 = 1;
        TRY(launch_gemm(sd, ctx->stream));
    }
    return launch_diag_inv_f32(W, ldw, n, Dinv, ctx->stream);
}

static int check_enqueue(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda,
                         const double *B, int64_t ldb, const double *Bdiag, const double *Lambda,
                         const double *X, int64_t ldx, double *res_d)
{
    const int64_t ldr = round_ld(n);
    void *p;
    TRY(ws_get(ctx, WS_Y, sizeof(double) * (size_t)ldr * (size_t)s, &p));
    double *AX = (double *)p;
    TRY(ws_get(ctx, WS_Y2, sizeof(double) * (size_t)ldr * (size_t)s, &p));
    double *BX = (double *)p;
    const int PA = fro_parts(n);
    TRY(ws_get(ctx, WS_S, sizeof(double) * (size_t)(s * s + 2 * s + 2 * PA + 64), &p));
    double *G = (double *)p, *cols = G + s * s, *partA = cols + 2 * s, *partB = partA + PA;
    GemmDesc d{};
    d.m = n; d.n = s; d.k = n;
    d.A = A; d.lda = lda; d.a_layout = 1;
    d.B = X; d.ldb = ldx; d.b_layout = 0;
    d.C = AX; d.ldc = ldr; d.c_layout = 0;
    d.alpha = 1.0; d.beta = 0.0;
    TRY(launch_gemm_f64(d, ctx->stream));
    d.A = B; d.lda = ldb; d.a_layout = Bdiag ? 2 : 1; d.a_diag = Bdiag;
    d.C = BX;
    TRY(launch_gemm_f64(d, ctx->stream));
    GemmDesc g{};
    g.m = s; g.n = s; g.k = n;
    g.A = X; g.lda = ldx; g.a_layout = 1;   // A(i,k) = X^T(i,k) = X[i*ldx + k]
    g.B = BX; g.ldb = ldr; g.b_layout = 0;
    g.C = G; g.ldc = s; g.c_layout = 0;
    g.alpha = 1.0; g.beta = 0.0;
    TRY(launch_gemm_f64(g, ctx->stream));
    TRY(launch_check_cols(AX, BX, ldr, X, ldx, n, s, Lambda, cols, ctx->stream));
    TRY(launch_fro_norm_parts(A, lda, n, 0, nullptr, partA, ctx->stream));
    TRY(launch_fro_norm_parts(B, ldb, n, Bdiag ? 2 : 0, Bdiag, partB, ctx->stream));
    TRY(launch_check_finalize(cols, s, G, s, partA, PA, partB, PA, Lambda, res_d, ctx->stream));
    return 0;
}

// FP32 operator data for a factor U~ (FP32): A~ = fl32(A), the FP64 inverses
// of U~'s diagonal blocks and its super-block inverses.
static int mixed_operator(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const float *U32,
                          int64_t ldu32, bool have_dinv, LzOp *op, bool need_w = true)
{
    const int64_t ld32 = round_ld(n);
    void *p;
    TRY(ws_get(ctx, WS_A32, sizeof(float) * (size_t)ld32 * (size_t)n, &p));
    float *A32 = (float *)p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    double *sb = (double *)p;
    float *W32 = nullptr;
    TRY(launch_to_f32(A, lda, A32, ld32, n, n, ctx->stream));
    if (!have_dinv) TRY(launch_diag_inv_f32(U32, ldu32, n, Dinv, ctx->stream));
    if (need_w) {
        TRY(ws_get(ctx, WS_W, sizeof(float) * (size_t)ld32 * (size_t)n, &p));
        W32 = (float *)p;
        TRY(launch_make_w_f32(U32, ldu32, n, Dinv, sb, W32, ld32, ctx->stream));
    } else {  // block solves need only the super-block inverses
        const int64_t SB = trsv_sb_rows();
        TRY(launch_sb_inverses_f32(U32, ldu32, n, Dinv, sb, sb + cdiv(n, SB) * SB * SB, ctx->stream));
    }
    *op = LzOp{};
    op->f32 = 1;
    op->Dinv = Dinv;
    op->A32 = A32; op->lda32 = ld32;
    op->U32 = U32; op->ldu32 = ldu32;
    op->W32 = W32; op->ldw32 = ld32;
    op->sb = sb;
    return 0;
}

// Mixed mode after the Lanczos phase (k = s + guard Ritz vectors in Y):
// X0 = U~^-1 Y, the FP64 refinement on (A, B), the FP64 check.  Fills inf
// except t_gs1_ms and t_total_ms; 0, GSYEIG_ENOCONV, or an error.
static int mixed_finish(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t k, const double *A, int64_t lda,
                        const double *B, int64_t ldb, const gsyeig_opts &o, const float *U32, int64_t ld32,
                        const double *Dinv, const double *sb, const float *A32, double *Y, int64_t ldy,
                        const LzResult &r, const BlzResult &br, double *Lambda, double *X, int64_t ldx,
                        gsyeig_info &inf)
{
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    TRY(launch_backsolve_f32(U32, ld32, n, k, Dinv, Y, ldy, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[3], ctx->stream));
    RefineOp rop{U32, ld32, sb, A32, ld32};
    RefineCfg cfg{o.eta_tol, o.refine_iters, o.refine_inner};
    RefineStats rs{};
    TRY(refine_run(ctx, n, s, k, o.which, A, lda, B, ldb, rop, cfg, Lambda, X, ldx, &rs));
    TRY(launch_sign_normalise(X, ldx, n, s, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[4], ctx->stream));
    double *res_d = (double *)ctx->dscal + 64;
    TRY(check_enqueue(ctx, n, s, A, lda, B, ldb, nullptr, Lambda, X, ldx, res_d));
    HIP_TRY(hipEventRecord(ctx->ev[5], ctx->stream));
    double *h = (double *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, res_d, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    inf.eta_max = h[0];
    inf.rho_f = h[1];
    inf.omega = h[2];
    inf.normA_f = h[3];
    inf.normB_f = h[4];
    float t;
    inf.t_ki_ms = r.t_loop_ms;
    inf.t_ki5_ms = r.t_ritz_ms;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3])); inf.t_bt1_ms = t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[3], ctx->ev[4])); inf.t_refine_ms = t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[4], ctx->ev[5])); inf.t_check_ms = t;
    inf.steps = r.steps;
    inf.converged = (r.nconv >= s) ? rs.nconv : std::min<int64_t>(r.nconv, rs.nconv);
    inf.prof_samples = ctx->prof_samples;
    inf.t_ki1_ms_sum = ctx->prof_ms[0];
    inf.t_ki2_ms_sum = ctx->prof_ms[1];
    inf.t_ki3_ms_sum = ctx->prof_ms[2];
    inf.eta_phase1 = rs.eta0;
    inf.refine_iters = rs.iters;
    inf.block_applies = rs.block_applies;
    inf.block_cols = rs.kept;
    inf.restarts = br.restarts;
    inf.basis = br.basis;
    inf.kept = br.keep;
    inf.t_rr_ms = br.t_rr_ms;
    inf.rr_count = br.rr_count;
    inf.reorth_steps = r.reorth_steps;
    return (r.nconv >= s && rs.eta <= o.eta_tol) ? 0 : GSYEIG_ENOCONV;
}

// Mixed mode of gsyeig_solve: GS1 with FP32 trailing updates, Lanczos with
// FP32 sweeps (FP64 vectors, alpha/beta, CGS2, T), Ritz vectors for s +
// guard pairs, X0 = U~^-1 Y, FP64 refinement on (A, B), FP64 check.  B is
// not modified.
static int solve_mixed(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, const double *B,
                       int64_t ldb, const gsyeig_opts &o, double *Lambda, double *X, int64_t ldx,
                       gsyeig_info *info)
{
    const int64_t k = mixed_block(n, s, &o);
    if (k < s) return -3;
    const int64_t ld32 = round_ld(n);
    void *p;
    TRY(ws_get(ctx, WS_U32, sizeof(float) * (size_t)ld32 * (size_t)n, &p));
    float *U32 = (float *)p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    int *info_d = (int *)ctx->dscal + 16;
    gsyeig_info inf;
    memset(&inf, 0, sizeof(inf));
    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    TRY(potrf_mixed_enqueue(ctx, n, B, ldb, U32, ld32, Dinv, info_d));
    LzOp op;
    TRY(mixed_operator(ctx, n, A, lda, U32, ld32, true, &op));
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    int *hi = (int *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(hi, info_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (hi[0] != 0) return hi[0];

    double *Y;
    int64_t ldy;
    TRY(refine_x0(ctx, n, k, &Y, &ldy));
    TRY(ws_get(ctx, WS_BDIAG, sizeof(double) * (size_t)(n + 8), &p));
    double *theta_k = (double *)p;
    LzResult r{};
    BlzResult br{};
    if (o.block > 1) {
        BlkOp bop{U32, 1, ld32, op.W32, 1, op.ldw32, op.sb, op.A32, 1, ld32, o.block_acc32 ? 1 : 0};
        TRY(blz_solve(ctx, n, s, k, bop, &o, theta_k, Y, ldy, &br));
        r.steps = br.steps;
        r.nconv = br.nconv;
        r.t_loop_ms = br.t_loop_ms;
        r.t_ritz_ms = br.t_ritz_ms;
    } else {
        const int lrc = lz_solve(ctx, n, s, k, op, &o, theta_k, Y, ldy, &r);
        if (lrc && lrc != GSYEIG_ENOCONV) return lrc;
        if (lrc == GSYEIG_ENOCONV) {  // no valid Ritz vectors to refine: report the Lanczos phase
            float t;
            HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1])); inf.t_gs1_ms = t;
            inf.t_ki_ms = r.t_loop_ms;
            inf.t_ki5_ms = r.t_ritz_ms;
            inf.steps = r.steps;
            inf.converged = 0;
            inf.reorth_steps = r.reorth_steps;
            inf.eta_max = inf.eta_phase1 = HUGE_VAL;
            if (info) *info = inf;
            return GSYEIG_ENOCONV;
        }
    }
    float t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
    inf.t_gs1_ms = t;
    const int rc = mixed_finish(ctx, n, s, k, A, lda, B, ldb, o, U32, ld32, Dinv, op.sb, op.A32, Y, ldy, r, br,
                                Lambda, X, ldx, inf);
    if (rc && rc != GSYEIG_ENOCONV) return rc;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[5]));
    inf.t_total_ms = t;
    if (info) *info = inf;
    return rc;
}

// FP64 mode after the Lanczos phase (the s Ritz vectors Y in X): X = U^-1 Y,
// the sign convention, the FP64 check (bdiag: B's diagonal before the
// factorisation overwrote it).  Fills inf except t_gs1_ms, t_gs2_ms and
// t_total_ms.
static int fp64_finish(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, const double *B,
                       int64_t ldb, const double *bdiag, const double *Dinv, double *Lambda, double *X, int64_t ldx,
                       const LzResult &r, const BlzResult &br, gsyeig_info &inf)
{
    HIP_TRY(hipEventRecord(ctx->ev[2], ctx->stream));
    TRY(launch_backsolve(B, ldb, n, s, Dinv, X, ldx, ctx->stream));
    TRY(launch_sign_normalise(X, ldx, n, s, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[3], ctx->stream));
    double *res_d = (double *)ctx->dscal + 64;
    TRY(check_enqueue(ctx, n, s, A, lda, B, ldb, bdiag, Lambda, X, ldx, res_d));
    HIP_TRY(hipEventRecord(ctx->ev[4], ctx->stream));
    double *h = (double *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, res_d, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    inf.eta_max = h[0];
    inf.rho_f = h[1];
    inf.omega = h[2];
    inf.normA_f = h[3];
    inf.normB_f = h[4];
    float t;
    inf.t_ki_ms = r.t_loop_ms;
    inf.t_ki5_ms = r.t_ritz_ms;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[2], ctx->ev[3])); inf.t_bt1_ms = t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[3], ctx->ev[4])); inf.t_check_ms = t;
    inf.steps = r.steps;
    inf.converged = r.nconv;
    inf.prof_samples = ctx->prof_samples;
    inf.t_ki1_ms_sum = ctx->prof_ms[0];
    inf.t_ki2_ms_sum = ctx->prof_ms[1];
    inf.t_ki3_ms_sum = ctx->prof_ms[2];
    inf.restarts = br.restarts;
    inf.basis = br.basis;
    inf.kept = br.keep;
    inf.t_rr_ms = br.t_rr_ms;
    inf.rr_count = br.rr_count;
    inf.reorth_steps = r.reorth_steps;
    inf.cluster_fallbacks = ctx->n_fallback;
    inf.fallback_reason = ctx->fallback_why;
    return 0;
}

extern "C" int gsyeig_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, double *B,
                            int64_t ldb, const gsyeig_opts *opts, double *Lambda, double *X, int64_t ldx,
                            gsyeig_info *info);

// The inverse pencil (Sec. 3.1 used it for the MD problem): with A SPD the
// s smallest eigenvalues of (A, B) are the reciprocals of the s largest of
// (B, A), which Lanczos finds quickly.  The pencil (B, A) is solved by the
// same path (in FP64 mode A is factored from a copy, so A and B are left as
// they are), then lambda = 1/mu, the order is reversed and x is rescaled
// from x^T A x = 1 to x^T B x = 1; the FP64 check runs on (A, B).
static int solve_inverted(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, double *B,
                          int64_t ldb, const gsyeig_opts &o, double *Lambda, double *X, int64_t ldx,
                          gsyeig_info *info)
{
    gsyeig_opts oi = o;
    oi.invert = 0;
    oi.which = 1 - o.which;
    const int64_t ldw = round_ld(n);
    void *p;
    double *Af = const_cast<double *>(A);
    int64_t ldf = lda;
    if (o.prec == GSYEIG_FP64) {  // the factor overwrites its matrix: work on a copy of A
        TRY(ws_get(ctx, WS_ACOPY, sizeof(double) * (size_t)ldw * (size_t)n, &p));
        Af = (double *)p;
        ldf = ldw;
        TRY(launch_blk_copy(A, lda, Af, ldf, n, n, ctx->stream));
    }
    TRY(ws_get(ctx, WS_INV, sizeof(double) * ((size_t)ldw * (size_t)s + (size_t)s + 64), &p));
    double *Xi = (double *)p, *mu = Xi + ldw * s;
    gsyeig_info inf;
    memset(&inf, 0, sizeof(inf));
    const int rc = gsyeig_solve(ctx, n, s, B, ldb, Af, ldf, &oi, mu, Xi, ldw, &inf);
    if (rc != 0 && rc != GSYEIG_ENOCONV) return rc;
    HIP_TRY(hipEventRecord(ctx->ev[4], ctx->stream));
    // FP64 Rayleigh-Ritz of (A, B) on span(X): the inverted pairs are only as
    // B-orthogonal as they are accurate (residual / gap); projecting the
    // original pencil makes X^T B X = I to rounding and can only improve the
    // pairs.  No correction rounds (the operator is not used).
    double *X0;
    int64_t ld0;
    TRY(refine_x0(ctx, n, s, &X0, &ld0));
    TRY(launch_invert_pairs(mu, Xi, ldw, Lambda, X0, ld0, n, s, ctx->stream));
    RefineOp nop{};
    RefineCfg rcfg{o.eta_tol, 0, 0};
    RefineStats rrs{};
    TRY(refine_run(ctx, n, s, s, 0, A, lda, B, ldb, nop, rcfg, Lambda, X, ldx, &rrs));
    TRY(launch_sign_normalise(X, ldx, n, s, ctx->stream));
    double *res_d = (double *)ctx->dscal + 64;
    TRY(check_enqueue(ctx, n, s, A, lda, B, ldb, nullptr, Lambda, X, ldx, res_d));
    HIP_TRY(hipEventRecord(ctx->ev[5], ctx->stream));
    double *h = (double *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, res_d, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    inf.eta_max = h[0];
    inf.rho_f = h[1];
    inf.omega = h[2];
    inf.normA_f = h[3];
    inf.normB_f = h[4];
    float t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[4], ctx->ev[5]));
    inf.t_check_ms += t;
    inf.t_total_ms += t;
    if (info) *info = inf;
    return rc;
}

// ------------------------------------------------------------------ C ABI
// ------------------------------------------------------------------ batch
// Worker contexts of the batched solves (own streams), created once and
// kept by the parent context.
static int ensure_workers(gsyeig_ctx *ctx, int64_t nstreams)
{
    while (ctx->nworkers < nstreams) {
        hipStream_t st;
        HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        gsyeig_ctx *w = nullptr;
        int rc = gsyeig_create(&w, st);
        if (rc) {
            (void)hipStreamDestroy(st);
            return rc;
        }
        ctx->wstreams[ctx->nworkers] = st;
        ctx->workers[ctx->nworkers++] = w;
    }
    return 0;
}

// f(worker, k) for k < count on nstreams host threads, each driving one
// worker context; items are taken in order.  Returns the first nonzero f
// result (the remaining items still run).
template <typename F>
static int run_workers(gsyeig_ctx *ctx, int64_t nstreams, int64_t count, F f)
{
    std::atomic<int64_t> next(0);
    std::atomic<int> err(0);
    auto work = [&](int wi) {
        gsyeig_ctx *w = ctx->workers[wi];
        w->trsv_block = ctx->trsv_block;
        w->trsv_sweep = ctx->trsv_sweep;
        if (hipSetDevice(ctx->device) != hipSuccess) {
            int z = 0;
            err.compare_exchange_strong(z, GSYEIG_EHIP);
            return;
        }
        for (;;) {
            const int64_t k = next.fetch_add(1);
            if (k >= count) break;
            const int rc = f(w, k);
            if (rc) {
                int z = 0;
                err.compare_exchange_strong(z, rc);
            }
        }
    };
    const int nt = (int)std::min<int64_t>(nstreams, count);
    std::vector<std::thread> th;
    for (int wi = 0; wi < nt; ++wi) th.emplace_back(work, wi);
    for (auto &t : th) t.join();
    return err.load();
}

static bool batch_lz_eligible(int64_t n, int64_t s, int64_t lda, int64_t ldb, int64_t ldx, const gsyeig_opts &o)
{
    if (n < 1 || n > LZB_NMAX || s < 1 || s > n || lda < n || ldb < n || ldx < n) return false;
    if (o.block != 1 || o.invert || o.variant != GSYEIG_KI || o.reorth != 2 || o.v0) return false;
    if (o.prec != GSYEIG_FP64 && o.prec != GSYEIG_MIXED) return false;
    return o.prec == GSYEIG_FP64 || mixed_block(n, s, &o) >= s;
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Row stride of the batch pool's matrices: whole 64-element blocks, moved
// off multiples of 512 elements, whose rows would all start in the same
// HBM channel (the kernel reads eight rows of a column group at once).
static int64_t batch_ld(int64_t n)
{
    const int64_t ld = round_ld(n);
    return (ld % 512 == 0) ? ld + 64 : ld;
}

// The batched Lanczos kernel reads rows with 16-byte buffer loads that may
// run past column n - 1 into the row's padding, through a resource whose
// extent (n rows of ld elements) stays below 2^31 bytes: a caller's FP64
// matrix is read in place when its base is 16-byte aligned, rows are an even
// number of doubles (not a multiple of 512), n is even and the extent fits;
// otherwise from a copy.
static bool aligned16(const double *p, int64_t ld, int64_t n)
{
    return ((uintptr_t)p % 16 == 0) && (ld % 2 == 0) && (ld % 512 != 0) && (n % 2 == 0) &&
           n * ld * (int64_t)sizeof(double) < ((int64_t)1 << 31);
}

// One instance's device data in the batch pool.
struct BatchInst {
    int64_t i;                   // index in the caller's arrays
    int64_t nvec, mmax, ldv, ldom, ld32;
    double *Dinv;                // inverses of the factor's 64 x 64 diagonal blocks
    float *U32, *A32;            // mixed: FP32 factor and A
    double *sb;                  // mixed: super-block inverses of U~ (refinement)
    double *bdiag;               // FP64: B's diagonal before the factorisation
    double *Ucp, *Acp;           // FP64: 16-byte aligned copies of U and A (if theirs are not)
    double *V, *alpha, *beta, *om, *chk;
    float t_gs1_ms;
    int gs1;                     // 0, or the leading minor of B that is not positive definite
};

// An instance whose one-launch Lanczos phase gave no valid Ritz pairs
// (its basis lost orthogonality, or it reached the step cap) is solved again
// by the per-instance path on worker w: mixed mode from (A, B) as
// gsyeig_solve does (B is untouched); FP64 mode from the factor already in
// B and Dinv (B was overwritten by it).  Returns the instance's code.
static int batch_resolve(gsyeig_ctx *w, int64_t n, int64_t s, const double *A, int64_t lda, double *B,
                         int64_t ldb, const gsyeig_opts &o, double *Dinv, const double *bdiag, double *Lambda,
                         double *X, int64_t ldx, gsyeig_info &inf)
{
    memset(&inf, 0, sizeof(inf));
    if (o.prec == GSYEIG_MIXED) return gsyeig_solve(w, n, s, A, lda, B, ldb, &o, Lambda, X, ldx, &inf);
    w->n_fallback = w->fallback_why = 0;
    HIP_TRY(hipEventRecord(w->ev[0], w->stream));
    TRY(prepare_solves(w, n, B, ldb, Dinv));
    LzResult r{};
    const int lrc = lz_solve(w, n, s, s, op_fp64(A, lda, B, ldb, Dinv), &o, Lambda, X, ldx, &r);
    if (lrc && lrc != GSYEIG_ENOCONV) return lrc;
    BlzResult br{};
    TRY(fp64_finish(w, n, s, A, lda, B, ldb, bdiag, Dinv, Lambda, X, ldx, r, br, inf));
    float t;
    HIP_TRY(hipEventElapsedTime(&t, w->ev[0], w->ev[4]));
    inf.t_total_ms = t;
    return (r.nconv >= s) ? 0 : GSYEIG_ENOCONV;
}

// The batched solve (batch_mode 0) of the instances idx (largest first):
// GS1 and the operator data of each on the worker streams; the Lanczos
// phase of all of them in one launch of k_lzb (one workgroup per instance,
// largest first from a device-side queue, each running until its
// convergence pre-check passes); the full convergence check, KI5, BT1 and
// (mixed) the refinement and the check of each on the workers.  An instance
// whose full check fails goes back to the Lanczos kernel for more steps.
static int solve_batched_lz(gsyeig_ctx *ctx, const std::vector<int64_t> &idx, const int64_t *n, const int64_t *s,
                            const double *const *A, const int64_t *lda, double *const *B, const int64_t *ldb,
                            const gsyeig_opts &o, double *const *Lambda, double *const *X, const int64_t *ldx,
                            int64_t nstreams, int *status, gsyeig_info *infos)
{
    const bool mixed = o.prec == GSYEIG_MIXED;
    const int64_t cnt = (int64_t)idx.size();
    std::vector<BatchInst> bi(cnt);
    size_t total = al256(sizeof(LzbDesc) * cnt) + al256(sizeof(int) * cnt) + 256;
    for (int64_t j = 0; j < cnt; ++j) {
        BatchInst &b = bi[j];
        const int64_t i = idx[j], nn = n[i];
        b.i = i;
        b.nvec = mixed ? mixed_block(nn, s[i], &o) : s[i];
        b.mmax = std::max<int64_t>(eff_max_steps(nn, s[i], &o), std::min<int64_t>(b.nvec, nn));
        b.ldv = round_ld(nn);
        b.ldom = b.mmax + 8;
        b.ld32 = batch_ld(nn);
        total += al256(tri_aux_bytes(nn)) + al256(sizeof(double) * (size_t)b.ldv * (size_t)(b.mmax + 1)) +
                 2 * al256(sizeof(double) * (size_t)b.mmax) + al256(sizeof(double) * (size_t)(3 * b.ldom + 8)) +
                 al256(sizeof(double) * (size_t)lzb_scratch_doubles(nn, b.mmax));
        if (mixed)
            total += 2 * al256(sizeof(float) * (size_t)b.ld32 * (size_t)nn) + al256(trsv_w_side_bytes(nn));
        else
            total += al256(sizeof(double) * (size_t)nn) +
                     (aligned16(B[i], ldb[i], nn) ? 0 : al256(sizeof(double) * (size_t)b.ld32 * (size_t)nn)) +
                     (aligned16(A[i], lda[i], nn) ? 0 : al256(sizeof(double) * (size_t)b.ld32 * (size_t)nn));
    }
    void *pool;
    TRY(ws_get(ctx, WS_BATCH, total, &pool));
    char *cur = (char *)pool;
    auto take = [&](size_t bytes) {
        char *p = cur;
        cur += al256(bytes);
        return p;
    };
    LzbDesc *desc_d = (LzbDesc *)take(sizeof(LzbDesc) * cnt);
    int *order_d = (int *)take(sizeof(int) * cnt);
    unsigned *next_d = (unsigned *)take(256);
    for (int64_t j = 0; j < cnt; ++j) {
        BatchInst &b = bi[j];
        const int64_t nn = n[b.i];
        b.Dinv = (double *)take(tri_aux_bytes(nn));
        b.V = (double *)take(sizeof(double) * (size_t)b.ldv * (size_t)(b.mmax + 1));
        b.alpha = (double *)take(sizeof(double) * (size_t)b.mmax);
        b.beta = (double *)take(sizeof(double) * (size_t)b.mmax);
        b.om = (double *)take(sizeof(double) * (size_t)(3 * b.ldom + 8));
        b.chk = (double *)take(sizeof(double) * (size_t)lzb_scratch_doubles(nn, b.mmax));
        b.U32 = b.A32 = nullptr;
        b.sb = b.bdiag = b.Ucp = b.Acp = nullptr;
        if (mixed) {
            b.U32 = (float *)take(sizeof(float) * (size_t)b.ld32 * (size_t)nn);
            b.A32 = (float *)take(sizeof(float) * (size_t)b.ld32 * (size_t)nn);
            b.sb = (double *)take(trsv_w_side_bytes(nn));
        } else {
            b.bdiag = (double *)take(sizeof(double) * (size_t)nn);
            if (!aligned16(B[b.i], ldb[b.i], nn)) b.Ucp = (double *)take(sizeof(double) * (size_t)b.ld32 * (size_t)nn);
            if (!aligned16(A[b.i], lda[b.i], nn)) b.Acp = (double *)take(sizeof(double) * (size_t)b.ld32 * (size_t)nn);
        }
    }

    // GS1 and the operator data, each instance on a worker stream
    TRY(run_workers(ctx, nstreams, cnt, [&](gsyeig_ctx *w, int64_t j) {
        BatchInst &b = bi[j];
        const int64_t i = b.i, nn = n[i];
        int *info_d = (int *)w->dscal + 16;
        HIP_TRY(hipEventRecord(w->ev[0], w->stream));
        if (mixed) {
            // the kernel's row sums read U~'s row padding: zero
            HIP_TRY(hipMemsetAsync(b.U32, 0, sizeof(float) * (size_t)b.ld32 * (size_t)nn, w->stream));
            TRY(potrf_mixed_enqueue(w, nn, B[i], ldb[i], b.U32, b.ld32, b.Dinv, info_d));
            TRY(launch_to_f32(A[i], lda[i], b.A32, b.ld32, nn, nn, w->stream));
            const int64_t SB = trsv_sb_rows();
            TRY(launch_sb_inverses_f32(b.U32, b.ld32, nn, b.Dinv, b.sb, b.sb + cdiv(nn, SB) * SB * SB, w->stream));
        } else {
            TRY(launch_copy_diag(B[i], ldb[i], nn, b.bdiag, w->stream));
            TRY(potrf_core(w, nn, B[i], ldb[i], b.Dinv, info_d));
            if (b.Ucp) {
                HIP_TRY(hipMemsetAsync(b.Ucp, 0, sizeof(double) * (size_t)b.ld32 * (size_t)nn, w->stream));
                TRY(launch_blk_copy(B[i], ldb[i], b.Ucp, b.ld32, nn, nn, w->stream));
            }
            if (b.Acp) TRY(launch_blk_copy(A[i], lda[i], b.Acp, b.ld32, nn, nn, w->stream));
        }
        HIP_TRY(hipEventRecord(w->ev[1], w->stream));
        int *hi = (int *)w->host_pinned;
        HIP_TRY(hipMemcpyAsync(hi, info_d, sizeof(int), hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        b.gs1 = hi[0];
        HIP_TRY(hipEventElapsedTime(&b.t_gs1_ms, w->ev[0], w->ev[1]));
        return 0;
    }));

    std::vector<LzbDesc> desc(cnt);
    std::vector<int> pend;
    for (int64_t j = 0; j < cnt; ++j) {
        const BatchInst &b = bi[j];
        const int64_t i = b.i;
        if (b.gs1) {
            status[i] = b.gs1;
            continue;
        }
        LzbDesc &d = desc[j];
        memset(&d, 0, sizeof(d));
        d.n = n[i];
        d.s = s[i];
        d.nvec = b.nvec;
        d.mmax = b.mmax;
        d.every = std::max<int64_t>(1, o.check_every);
        d.which = o.which;
        d.tol = o.tol;
        d.U = mixed ? (const void *)b.U32 : b.Ucp ? (const void *)b.Ucp : (const void *)B[i];
        d.ldu = (mixed || b.Ucp) ? b.ld32 : ldb[i];
        d.Dinv = b.Dinv;
        d.A = mixed ? (const void *)b.A32 : b.Acp ? (const void *)b.Acp : (const void *)A[i];
        d.lda = (mixed || b.Acp) ? b.ld32 : lda[i];
        d.seed = o.seed;
        d.V = b.V;
        d.ldv = b.ldv;
        d.alpha = b.alpha;
        d.beta = b.beta;
        d.om = b.om;
        d.ldom = b.ldom;
        d.chk = b.chk;
        d.next_check = d.every;
        d.prev_m = -1;
        pend.push_back((int)j);
    }
    while (!pend.empty()) {
        // the Lanczos phase of every pending instance: one launch
        HIP_TRY(hipMemcpyAsync(desc_d, desc.data(), sizeof(LzbDesc) * cnt, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(order_d, pend.data(), sizeof(int) * pend.size(), hipMemcpyHostToDevice,
                               ctx->stream));
        TRY(launch_lzb(desc_d, order_d, (int)pend.size(), next_d, mixed ? 1 : 0, ctx->stream));
        HIP_TRY(hipMemcpyAsync(desc.data(), desc_d, sizeof(LzbDesc) * cnt, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        // full check, KI5, BT1, refinement and check on the workers
        std::mutex mu;
        std::vector<int> again;
        TRY(run_workers(ctx, nstreams, (int64_t)pend.size(), [&](gsyeig_ctx *w, int64_t k) {
            const int j = pend[k];
            const BatchInst &b = bi[j];
            LzbDesc &d = desc[j];
            const int64_t i = b.i, nn = n[i], m = d.k, nvec = b.nvec;
            void *p;
            TRY(ws_get(w, WS_T, sizeof(double) * (size_t)(2 * nvec + 16), &p));
            double *theta = (double *)p, *lastc = theta + nvec + 1;
            TRY(ws_get(w, WS_TRI, sizeof(double) * (size_t)nvec * 7 * (size_t)m, &p));
            double *tri = (double *)p;
            int *hi = (int *)w->host_pinned;
            const float t_lz = (float)((double)d.ticks * 1e-5);
            auto resolve = [&]() {
                gsyeig_info inf;
                const int rc = batch_resolve(w, nn, s[i], A[i], lda[i], B[i], ldb[i], o, b.Dinv, b.bdiag, Lambda[i],
                                             X[i], ldx[i], inf);
                inf.t_gs1_ms += b.t_gs1_ms;
                inf.t_ki_ms += t_lz;  // the abandoned one-launch phase counts too
                inf.t_total_ms += b.t_gs1_ms + t_lz;
                status[i] = rc;
                if (infos) infos[i] = inf;
                return (rc > 0 || rc == GSYEIG_ENOCONV) ? 0 : rc;
            };
            if (d.status == 4) return resolve();
            int64_t nconv = s[i];
            bool have_theta = false;
            HIP_TRY(hipEventRecord(w->ev[6], w->stream));
            if (d.status != 1) {
                const int64_t w0 = o.which ? nvec - s[i] : 0;
                int *nconv_d = (int *)w->dscal;
                TRY(launch_tri_bisect(b.alpha, b.beta, m, nvec, o.which, theta, w->stream));
                TRY(launch_tri_vectors(b.alpha, b.beta, m, nvec, theta, nullptr, 0, tri, 0, lastc, w->stream));
                TRY(launch_conv_count(theta, lastc, b.beta + (m - 1), nvec, w0, s[i], 0, o.tol, nconv_d, w->stream));
                HIP_TRY(hipMemcpyAsync(hi, nconv_d, sizeof(int), hipMemcpyDeviceToHost, w->stream));
                HIP_TRY(hipStreamSynchronize(w->stream));
                nconv = hi[0];
                have_theta = true;
                if (nconv < s[i] && m < b.mmax) {  // more steps
                    d.status = 0;
                    d.next_check = m + d.every;
                    std::lock_guard<std::mutex> g(mu);
                    again.push_back(j);
                    return 0;
                }
            }
            if (!have_theta) TRY(launch_tri_bisect(b.alpha, b.beta, m, nvec, o.which, theta, w->stream));
            w->n_fallback = w->fallback_why = 0;
            double *Y, *theta_out;
            int64_t ldy;
            if (mixed) {
                TRY(refine_x0(w, nn, nvec, &Y, &ldy));
                TRY(ws_get(w, WS_BDIAG, sizeof(double) * (size_t)(nn + 8), &p));
                theta_out = (double *)p;
            } else {
                Y = X[i];
                ldy = ldx[i];
                theta_out = Lambda[i];
            }
            int *oinfo_d = (int *)w->dscal + 24;
            TRY(lz_ritz_vectors(w, nn, m, nvec, 2, b.alpha, b.beta, b.V, b.ldv, theta, lastc, tri, theta_out, Y, ldy,
                                oinfo_d));
            HIP_TRY(hipEventRecord(w->ev[7], w->stream));
            HIP_TRY(hipMemcpyAsync(hi + 2, oinfo_d + 2, sizeof(int), hipMemcpyDeviceToHost, w->stream));
            HIP_TRY(hipStreamSynchronize(w->stream));
            LzResult r{};
            r.steps = m;
            r.nconv = (hi[2] != 0) ? 0 : nconv;  // a basis that lost semi-orthogonality gives no valid vectors
            r.reorth_steps = d.reorth_steps;
            r.t_loop_ms = (float)((double)d.ticks * 1e-5);
            HIP_TRY(hipEventElapsedTime(&r.t_ritz_ms, w->ev[6], w->ev[7]));
            gsyeig_info inf;
            memset(&inf, 0, sizeof(inf));
            BlzResult br{};
            int rc;
            if (hi[2] != 0 || nconv < s[i]) {
                return resolve();
            } else if (mixed) {
                rc = mixed_finish(w, nn, s[i], nvec, A[i], lda[i], B[i], ldb[i], o, b.U32, b.ld32, b.Dinv, b.sb,
                                  b.A32, Y, ldy, r, br, Lambda[i], X[i], ldx[i], inf);
                if (rc && rc != GSYEIG_ENOCONV) return rc;
            } else {
                TRY(fp64_finish(w, nn, s[i], A[i], lda[i], B[i], ldb[i], b.bdiag, b.Dinv, Lambda[i], X[i], ldx[i], r,
                                br, inf));
                rc = (r.nconv >= s[i]) ? 0 : GSYEIG_ENOCONV;
            }
            inf.t_gs1_ms = b.t_gs1_ms;
            inf.t_total_ms = inf.t_gs1_ms + inf.t_ki_ms + inf.t_ki5_ms + inf.t_bt1_ms + inf.t_refine_ms + inf.t_check_ms;
            inf.cluster_fallbacks = w->n_fallback;
            inf.fallback_reason = w->fallback_why;
            status[i] = rc;
            if (infos) infos[i] = inf;
            return 0;
        }));
        std::sort(again.begin(), again.end());
        pend.swap(again);
    }
    return 0;
}

extern "C" {

const char *gsyeig_version(void) { return "gsyeig-gfx950 0.1.0"; }

int gsyeig_opts_default(gsyeig_opts *opts)
{
    if (!opts) return -1;
    opts_fill_defaults(opts);
    return 0;
}

int gsyeig_create(gsyeig_ctx **ctx_out, void *hip_stream)
{
    if (!ctx_out) return -1;
    gsyeig_ctx *ctx = new (std::nothrow) gsyeig_ctx;
    if (!ctx) return GSYEIG_ENOMEM;
    memset(ctx, 0, sizeof(*ctx));
    ctx->stream = (hipStream_t)hip_stream;
    ctx->symv_map_n = -1;
    ctx->trsv_block = 512;
    ctx->trsv_sweep = 0;
    ctx->trsvq_n = -1;
    if (hipGetDevice(&ctx->device) != hipSuccess) { delete ctx; return GSYEIG_EHIP; }
    if (hipHostMalloc(&ctx->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
        delete ctx;
        return GSYEIG_EHIP;
    }
    if (hipMalloc(&ctx->dscal, 4096) != hipSuccess) { delete ctx; return GSYEIG_EHIP; }
    for (int i = 0; i < 10; ++i)
        if (hipEventCreate(&ctx->ev[i]) != hipSuccess) { delete ctx; return GSYEIG_EHIP; }
    for (int i = 0; i < 64; ++i)
        if (hipEventCreate(&ctx->pev[i]) != hipSuccess) { delete ctx; return GSYEIG_EHIP; }
    if (hipMalloc((void **)&ctx->ctl_lz, sizeof(LzCtl)) != hipSuccess) { delete ctx; return GSYEIG_EHIP; }
    int rc = ctl_reserve(ctx, 65536);
    if (!rc) rc = lzctl_init(ctx);
    if (rc) { delete ctx; return rc; }
    void *scr;  // set-up of gsyeig_symv_noalloc on this device (its scratch array's address)
    if ((rc = noalloc_scratch(&scr))) { delete ctx; return rc; }
    *ctx_out = ctx;
    return 0;
}

int gsyeig_destroy(gsyeig_ctx *ctx)
{
    if (!ctx) return -1;
    for (int i = 0; i < ctx->nworkers; ++i) {
        gsyeig_destroy(ctx->workers[i]);
        (void)hipStreamDestroy(ctx->wstreams[i]);
    }
    (void)hipStreamSynchronize(ctx->stream);
    for (int i = 0; i < WS_COUNT; ++i)
        if (ctx->ws[i]) (void)hipFree(ctx->ws[i]);
    if (ctx->ctl_n) (void)hipFree(ctx->ctl_n);
    if (ctx->ctl_t) (void)hipFree(ctx->ctl_t);
    if (ctx->ctl_lz) (void)hipFree(ctx->ctl_lz);
    if (ctx->dscal) (void)hipFree(ctx->dscal);
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    for (int i = 0; i < 10; ++i)
        if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
    for (int i = 0; i < 64; ++i)
        if (ctx->pev[i]) (void)hipEventDestroy(ctx->pev[i]);
    delete ctx;
    return 0;
}

int gsyeig_set_trsv_block(gsyeig_ctx *ctx, int64_t rows)
{
    if (!ctx) return -1;
    if (rows != 64 && rows != trsv_sb_rows()) return -2;
    ctx->trsv_block = rows;
    return 0;
}

}  // extern "C"

// time `reps` applications of f after `warm` untimed ones (ms per call)
template <typename F>
static int time_calls(gsyeig_ctx *ctx, int warm, int reps, F f, double *ms)
{
    for (int k = 0; k < warm; ++k) TRY(f());
    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    for (int k = 0; k < reps; ++k) TRY(f());
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    HIP_TRY(hipEventSynchronize(ctx->ev[1]));
    float t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
    *ms = t / reps;
    return 0;
}

static int autotune_measure(gsyeig_ctx *ctx, int64_t nm, int prec, double *U, double *A, int64_t ld, double *w,
                            double *z, double *Cb, gsyeig_tuning *t)
{
    TRY(launch_synth_operands(U, A, ld, nm, 0x6374ull + (uint64_t)nm, ctx->stream));
    TRY(launch_fill_splitmix(w, nm, 17, ctx->stream));
    TRY(ctl_reserve(ctx, nm));
    void *p;
    TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)nm, &p));
    double *tmp = (double *)p;
    const int64_t save_block = ctx->trsv_block;
    const int save_sweep = ctx->trsv_sweep;
    struct Cand { int block, sweep; } cands[5] = {{512, 0}, {512, 1}, {512, 2}, {512, 3}, {64, 0}};
    float *U32 = nullptr;
    if (prec == GSYEIG_MIXED) {
        TRY(ws_get(ctx, WS_U32, sizeof(float) * (size_t)ld * (size_t)nm, &p));
        U32 = (float *)p;
        TRY(launch_to_f32(U, ld, U32, ld, nm, nm, ctx->stream));
    }
    double best = 1e300;
    for (int c = 0; c < 5; ++c) {
        t->op_ms_cand[c] = 0.0;
        if (prec == GSYEIG_MIXED && cands[c].block == 64) continue;  // FP32 storage: super-block sweeps only
        ctx->trsv_block = cands[c].block;
        ctx->trsv_sweep = cands[c].sweep;
        LzOp op;
        if (prec == GSYEIG_MIXED) {
            TRY(mixed_operator(ctx, nm, A, ld, U32, ld, false, &op));
        } else {
            double *Dinv;
            TRY(dinv_from_u(ctx, nm, U, ld, &Dinv));
            op = op_fp64(A, ld, U, ld, Dinv);
        }
        double ms;
        TRY(time_calls(ctx, 2, 5, [&]() { return apply_op(ctx, nm, op, w, z, tmp); }, &ms));
        t->op_ms_cand[c] = ms;
        if (ms < best) {
            best = ms;
            t->trsv_block = cands[c].block;
            t->trsv_sweep = cands[c].sweep;
            t->op_ms = ms;
        }
    }
    ctx->trsv_block = save_block;
    ctx->trsv_sweep = save_sweep;
    // product tile: an n x n x 256 update (the shape of the Cholesky's
    // trailing products and of the block solves of GS2), both tile rules
    const int64_t nc = std::min<int64_t>(nm, 8192);
    const int64_t save_big = gemm_big_min();
    const int64_t rules[2] = {2048, 0};
    double gbest = 1e300;
    for (int r = 0; r < 2; ++r) {
        gemm_set_big_min(rules[r]);
        GemmDesc d{};
        d.m = nc; d.n = nc; d.k = 256;
        d.A = A; d.lda = ld; d.a_layout = 1;
        d.B = U; d.ldb = ld; d.b_layout = 1;
        d.C = Cb; d.ldc = nc; d.c_layout = 0;
        d.alpha = 1.0; d.beta = 0.0;
        d.f32 = (prec == GSYEIG_MIXED) ? 1 : 0;
        double ms;
        TRY(time_calls(ctx, 1, 3, [&]() { return launch_gemm(d, ctx->stream); }, &ms));
        t->gemm_ms_cand[r] = ms;
        if (ms < gbest) {
            gbest = ms;
            t->gemm_big_min = rules[r];
            t->gemm_ms = ms;
        }
    }
    gemm_set_big_min(save_big);
    return 0;
}

extern "C" {

int gsyeig_autotune(gsyeig_ctx *ctx, int64_t n, int prec, const char *cache_path, gsyeig_tuning *out)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (prec != GSYEIG_FP64 && prec != GSYEIG_MIXED) return -3;
    int64_t nb = 1024;
    while (nb < n && nb < 65536) nb *= 2;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, ctx->device));
    const char *arch = prop.gcnArchName;
    gsyeig_tuning t;
    memset(&t, 0, sizeof(t));
    t.n_bucket = nb;
    t.prec = prec;
    std::vector<TuneEntry> ents;
    std::string others;
    if (cache_path) {
        TRY(tune_cache_load(cache_path, arch, &ents, &others));
        for (const TuneEntry &e : ents)
            if (e.prec == prec && e.n_bucket == nb) {
                t.trsv_block = e.trsv_block;
                t.trsv_sweep = e.trsv_sweep;
                t.gemm_big_min = e.gemm_big_min;
                t.op_ms = e.op_ms;
                t.gemm_ms = e.gemm_ms;
                t.from_cache = 1;
                ctx->trsv_block = t.trsv_block;
                ctx->trsv_sweep = t.trsv_sweep;
                gemm_set_big_min(t.gemm_big_min);
                if (out) *out = t;
                return 0;
            }
    }
    const int64_t nm = std::min<int64_t>(nb, 32768), ld = round_ld(nm);
    const int64_t nc = std::min<int64_t>(nm, 8192);
    double *U = nullptr, *A = nullptr, *v = nullptr, *Cb = nullptr;
    int rc = 0;
    if (hipMalloc(&U, sizeof(double) * (size_t)ld * (size_t)nm) != hipSuccess ||
        hipMalloc(&A, sizeof(double) * (size_t)ld * (size_t)nm) != hipSuccess ||
        hipMalloc(&v, sizeof(double) * 2 * (size_t)ld) != hipSuccess ||
        hipMalloc(&Cb, sizeof(double) * (size_t)nc * (size_t)nc) != hipSuccess) {
        (void)hipGetLastError();
        rc = GSYEIG_ENOMEM;
    }
    if (!rc) rc = autotune_measure(ctx, nm, prec, U, A, ld, v, v + ld, Cb, &t);
    (void)hipStreamSynchronize(ctx->stream);
    if (U) (void)hipFree(U);
    if (A) (void)hipFree(A);
    if (v) (void)hipFree(v);
    if (Cb) (void)hipFree(Cb);
    if (rc) return rc;
    ctx->trsv_block = t.trsv_block;
    ctx->trsv_sweep = t.trsv_sweep;
    gemm_set_big_min(t.gemm_big_min);
    if (out) *out = t;
    if (cache_path) {
        ents.push_back(TuneEntry{prec, nb, t.trsv_block, t.trsv_sweep, t.gemm_big_min, t.op_ms, t.gemm_ms});
        return tune_cache_store(cache_path, arch, ents, others);
    }
    return 0;
}

int gsyeig_set_trsv_sweep(gsyeig_ctx *ctx, int kind)
{
    if (!ctx) return -1;
    if (kind < 0 || kind > 3) return -2;
    ctx->trsv_sweep = kind;
    return 0;
}

int gsyeig_set_spin_limit(gsyeig_ctx *ctx, unsigned limit)
{
    if (!ctx) return -1;
    ctx->spin_limit = limit;
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&ctx->ctl_n->spin, (int)limit, 1, ctx->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&ctx->ctl_t->spin, (int)limit, 1, ctx->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&ctx->ctl_lz->spin, (int)limit, 1, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int gsyeig_sync(gsyeig_ctx *ctx)
{
    if (!ctx) return -1;
    return ctl_check(ctx);
}

int gsyeig_workspace_size(int64_t n, int64_t s, const gsyeig_opts *opts, size_t *bytes)
{
    if (n < 1) return -1;
    if (s < 1 || s > n) return -2;
    if (!bytes) return -4;
    gsyeig_opts o;
    if (opts) o = *opts; else opts_fill_defaults(&o);
    const int64_t mmax = eff_max_steps(n, s, &o);
    const int64_t ldv = round_ld(n), nblk = cdiv(n, NB);
    size_t b = 0;
    b += 3 * sizeof(double) * (size_t)nblk * NB * NB;             // Dinv, M, M'
    b += sizeof(double) * (size_t)ldv * (size_t)(mmax + 1);       // V
    b += sizeof(double) * (size_t)(2 * mmax + 2 * s + 16);        // T
    b += sizeof(double) * (size_t)s * 7 * (size_t)mmax;           // tridiagonal scratch
    b += sizeof(double) * (size_t)mmax * (size_t)s;               // S
    b += 2 * sizeof(double) * (size_t)ldv * (size_t)s;            // check blocks
    b += sizeof(double) * (size_t)nblk * nblk * NB;               // SYMV column partials
    b += trsv_w_side_bytes(n);                                    // super-block inverses, link blocks
    b += sizeof(double) * (size_t)ldv * (size_t)n;                // W (super-block solves)
    b += sizeof(double) * (size_t)nblk * cdiv(nblk, 4) * NB;      // SYMV row partials
    b += sizeof(double) * (size_t)(lz_red_parts(n) * (mmax + 8) + 4 * n + 2048);
    if (o.block > 1) {
        const int64_t nv = (o.prec == GSYEIG_MIXED) ? mixed_block(n, s, &o) : s;
        if (blz_check_dims(n, s, nv, &o)) return -8;
        b += blz_bytes(n, s, nv, &o);                                 // block basis, projected matrix
    }
    if (o.reorth == 2)  // omega estimates; Gram matrix of the basis and its diagonal-block inverses
        b += sizeof(double) * ((size_t)(3 * (mmax + 8) + 8) + (size_t)mmax * (size_t)mmax +
                               (size_t)cdiv(mmax, NB) * NB * NB);
    if (o.variant != GSYEIG_KI) b += 2 * sizeof(double) * (size_t)ldv * (size_t)n;  // C and its scratch
    if (o.variant == GSYEIG_TD) b += syev_small_scratch(n, s) + sizeof(double) * (size_t)(n + 1) * (size_t)s;
    if (o.invert) {
        b += sizeof(double) * (size_t)ldv * (size_t)s;                // inverse-pencil vectors
        if (o.prec == GSYEIG_FP64) b += sizeof(double) * (size_t)ldv * (size_t)n;  // copy of A
    }
    if (o.prec == GSYEIG_MIXED) {
        const int64_t k = mixed_block(n, s, &o);
        b += 2 * sizeof(float) * (size_t)ldv * (size_t)n;           // A~, U~ (FP32)
        b += refine_bytes(n, k);                                      // refinement blocks
        b += sizeof(double) * (size_t)(k - s) * 8 * (size_t)mmax;     // wider Ritz extraction
    }
    *bytes = b;
    return 0;
}

int gsyeig_potrf(gsyeig_ctx *ctx, int64_t n, double *B, int64_t ldb, const gsyeig_opts *opts,
                 void *U_lowprec)
{
    (void)opts;
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!B) return -3;
    if (ldb < n) return -4;
    if (opts && opts->prec == GSYEIG_MIXED && !U_lowprec) return -6;
    double *Dinv;
    int *info_d = (int *)ctx->dscal + 16;
    if (U_lowprec) {
        void *p;
        TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
        TRY(potrf_mixed_enqueue(ctx, n, B, ldb, (float *)U_lowprec, n, (double *)p, info_d));
    } else {
        TRY(potrf_enqueue(ctx, n, B, ldb, &Dinv, info_d));
    }
    int *h = (int *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, info_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return h[0];
}

int gsyeig_trsv(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, int trans,
                const double *b, double *x)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!U) return -3;
    if (ldu < n) return -4;
    if (trans != 0 && trans != 1) return -5;
    if (!b) return -6;
    if (!x) return -7;
    TRY(ctl_reserve(ctx, n));
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    return trans == 0 ? solve_n(ctx, n, U, ldu, Dinv, b, x) : solve_t(ctx, n, U, ldu, Dinv, b, x);
}

int gsyeig_symv(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x, double *y)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!x) return -5;
    if (!y) return -6;
    return launch_symv(ctx, n, A, lda, x, y);
}

int gsyeig_apply_op(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *U,
                    int64_t ldu, const double *w, double *z)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!U) return -5;
    if (ldu < n) return -6;
    if (!w) return -7;
    if (!z) return -8;
    TRY(ctl_reserve(ctx, n));
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    void *p;
    TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)n, &p));
    return apply_op(ctx, n, op_fp64(A, lda, U, ldu, Dinv), w, z, (double *)p);
}

int gsyeig_form_c(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *U, int64_t ldu,
                  double *C, int64_t ldc)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!U) return -5;
    if (ldu < n) return -6;
    if (!C) return -7;
    if (ldc < n) return -8;
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    const double *sb;
    TRY(block_sb_fp64(ctx, n, U, ldu, Dinv, &sb));
    const double *Wd = (ctx->trsv_block == 64) ? nullptr : (const double *)ctx->ws[WS_W];
    void *pt;
    TRY(ws_get(ctx, WS_CKE2, sizeof(double) * (size_t)round_ld(n) * (size_t)n, &pt));
    return form_c(A, lda, U, ldu, Wd, round_ld(n), sb, n, C, ldc, (double *)pt, round_ld(n), ctx->stream);
}

int gsyeig_lanczos_run(gsyeig_ctx *ctx, int64_t n, int64_t k, const double *A, int64_t lda,
                       const double *U, int64_t ldu, const double *v0, double *alpha, double *beta,
                       double *V, int64_t ldv)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (k < 1 || k > n) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!U) return -6;
    if (ldu < n) return -7;
    if (!v0) return -8;
    if (!alpha) return -9;
    if (!beta) return -10;
    if (!V) return -11;
    if (ldv < n) return -12;
    TRY(ctl_reserve(ctx, n));
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    LzBufs b;
    TRY(lz_bufs(ctx, n, k, &b));
    TRY(launch_normalize_into(v0, V, n, b.red, nullptr, ctx->stream));
    const LzOp op = op_fp64(A, lda, U, ldu, Dinv);
    b.reorth = 0;  // this entry point always applies both Gram-Schmidt passes
    for (int64_t j = 0; j < k; ++j) TRY(lz_step(ctx, n, op, V, ldv, alpha, beta, j, b));
    return 0;
}

int gsyeig_tridiag_eig(gsyeig_ctx *ctx, int64_t m, const double *alpha, const double *beta,
                       int64_t nwant, int which, double *theta, double *S, int64_t lds)
{
    if (!ctx) return -1;
    if (m < 1) return -2;
    if (!alpha) return -3;
    if (!beta && m > 1) return -4;
    if (nwant < 1 || nwant > m) return -5;
    if (which != 0 && which != 1) return -6;
    if (!theta) return -7;
    if (S && lds < m) return -9;
    void *p;
    TRY(ws_get(ctx, WS_T, sizeof(double) * (size_t)(2 * nwant + 16), &p));
    double *th = (double *)p, *lastc = th + nwant + 1;
    TRY(ws_get(ctx, WS_TRI, sizeof(double) * (size_t)nwant * 7 * (size_t)m, &p));
    double *tri = (double *)p;
    TRY(launch_tri_bisect(alpha, beta ? beta : alpha, m, nwant, which, th, ctx->stream));
    if (S) TRY(launch_tri_vectors(alpha, beta ? beta : alpha, m, nwant, th, S, lds, tri, 1, lastc,
                                  ctx->stream));
    return launch_copy(th, theta, nwant, ctx->stream);
}

int gsyeig_lanczos(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda,
                   const double *U, int64_t ldu, const gsyeig_opts *opts, double *theta, double *Y,
                   int64_t ldy, int64_t *steps_out)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (s < 1 || s > n) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!U) return -6;
    if (ldu < n) return -7;
    if (!theta) return -9;
    if (!Y) return -10;
    if (ldy < n) return -11;
    gsyeig_opts o;
    if (opts) o = *opts; else opts_fill_defaults(&o);
    if (o.prec != GSYEIG_FP64 || o.block < 1 || o.invert || o.reorth < 0 || o.reorth > 2) return -8;
    if (o.block > 1) TRY(blz_check_dims(n, s, s, &o));
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    if (o.block > 1) {
        const double *sb;
        TRY(block_sb_fp64(ctx, n, U, ldu, Dinv, &sb));
        const double *Wd = (ctx->trsv_block == 64) ? nullptr : (const double *)ctx->ws[WS_W];
        BlkOp bop{U, 0, ldu, Wd, 0, round_ld(n), sb, A, 0, lda, 0};
        BlzResult br{};
        TRY(blz_solve(ctx, n, s, s, bop, &o, theta, Y, ldy, &br));
        if (steps_out) *steps_out = br.steps;
        return (br.nconv >= s) ? 0 : GSYEIG_ENOCONV;
    }
    LzResult r{};
    const int lrc = lz_solve(ctx, n, s, s, op_fp64(A, lda, U, ldu, Dinv), &o, theta, Y, ldy, &r);
    if (steps_out) *steps_out = r.steps;
    if (lrc) return lrc;
    return (r.nconv >= s) ? 0 : GSYEIG_ENOCONV;
}

int gsyeig_backsolve(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *U, int64_t ldu,
                     double *Y_to_X, int64_t ldy)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (s < 1) return -3;
    if (!U) return -4;
    if (ldu < n) return -5;
    if (!Y_to_X) return -6;
    if (ldy < n) return -7;
    double *Dinv;
    TRY(dinv_from_u(ctx, n, U, ldu, &Dinv));
    return launch_backsolve(U, ldu, n, s, Dinv, Y_to_X, ldy, ctx->stream);
}

int gsyeig_check(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda,
                 const double *B, int64_t ldb, const double *Bdiag, const double *Lambda,
                 const double *X, int64_t ldx, gsyeig_info *out)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (s < 1 || s > n) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!B) return -6;
    if (ldb < n) return -7;
    if (!Lambda) return -9;
    if (!X) return -10;
    if (ldx < n) return -11;
    if (!out) return -12;
    double *res_d = (double *)ctx->dscal + 64;
    TRY(check_enqueue(ctx, n, s, A, lda, B, ldb, Bdiag, Lambda, X, ldx, res_d));
    double *h = (double *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(h, res_d, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    out->eta_max = h[0];
    out->rho_f = h[1];
    out->omega = h[2];
    out->normA_f = h[3];
    out->normB_f = h[4];
    return 0;
}

int gsyeig_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, double *B,
                 int64_t ldb, const gsyeig_opts *opts, double *Lambda, double *X, int64_t ldx,
                 gsyeig_info *info)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (s < 1 || s > n) return -3;
    if (!A) return -4;
    if (lda < n) return -5;
    if (!B) return -6;
    if (ldb < n) return -7;
    gsyeig_opts o;
    if (opts) o = *opts; else opts_fill_defaults(&o);
    if (!o.invert) ctx->n_fallback = ctx->fallback_why = 0;
    if ((o.prec != GSYEIG_FP64 && o.prec != GSYEIG_MIXED) || o.block < 1 || (o.invert != 0 && o.invert != 1) ||
        o.reorth < 0 || o.reorth > 2 ||
        (o.which != 0 && o.which != 1) || o.variant < GSYEIG_KI || o.variant > GSYEIG_TD ||
        (o.variant != GSYEIG_KI && (o.prec != GSYEIG_FP64 || o.block != 1 || o.invert)))
        return -8;
    if (o.block > 1) TRY(blz_check_dims(n, s, o.prec == GSYEIG_MIXED ? mixed_block(n, s, &o) : s, &o));
    if (!Lambda) return -9;
    if (!X) return -10;
    if (ldx < n) return -11;
    if (o.invert) {
        ctx->n_fallback = 0;
        const int rc = solve_inverted(ctx, n, s, A, lda, B, ldb, o, Lambda, X, ldx, info);
        if (info) {
            info->cluster_fallbacks = ctx->n_fallback;
            info->fallback_reason = ctx->fallback_why;
        }
        return rc;
    }
    if (o.prec == GSYEIG_MIXED) {
        const int rc = solve_mixed(ctx, n, s, A, lda, B, ldb, o, Lambda, X, ldx, info);
        if (info) {
            info->cluster_fallbacks = ctx->n_fallback;
            info->fallback_reason = ctx->fallback_why;
        }
        return rc;
    }

    gsyeig_info inf;
    memset(&inf, 0, sizeof(inf));
    void *p;
    TRY(ws_get(ctx, WS_BDIAG, sizeof(double) * (size_t)n, &p));
    double *bdiag = (double *)p;
    int *info_d = (int *)ctx->dscal + 16;
    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    TRY(launch_copy_diag(B, ldb, n, bdiag, ctx->stream));
    double *Dinv;
    TRY(potrf_enqueue(ctx, n, B, ldb, &Dinv, info_d));
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    int *hi = (int *)ctx->host_pinned;
    HIP_TRY(hipMemcpyAsync(hi, info_d, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (hi[0] != 0) return hi[0];

    LzResult r{};
    BlzResult br{};
    LzOp lop = op_fp64(A, lda, B, ldb, Dinv);
    if (o.variant == GSYEIG_KE || o.variant == GSYEIG_TD) {
        // GS2: C = U^-T A U^-1 with the block solves of the factor (TD keeps
        // C at leading dimension n, the dense eigensolver's layout)
        const double *sb;
        TRY(block_sb_fp64(ctx, n, B, ldb, Dinv, &sb));
        const double *Wd = (ctx->trsv_block == 64) ? nullptr : (const double *)ctx->ws[WS_W];
        const int64_t ldc = (o.variant == GSYEIG_TD) ? n : round_ld(n);
        void *pc, *pt;
        TRY(ws_get(ctx, WS_CKE, sizeof(double) * (size_t)ldc * (size_t)n, &pc));
        TRY(ws_get(ctx, WS_CKE2, sizeof(double) * (size_t)ldc * (size_t)n, &pt));
        TRY(form_c(A, lda, B, ldb, Wd, round_ld(n), sb, n, (double *)pc, ldc, (double *)pt, ldc, ctx->stream));
        lop.C = (const double *)pc;
        lop.ldc = ldc;
    }
    HIP_TRY(hipEventRecord(ctx->ev[8], ctx->stream));
    if (o.block > 1) {
        const double *sb;
        TRY(block_sb_fp64(ctx, n, B, ldb, Dinv, &sb));
        const double *Wd = (ctx->trsv_block == 64) ? nullptr : (const double *)ctx->ws[WS_W];
        BlkOp bop{B, 0, ldb, Wd, 0, round_ld(n), sb, A, 0, lda, 0};
        TRY(blz_solve(ctx, n, s, s, bop, &o, Lambda, X, ldx, &br));
        r.steps = br.steps;
        r.nconv = br.nconv;
        r.t_loop_ms = br.t_loop_ms;
        r.t_ritz_ms = br.t_ritz_ms;
    } else if (o.variant == GSYEIG_TD) {
        // TD1-TD3 (Sec. 2.2): Householder reduction of C to tridiagonal form,
        // the s wanted eigenpairs of the tridiagonal matrix (bisection,
        // inverse iteration), back-transformation by the reflectors
        void *p;
        TRY(ws_get(ctx, WS_TRI, syev_small_scratch(n, s), &p));
        double *scr = (double *)p;
        TRY(ws_get(ctx, WS_Y2, sizeof(double) * ((size_t)n * (size_t)s + (size_t)s + 8), &p));
        double *Q = (double *)p, *w = Q + n * s;
        HIP_TRY(hipEventRecord(ctx->ev[6], ctx->stream));
        ctx->syev_site = 4;
        TRY(syev_dense(ctx, n, lop.C ? const_cast<double *>(lop.C) : nullptr, s, o.which, w, Q, scr, ctx->stream));
        TRY(launch_copy(w, Lambda, s, ctx->stream));
        TRY(launch_blk_copy(Q, n, X, ldx, n, s, ctx->stream));
        HIP_TRY(hipEventRecord(ctx->ev[7], ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        HIP_TRY(hipEventElapsedTime(&r.t_loop_ms, ctx->ev[6], ctx->ev[7]));
        r.steps = 0;
        r.nconv = s;
    } else {
        const int lrc = lz_solve(ctx, n, s, s, lop, &o, Lambda, X, ldx, &r);
        if (lrc && lrc != GSYEIG_ENOCONV) return lrc;  // ENOCONV: finish, report in info
    }
    float t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1])); inf.t_gs1_ms = t;
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[1], ctx->ev[8])); inf.t_gs2_ms = t;
    TRY(fp64_finish(ctx, n, s, A, lda, B, ldb, bdiag, Dinv, Lambda, X, ldx, r, br, inf));
    HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[4])); inf.t_total_ms = t;
    if (info) *info = inf;
    return (r.nconv >= s) ? 0 : GSYEIG_ENOCONV;
}

int gsyeig_trsv_lp(gsyeig_ctx *ctx, int64_t n, const float *U, int64_t ldu, int trans, const double *b,
                   double *x)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!U) return -3;
    if (ldu < n) return -4;
    if (trans != 0 && trans != 1) return -5;
    if (!b) return -6;
    if (!x) return -7;
    TRY(ctl_reserve(ctx, n));
    void *p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    double *sb = (double *)p;
    const int64_t ldw = round_ld(n);
    TRY(ws_get(ctx, WS_W, sizeof(float) * (size_t)ldw * (size_t)n, &p));
    float *W32 = (float *)p;
    TRY(launch_diag_inv_f32(U, ldu, n, Dinv, ctx->stream));
    TRY(launch_make_w_f32(U, ldu, n, Dinv, sb, W32, ldw, ctx->stream));
    TRY(ctl_clear_err(ctx));
    if (trans == 0) {
        if (b == x) {  // the diagonal part reads b across its super-block: solve from a copy
            TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)n, &p));
            TRY(launch_copy(b, (double *)p, n, ctx->stream));
            b = (const double *)p;
        }
        TRY(sweep_n(ctx, n, W32, 1, ldw, sb, b, x));
    } else {
        TRY(sweep_t(ctx, n, W32, 1, ldw, sb, b, nullptr, nullptr, 0, 0, x));
    }
    return ctl_check(ctx);
}

int gsyeig_apply_op_lp(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const float *U, int64_t ldu,
                       const double *w, double *z)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!U) return -5;
    if (ldu < n) return -6;
    if (!w) return -7;
    if (!z) return -8;
    TRY(ctl_reserve(ctx, n));
    void *p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    double *sb = (double *)p;
    const int64_t ldw = round_ld(n);
    TRY(ws_get(ctx, WS_W, sizeof(float) * (size_t)ldw * (size_t)n, &p));
    float *W32 = (float *)p;
    TRY(launch_diag_inv_f32(U, ldu, n, Dinv, ctx->stream));
    TRY(launch_make_w_f32(U, ldu, n, Dinv, sb, W32, ldw, ctx->stream));
    TRY(ws_get(ctx, WS_TMP2, sizeof(double) * (size_t)n, &p));
    double *tmp = (double *)p;
    if (w == z) {  // the first sweep reads w while the last one writes z
        TRY(ws_get(ctx, WS_TMP1, sizeof(double) * (size_t)n, &p));
        TRY(launch_copy(w, (double *)p, n, ctx->stream));
        w = (const double *)p;
    }
    LzOp op{};
    op.f32 = 1;
    op.Dinv = Dinv;
    op.A32 = A; op.lda32 = lda;
    op.U32 = U; op.ldu32 = ldu;
    op.W32 = W32; op.ldw32 = ldw;
    op.sb = sb;
    TRY(ctl_clear_err(ctx));
    TRY(apply_op(ctx, n, op, w, z, tmp));
    return ctl_check(ctx);
}

int gsyeig_symv_lp(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x, double *y)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!x) return -5;
    if (!y) return -6;
    TRY(launch_symv_f32(ctx, n, A, lda, x, y));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int gsyeig_trsm_lp(gsyeig_ctx *ctx, int64_t n, const float *U, int64_t ldu, int trans, int64_t k,
                   const double *V, int64_t ldv, double *X, int64_t ldx)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (!U) return -3;
    if (ldu < n) return -4;
    if (trans != 0 && trans != 1) return -5;
    if (k < 1) return -6;
    if (!V) return -7;
    if (ldv < n) return -8;
    if (!X) return -9;
    if (ldx < n) return -10;
    void *p;
    TRY(ws_get(ctx, WS_DINV, tri_aux_bytes(n), &p));
    double *Dinv = (double *)p;
    TRY(ws_get(ctx, WS_SB, trsv_w_side_bytes(n), &p));
    double *sb = (double *)p;
    const int64_t ldw = round_ld(n);
    TRY(ws_get(ctx, WS_Y, sizeof(double) * (size_t)ldw * (size_t)k, &p));
    double *W = (double *)p;
    TRY(launch_diag_inv_f32(U, ldu, n, Dinv, ctx->stream));
    TRY(launch_sb_inverses_f32(U, ldu, n, Dinv, sb, sb + cdiv(n, trsv_sb_rows()) * trsv_sb_rows() * trsv_sb_rows(),
                               ctx->stream));
    TRY(launch_blk_copy(V, ldv, W, ldw, n, k, ctx->stream));
    TRY(launch_trsm_sb_f32(trans, U, ldu, n, sb, W, ldw, X, ldx, k, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int gsyeig_syev_small(gsyeig_ctx *ctx, int64_t N, const double *H, int64_t ldh, int64_t nwant, int which,
                      double *w, double *Q, int64_t ldq)
{
    if (!ctx) return -1;
    if (N < 1 || N > syev_small_max()) return -2;
    if (!H) return -3;
    if (ldh < N) return -4;
    if (nwant < 1 || nwant > N) return -5;
    if (which != 0 && which != 1) return -6;
    if (!w) return -7;
    if (!Q) return -8;
    if (ldq < N) return -9;
    void *p;
    const size_t need = sizeof(double) * (size_t)(N * N + N * nwant + nwant + 8) + syev_small_scratch(N, nwant);
    TRY(ws_get(ctx, WS_S, need, &p));
    double *Hc = (double *)p, *Qc = Hc + N * N, *wc = Qc + N * nwant, *scr = wc + nwant + 8;
    TRY(launch_blk_copy(H, ldh, Hc, N, N, N, ctx->stream));
    TRY(syev_small(ctx, N, Hc, nwant, which, wc, Qc, scr, ctx->stream));
    TRY(launch_copy(wc, w, nwant, ctx->stream));
    TRY(launch_blk_copy(Qc, N, Q, ldq, N, nwant, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return 0;
}

int gsyeig_refine(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t k, const double *A, int64_t lda,
                  const double *B, int64_t ldb, const float *U_lowprec, int64_t ldu, const gsyeig_opts *opts,
                  const double *X0, int64_t ldx0, double *Lambda, double *X, int64_t ldx, gsyeig_info *info)
{
    if (!ctx) return -1;
    if (n < 1) return -2;
    if (s < 1 || s > n) return -3;
    if (k < s || k > n || 2 * k > syev_small_max()) return -4;
    if (!A || lda < n) return -5;
    if (!B || ldb < n) return -7;
    if (!U_lowprec || ldu < n) return -9;
    gsyeig_opts o;
    if (opts) o = *opts; else opts_fill_defaults(&o);
    if (o.which != 0 && o.which != 1) return -11;
    if (!X0 || ldx0 < n) return -12;
    if (!Lambda) return -14;
    if (!X || ldx < n) return -15;
    LzOp op;
    TRY(mixed_operator(ctx, n, A, lda, U_lowprec, ldu, false, &op));
    double *Z0;
    int64_t ldz;
    TRY(refine_x0(ctx, n, k, &Z0, &ldz));
    TRY(launch_blk_copy(X0, ldx0, Z0, ldz, n, k, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[0], ctx->stream));
    RefineOp rop{U_lowprec, ldu, op.sb, op.A32, op.lda32};
    RefineCfg cfg{o.eta_tol, o.refine_iters, o.refine_inner};
    RefineStats rs{};
    TRY(refine_run(ctx, n, s, k, o.which, A, lda, B, ldb, rop, cfg, Lambda, X, ldx, &rs));
    TRY(launch_sign_normalise(X, ldx, n, s, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->ev[1], ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (info) {
        gsyeig_info inf;
        memset(&inf, 0, sizeof(inf));
        float t;
        HIP_TRY(hipEventElapsedTime(&t, ctx->ev[0], ctx->ev[1]));
        inf.t_refine_ms = t;
        inf.t_total_ms = t;
        inf.eta_max = rs.eta;
        inf.eta_phase1 = rs.eta0;
        inf.converged = rs.nconv;
        inf.refine_iters = rs.iters;
        inf.block_applies = rs.block_applies;
        inf.block_cols = rs.kept;
        *info = inf;
    }
    return (rs.eta <= o.eta_tol) ? 0 : GSYEIG_ENOCONV;
}

// Many independent pencils (row a10 of the hot path): instances are taken
// largest-first from a shared counter by `nstreams` host threads, each
// driving its own worker context on its own HIP stream, so small solves
// overlap on the GPU.  Each instance runs exactly the single-solve path, so
// its results are bitwise those of gsyeig_solve.
int gsyeig_solve_batched(gsyeig_ctx *ctx, int64_t count, const int64_t *n, const int64_t *s,
                         const double *const *A, const int64_t *lda, double *const *B,
                         const int64_t *ldb, const gsyeig_opts *opts, double *const *Lambda,
                         double *const *X, const int64_t *ldx, int64_t nstreams, int *status,
                         gsyeig_info *infos)
{
    if (!ctx) return -1;
    if (count < 0) return -2;
    if (count == 0) return 0;
    if (!n) return -3;
    if (!s) return -4;
    if (!A) return -5;
    if (!lda) return -6;
    if (!B) return -7;
    if (!ldb) return -8;
    if (!Lambda) return -10;
    if (!X) return -11;
    if (!ldx) return -12;
    if (nstreams < 1 || nstreams > GSYEIG_MAX_STREAMS) return -13;
    if (!status) return -14;
    gsyeig_opts o;
    if (opts) o = *opts; else opts_fill_defaults(&o);
    if (o.batch_mode != 0 && o.batch_mode != 1) return -9;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    TRY(ensure_workers(ctx, nstreams));
    for (int64_t i = 0; i < count; ++i) status[i] = GSYEIG_EHIP;
    // the instances the one-launch Lanczos phase takes, and the others
    std::vector<int64_t> lz, rest;
    for (int64_t i = 0; i < count; ++i) {
        const bool ok = o.batch_mode == 0 && batch_lz_eligible(n[i], s[i], lda[i], ldb[i], ldx[i], o) &&
                        A[i] && B[i] && Lambda[i] && X[i];
        (ok ? lz : rest).push_back(i);
    }
    auto larger = [&](int64_t a, int64_t b) { return n[a] > n[b]; };
    std::stable_sort(lz.begin(), lz.end(), larger);
    std::stable_sort(rest.begin(), rest.end(), larger);
    if (!lz.empty())
        TRY(solve_batched_lz(ctx, lz, n, s, A, lda, B, ldb, o, Lambda, X, ldx, nstreams, status, infos));
    if (!rest.empty()) {
        TRY(run_workers(ctx, nstreams, (int64_t)rest.size(), [&](gsyeig_ctx *w, int64_t k) {
            const int64_t i = rest[k];
            gsyeig_info inf;
            memset(&inf, 0, sizeof(inf));
            status[i] = gsyeig_solve(w, n[i], s[i], A[i], lda[i], B[i], ldb[i], &o, Lambda[i], X[i], ldx[i], &inf);
            if (infos) infos[i] = inf;
            return 0;
        }));
    }
    for (int64_t i = 0; i < count; ++i)
        if (status[i]) return status[i];
    return 0;
}

}  // extern "C"
