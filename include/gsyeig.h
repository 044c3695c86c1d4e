/*
 * gsyeig.h -- C ABI of the MI355X (gfx950) Krylov solver for the dense
 * symmetric-definite generalized eigenproblem
 *
 *        A X = B X Lambda,   A = A^T,  B = B^T positive definite,      (Eq. 1)
 *
 * for the s algebraically smallest (or largest) eigenpairs, s << n, by the
 * paper's variant KI (Section 2.3: a Krylov method that applies C only
 * implicitly, through the factor; Table 1 keys GS1, KI1-KI5, BT1):
 *
 *   GS1  B = U^T U, U upper triangular                          (Eq. 2)
 *   KI1  wbar = U^-1 w          (triangular solve)
 *   KI2  what = A wbar          (symmetric matrix-vector product)
 *   KI3  z    = U^-T what       (triangular solve)     -> z = C w, Eq. 3
 *   KI4  Lanczos update; by default partial re-orthogonalisation (the
 *        omega recurrence decides which steps run classical Gram-Schmidt
 *        twice against the whole basis; opts.reorth selects the others)
 *   KI5  Ritz values/vectors from the tridiagonal T_m and basis V_m
 *   BT1  X = U^-1 Y                                            (Eq. 4)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every matrix/vector pointer is a DEVICE pointer (HBM of the GPU that is
 *   current when the context was created) unless the argument says "host".
 *   The caller allocates and owns them; the library never frees them.
 * - Square matrices (A, B, U) are ROW-MAJOR with leading dimension ld >= n:
 *   element (i, j) is at p[i*ld + j].  A and B are read in full storage.
 *   U is upper triangular; only its upper triangle (incl. diagonal) is read.
 * - Blocks of vectors (Y, X, V; n x s) are COLUMN-MAJOR with ld >= n: vector
 *   j occupies p[j*ld .. j*ld + n-1] (a row-major (s, n) torch tensor).
 * - All work is enqueued on the context's HIP stream.  Entry points that
 *   return results on the device are asynchronous unless stated otherwise;
 *   gsyeig_potrf, gsyeig_lanczos and gsyeig_solve synchronise the stream
 *   because they must report an info code.
 * - Return codes (LAPACK style):
 *      0            success
 *     -i            argument i (1-based) is illegal (n < 1, s > n, ld < n,
 *                   NULL pointer, ...); nothing was enqueued
 *     +k (k <= n)   the leading minor of order k of B is not positive
 *                   definite (Eq. 2 fails)
 *     GSYEIG_ENOCONV  fewer than s pairs met the tolerance within max_steps
 *     GSYEIG_EHIP     a HIP runtime call failed
 *     GSYEIG_ESPIN    a persistent kernel's bounded wait expired (internal
 *                     error; outputs undefined, the GPU is left usable).
 *                     Synchronous calls report the waits of their own
 *                     kernels; asynchronous ones through gsyeig_sync.
 * - Contexts are not thread-safe; use one per host thread/stream.
 */
#ifndef GSYEIG_H
#define GSYEIG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSYEIG_ENOCONV 0x40000000
#define GSYEIG_EHIP 0x40000001
#define GSYEIG_ESPIN 0x40000002
#define GSYEIG_ENOMEM 0x40000003
#define GSYEIG_ETOOBIG 0x40000004
#define GSYEIG_NOALLOC_MAX_N 16384
#define GSYEIG_MAX_STREAMS 16

typedef struct gsyeig_ctx gsyeig_ctx;

typedef enum { GSYEIG_FP64 = 0, GSYEIG_MIXED = 1 } gsyeig_prec;
typedef enum { GSYEIG_KI = 0, GSYEIG_KE = 1, GSYEIG_TD = 2 } gsyeig_variant;

typedef struct {
    int prec;              /* GSYEIG_FP64 (every step in FP64), or GSYEIG_MIXED:  */
                           /*   FP32 copies of A and U for the Lanczos sweeps and */
                           /*   the Cholesky trailing updates, then FP64          */
                           /*   Rayleigh-Ritz refinement on the original (A, B)   */
    int block;             /* Lanczos block size; 1 = single-vector Lanczos       */
    int which;             /* 0 = s smallest (default), 1 = s largest             */
    int invert;            /* 1: A must be SPD; solve the inverse pencil (B, A)  */
                           /*   for mu = 1/lambda (Sec. 3.1's MD run), return    */
                           /*   the pairs of (A, B) (gsyeig_solve only)           */
    double tol;            /* Ritz-residual tolerance relative to ||T_m||          */
                           /*   (default 1e-12); Section 3.3 used tol = 0, i.e.   */
                           /*   machine precision, in ARPACK's dsaupd             */
    int64_t max_steps;     /* cap on operator applications m (default             */
                           /*   min(n, max(100 s + 2000, 10 sqrt(n s))))          */
    int64_t check_every;   /* steps between convergence checks (default 25)       */
    uint64_t seed;         /* start vector w_0 = SplitMix64(seed) in [-1,1)^n     */
    const double *v0;      /* optional device start vector (n); overrides seed    */
    int64_t profile_every; /* 0 = off; else time KI1/KI2/KI3 with hipEvents on    */
                           /*   every profile_every-th Lanczos step (sampled)     */
    /* mixed mode only */
    double eta_tol;        /* refinement target: max per-pair backward error eta  */
                           /*   over the wanted pairs (default 1e-10)             */
    int64_t refine_iters;  /* most correction rounds (default 10)                 */
    int64_t refine_inner;  /* MINRES steps per correction round (default 20)      */
    int64_t guard;         /* extra Ritz vectors carried through the refinement   */
                           /*   (0 = max(8, ceil(s/4)))                           */
    /* both modes */
    int64_t reorth;        /* re-orthogonalisation against all of V_k, by        */
                           /*   classical Gram-Schmidt: 0 = two passes every step */
                           /*   (Sec. 2.3, after Kahan); 1 = the second pass only */
                           /*   when the first kept less than 1/sqrt(2) of the    */
                           /*   norm; 2 (default) = partial: the omega recurrence */
                           /*   estimates w_j^T w_{k+1} on the device, and both   */
                           /*   passes run only on the steps where an estimate    */
                           /*   exceeds sqrt(u) and on the step after each (the   */
                           /*   basis stays semi-orthogonal; the Ritz vectors are */
                           /*   then made orthonormal by Cholesky QR).  Both 1    */
                           /*   and 2 monitor orthogonality and amend it, the    */
                           /*   alternative Sec. 2.3 names.  Block Lanczos always */
                           /*   orthogonalises each block twice.  Values outside */
                           /*   0..2 are rejected (-8).                           */
    /* block Lanczos (block > 1) */
    int64_t basis;         /* most basis vectors before a thick restart (0 =     */
                           /*   min(8192, n - block, max(keep + 4 block, 5 s)))   */
    int64_t keep;          /* Ritz vectors kept at a restart (0 = the extracted  */
                           /*   pairs, at least min(2 s, 4096, (n - block) / 2))  */
    int64_t block_acc32;   /* mixed mode: 1 = block products accumulate in FP32  */
                           /*   (FP32 MFMA; the Lanczos tolerance is then no     */
                           /*   finer than 64 u_32 = 3.8e-6, the refinement      */
                           /*   finishes the pairs); 0 (default) = FP64           */
                           /*   accumulation of the FP32-stored matrices          */
    int64_t variant;       /* GSYEIG_KI (default): Lanczos on the implicit       */
                           /*   operator C = U^-T A U^-1, two triangular solves   */
                           /*   and a symmetric product per step (Sec. 2.3, KI); */
                           /*   GSYEIG_KE: C formed once (key GS2, 2 n^3 flops on */
                           /*   the matrix cores), then one symmetric product per */
                           /*   step (Sec. 2.3, KE); GSYEIG_TD: no Krylov method: */
                           /*   C formed (GS2), reduced to tridiagonal form by    */
                           /*   Householder reflectors, its s wanted pairs by     */
                           /*   bisection and inverse iteration, back-transformed */
                           /*   (Sec. 2.2, TD1-TD3; the dense comparator).  KE    */
                           /*   and TD: FP64, block = 1, invert = 0 only          */
    int64_t batch_mode;    /* gsyeig_solve_batched only: 0 (default) = the       */
                           /*   Lanczos phase of every instance it can take      */
                           /*   (n <= 4096, variant KI, block 1, reorth 2, no    */
                           /*   v0, invert 0) runs in one launch, one workgroup  */
                           /*   per instance, largest first; 1 = every instance  */
                           /*   is a gsyeig_solve on a worker stream              */
} gsyeig_opts;

typedef struct {
    int64_t steps;         /* Lanczos steps m actually taken (block Lanczos:      */
                           /*   operator applications, b per block step)          */
    int64_t converged;     /* wanted pairs whose Ritz residual met tol             */
    double eta_max;        /* max_i ||A x_i - l_i B x_i|| / ((||A||F+|l_i| ||B||F)||x_i||) */
    double rho_f;          /* ||A X - B X L||_F / max(||A||_F, ||B||_F) (Tables 3/7) */
    double omega;          /* ||I - X^T B X||_F                                    */
    double normA_f, normB_f;
    /* wall time of each Table-1 key, milliseconds (hipEvent) */
    double t_gs1_ms;       /* Cholesky                                             */
    double t_ki_ms;        /* Lanczos loop: KI1 + KI2 + KI3 + KI4 + checks         */
    double t_ki5_ms;       /* Ritz vectors                                         */
    double t_bt1_ms;       /* back-transform                                       */
    double t_check_ms;     /* FP64 residual/orthogonality check                    */
    double t_total_ms;
    /* sampled per-launch kernel times (opts.profile_every > 0), milliseconds  */
    int64_t prof_samples;  /* number of sampled steps                          */
    double t_ki1_ms_sum;   /* sum over samples of the U^-1 sweep (KI1)         */
    double t_ki2_ms_sum;   /* ... of the A product (KI2)                       */
    double t_ki3_ms_sum;   /* ... of the U^-T sweep (KI3)                      */
    /* mixed mode only */
    double t_refine_ms;    /* FP64 refinement (Rayleigh-Ritz + corrections)    */
    double eta_phase1;     /* max eta after the first FP64 Rayleigh-Ritz of the */
                           /*   FP32-sweep Ritz vectors                         */
    int64_t refine_iters;  /* correction rounds taken                           */
    int64_t block_applies; /* FP32 block operator applications (block_cols wide)*/
    int64_t block_cols;    /* width of the refinement block (s + guard)         */
    /* block Lanczos (opts.block > 1) */
    int64_t restarts;      /* thick restarts taken                              */
    int64_t basis;         /* basis size at which it restarts                   */
    int64_t kept;          /* Ritz vectors kept at a restart                    */
    double t_rr_ms;        /* projected eigen-solves of the checks (in t_ki_ms) */
    int64_t rr_count;      /* number of those                                   */
    int64_t cluster_fallbacks; /* eigenvector sets that needed the sequential  */
                           /*   Gram-Schmidt-in-clusters path (diagnostic)      */
    int64_t fallback_reason; /* last one: 1 = two vectors overlapped > 0.5,   */
                           /*   2 = their Gram matrix was not positive definite */
    int64_t reorth_steps;  /* single-vector Lanczos: steps that ran the         */
                           /*   conditional Gram-Schmidt (reorth 1: the second  */
                           /*   pass; 2: both passes; 0: every step)            */
    double t_gs2_ms;       /* variants KE, TD: forming C = U^-T A U^-1 (GS2);   */
                           /*   for TD, t_ki_ms holds TD1-TD3 (reduction,       */
                           /*   tridiagonal eigenpairs, back-transformation)    */
                           /*   and steps is 0                                  */
} gsyeig_info;

/* Choices made by gsyeig_autotune. */
typedef struct {
    int64_t n_bucket;      /* the power of two >= n (1024..65536) the entry covers */
    int prec;              /* GSYEIG_FP64 or GSYEIG_MIXED (FP32 storage of A, U)   */
    int trsv_block;        /* 64 or 512 (gsyeig_set_trsv_block)                    */
    int trsv_sweep;        /* 0 or 1 (gsyeig_set_trsv_sweep)                        */
    int from_cache;        /* 1: taken from the cache file, nothing was measured    */
    int64_t gemm_big_min;  /* matrix-core products use 128x128 tiles when both     */
                           /*   output edges are >= this (0: 64x64 tiles only)     */
    double op_ms;          /* measured operator application (KI1-KI3) of the choice */
    double gemm_ms;        /* measured n x n x 256 product of the choice            */
    double op_ms_cand[5];  /* operator with 512-row sweeps of kinds 0..3, then the */
                           /*   64-row chain (FP32 storage: the 64-row chain is not */
                           /*   used, entry 4 is 0)                                 */
    double gemm_ms_cand[2];/* product with 128x128 tiles allowed, and without       */
} gsyeig_tuning;

/* Library version string (host, static storage). */
const char *gsyeig_version(void);

/* Fill *opts with the defaults listed above.  Returns 0, or -1 if NULL. */
int gsyeig_opts_default(gsyeig_opts *opts);

/* Create a context bound to `hip_stream` (a hipStream_t, NULL = the null
 * stream) on the current device.  Allocates a small control block; larger
 * workspace is grown on demand and owned by the context. */
int gsyeig_create(gsyeig_ctx **ctx, void *hip_stream);

/* Wait for the context's stream and free everything the context owns. */
int gsyeig_destroy(gsyeig_ctx *ctx);

/* Chain granularity of the triangular solves KI1/KI3 for subsequent calls
 * on this context: 64 = one 64-row diagonal block per chain link (each
 * link multiplies by the inverse of a 64x64 diagonal block); 512 (default) =
 * 512-row super-blocks applied through their explicit inverses (8x fewer
 * chain links; the forward error then carries the condition number of the
 * 512x512 diagonal blocks of U).  Returns 0, -1 (NULL ctx), -2 (other sizes).
 * Host-only setting; takes effect at the next factorisation or solve. */
int gsyeig_set_trsv_block(gsyeig_ctx *ctx, int64_t rows);

/* Kernel design of the 512-row super-block sweeps (KI1/KI3) on this
 * context.  Work-queue sweep: the panel products with already-solved
 * super-blocks are separate queue items taken in the order the chain needs
 * them, so the links wait only on their neighbours' values (k_trsv_q.hip);
 * per-tile sweep: one persistent workgroup per 64-row tile streams its
 * whole panel as the values arrive (k_trsv_w.hip).  kind 0 (default) =
 * both sweeps work-queue, 1 = both per-tile, 2 = KI1 per-tile and KI3
 * work-queue, 3 = KI1 work-queue and KI3 per-tile.  All compute the same
 * solve up to the grouping of the panel sums.  Host-only setting; returns
 * 0, -1 (NULL ctx) or -2 (kind outside 0..3). */
int gsyeig_set_trsv_sweep(gsyeig_ctx *ctx, int kind);

/* Project-written autotuner: picks the kernel variants of this library for
 * order n and precision `prec` by timing them on synthetic operands of the
 * same shape on the current device -- the triangular sweeps' super-block
 * size and kernel design (the implicit operator KI1-KI3 timed as a whole,
 * FP64 or FP32 storage) and the matrix-core product tile (64x64 or 128x128,
 * an n x n x 256 product, FP64 or FP32 compute) -- and applies them: the
 * sweep choice to ctx, the tile choice process-wide.  Measurements run at
 * min(n_bucket, 32768) (n_bucket = the power of two >= n, 1024..65536);
 * they allocate and free about 2 n^2 doubles of device memory.
 * cache_path (host string, may be NULL): a JSON file keyed by (device
 * architecture, prec, n_bucket); an entry found there is applied without
 * measuring, a new measurement is added to it.  *out (host, may be NULL)
 * receives the choices.  Synchronises.  Returns 0, -1 (NULL ctx), -2
 * (n < 1), -3 (prec), GSYEIG_ENOMEM, GSYEIG_EHIP (also for an unwritable
 * cache file, after applying the measured choices). */
int gsyeig_autotune(gsyeig_ctx *ctx, int64_t n, int prec, const char *cache_path, gsyeig_tuning *out);

/* Bound on the polls of each wait in the chained (persistent) triangular
 * sweeps of KI1/KI3 on this context: 0 restores the built-in bound (2^22
 * polls).  The work-queue sweeps read the bound once per workgroup; the
 * per-tile and 64-row sweeps consult it from the 33rd poll of a wait on, so
 * there values below 32 act as 32.  A wait that runs out stores 0.0 for the
 * awaited value, marks the
 * context's wait record and lets the kernel finish, so no wait can hang the
 * GPU; the call reports GSYEIG_ESPIN.  Meant for tests of that error path
 * (a tiny bound forces expiries in a healthy run).  Synchronises; returns
 * 0, -1 (NULL ctx) or GSYEIG_EHIP. */
int gsyeig_set_spin_limit(gsyeig_ctx *ctx, unsigned limit);

/* Wait for the context's stream and report the wait record of the chained
 * sweeps enqueued by asynchronous calls (gsyeig_trsv, gsyeig_apply_op,
 * gsyeig_lanczos_run) since the last report: GSYEIG_ESPIN if one of their
 * waits expired (the record is then cleared), else 0; GSYEIG_EHIP on a
 * runtime error.  Synchronous entry points clear the record when they
 * start and report only their own waits, so call this after asynchronous
 * work whose result matters. */
int gsyeig_sync(gsyeig_ctx *ctx);

/* Bytes of device workspace gsyeig_solve needs for (n, s, opts) (host-only
 * arithmetic; no GPU call). */
int gsyeig_workspace_size(int64_t n, int64_t s, const gsyeig_opts *opts, size_t *bytes);

/* GS1 (Eq. 2; Table 1): B = U^T U.
 * U_lowprec == NULL (FP64): in place; on return the upper triangle (incl.
 * diagonal) of B holds U; the strict lower triangle of B is left untouched
 * (so it still holds B's lower half).
 * U_lowprec != NULL (mixed precision; required when opts->prec is
 * GSYEIG_MIXED): B is only read; U~ is written as FP32 to U_lowprec (device,
 * n x n row-major, leading dimension n, zeros below the diagonal).  The 64x64
 * diagonal blocks are factored in FP64; the panel products and the trailing
 * SYRK updates are FP32 matrix-core products with FP32 accumulation, so
 * U~^T U~ = B + E with |E| of order n u_32 |U~|^T |U~|.
 * Synchronises; returns 0 or the failing minor k > 0. */
int gsyeig_potrf(gsyeig_ctx *ctx, int64_t n, double *B, int64_t ldb, const gsyeig_opts *opts,
                 void *U_lowprec);

/* KI1 / KI3 (Table 1): x = U^-1 b (trans = 0) or x = U^-T b (trans = 1).
 * x may alias b.  Asynchronous. */
int gsyeig_trsv(gsyeig_ctx *ctx, int64_t n, const double *U, int64_t ldu, int trans,
                const double *b, double *x);

/* KI2 (Table 1): y = A x, A symmetric in full storage.  Read set: the
 * 64x64 tiles A_IJ with J >= I of the upper block triangle -- the tiles
 * above the diagonal once, each used for both y_I and y_J, and the 64x64
 * diagonal tiles in full (both of their triangles, so A must be symmetric
 * there); tiles below the diagonal tiles are never read.  x and y must not
 * alias.  Asynchronous. */
int gsyeig_symv(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x,
                double *y);

/* KI2 for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x
 * exactly as gsyeig_symv computes it (same kernels, same summation order,
 * so the two agree bit for bit), enqueued on `hip_stream` (a hipStream_t,
 * NULL = the null stream) with no context and no allocation.  Its scratch
 * (the tile work list and the per-tile partial sums) lives in a file-scope
 * device array of about 42 MB that each GPU the library runs on holds until
 * the process ends; n is limited to GSYEIG_NOALLOC_MAX_N (16384), larger n
 * returns GSYEIG_ETOOBIG.  Every scratch value is written before it is read
 * in each call.  All calls on one GPU share that GPU's array, so calls that
 * overlap in time on one GPU (different streams or host threads) race;
 * serialise them.  The array's device address is resolved on the first call
 * on each device (or by gsyeig_create there), which loads the library's code
 * object if the runtime has not yet done so: make one call, or create a
 * context, at set-up.  A (row-major, lda >= n) is read as by gsyeig_symv
 * (upper block triangle, diagonal tiles in full); x and y must not alias.
 * Asynchronous.  Returns 0, -2 (n < 1), -3..-6 (NULL A, lda < n, NULL x,
 * NULL y), GSYEIG_ETOOBIG or GSYEIG_EHIP. */
int gsyeig_symv_noalloc(void *hip_stream, int64_t n, const double *A, int64_t lda, const double *x, double *y);

/* GS2 (Eq. 3; Table 1, variants KE and TD of Section 2): the explicit
 * standard-form matrix C = U^-T A U^-1 for the upper Cholesky factor U
 * (row-major, ldu; only its upper triangle is read) and symmetric A (only
 * read).  Two block triangular solves with all n columns as right-hand
 * sides (2 n^3 flops of FP64 matrix-core products), a transpose between
 * them, then C = (C + C^T) / 2.  C (n x n, ldc >= n) is exactly symmetric,
 * so its column- and row-major storage coincide.  Uses n x n FP64 of
 * context workspace besides C.  Asynchronous. */
int gsyeig_form_c(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *U, int64_t ldu,
                  double *C, int64_t ldc);

/* KI1-KI3: z = U^-T (A (U^-1 w)) = C w, the implicit operator of variant KI
 * (Section 2.3).  z may alias w.  Asynchronous. */
int gsyeig_apply_op(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *U,
                    int64_t ldu, const double *w, double *z);

/* KI1-KI4 for exactly k steps (Section 2.3, Lanczos with the three-term
 * recurrence and classical Gram-Schmidt re-orthogonalisation applied twice
 * on every step, whatever opts.reorth says elsewhere):
 *   w_0 = v0/||v0||; for j < k:  z = C w_j - beta_{j-1} w_{j-1};
 *   alpha_j = w_j^T z; z -= alpha_j w_j; twice { z -= W_j (W_j^T z) };
 *   beta_j = ||z||; w_{j+1} = z / beta_j.
 * alpha, beta: device (k).  V: device n x (k+1) column-major basis, ldv >= n.
 * v0: device start vector (n).  Asynchronous. */
int gsyeig_lanczos_run(gsyeig_ctx *ctx, int64_t n, int64_t k, const double *A, int64_t lda,
                       const double *U, int64_t ldu, const double *v0, double *alpha,
                       double *beta, double *V, int64_t ldv);

/* KI5, eigen-part (Section 2.3; the Ritz values and coefficient vectors of
 * the tridiagonal Lanczos matrix):
 * the nwant smallest (which = 0) or largest (which = 1) eigenvalues of the
 * symmetric tridiagonal T_m (diagonal alpha[0..m-1], off-diagonal
 * beta[0..m-2]) by Sturm-count bisection, ascending, into theta (device,
 * nwant); and, if S != NULL, the matching orthonormal eigenvectors by
 * inverse iteration (re-orthogonalised inside clusters) into S (device,
 * m x nwant column-major, lds >= m).  Asynchronous. */
int gsyeig_tridiag_eig(gsyeig_ctx *ctx, int64_t m, const double *alpha, const double *beta,
                       int64_t nwant, int which, double *theta, double *S, int64_t lds);

/* KI1-KI5: Lanczos on C = U^-T A U^-1 until the s wanted Ritz pairs have
 * Ritz residual estimate beta_m |e_m^T s_i| <= tol ||T_m|| (checked every
 * check_every steps) or max_steps is reached.  Returns the Ritz values
 * (theta, device, s, ascending) and Ritz vectors (device, n x s
 * column-major): Y = V_m S with reorth 0 or 1; with the default partial
 * re-orthogonalisation (reorth 2) the basis is only semi-orthogonal and
 * Y = V_m R^-1 S, where V_m^T V_m = R^T R (Cholesky), so that Y is
 * orthonormal.  U is the upper Cholesky factor (row-major).
 * *steps_out (host, may be NULL) receives m.  Synchronises.
 * Returns 0, GSYEIG_ENOCONV (results are the best available; with reorth 2
 * also when V_m^T V_m lost positive definiteness, and then Y is not
 * valid), or GSYEIG_ESPIN (a chained wait of this call expired). */
int gsyeig_lanczos(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda,
                   const double *U, int64_t ldu, const gsyeig_opts *opts, double *theta,
                   double *Y, int64_t ldy, int64_t *steps_out);

/* KI1 / KI3 with U stored FP32 (the mixed-precision sweeps): x = U^-1 b or
 * U^-T b for the FP32 upper-triangular U (row-major, ldu), FP64 b, x and
 * FP64 arithmetic.  The factor is applied as U = D (I + W) over 512-row
 * diagonal super-blocks D (their inverses formed in FP64) with
 * W = D^-1 U_offdiag stored FP32, so the result is the exact solve with
 * D (I + fl32(W)), an FP32-level perturbation of U (componentwise
 * relative error of order u_32 kappa(U), not FP64 rounding).  x may alias
 * b.  Synchronises; returns GSYEIG_ESPIN if a chained wait of this call
 * expired. */
int gsyeig_trsv_lp(gsyeig_ctx *ctx, int64_t n, const float *U, int64_t ldu, int trans, const double *b,
                   double *x);

/* KI1-KI3 with A and U stored FP32 (the operator of the mixed-precision
 * Lanczos sweeps, Section 2.3's implicit C with FP32 storage):
 * z = U^-T (A (U^-1 w)) with FP64 vectors and arithmetic; U is applied as
 * by gsyeig_trsv_lp (its upper triangle) and A as by gsyeig_symv.  The
 * U^-T sweep sums the A-product's tile partials itself, in the order of
 * gsyeig_symv_lp's reduction, so z equals the three separate calls bit for
 * bit.  z may alias w.  Synchronises; returns GSYEIG_ESPIN if a chained
 * wait of this call expired. */
int gsyeig_apply_op_lp(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const float *U, int64_t ldu,
                       const double *w, double *z);

/* KI2 with A stored FP32: y = A x (FP64 x, y and arithmetic; A is read as
 * by gsyeig_symv: upper block triangle, 64x64 diagonal tiles in full).
 * Synchronises. */
int gsyeig_symv_lp(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x, double *y);

/* Block form of KI1 / KI3 used by the mixed-precision refinement:
 * X = U^-1 V (trans = 0) or U^-T V (trans = 1) for k columns (n x k
 * column-major), U FP32 upper triangular.  Products run on the FP32 matrix
 * cores with FP32 accumulation over 512-row super-blocks, so X carries FP32
 * rounding (relative error of order u_32 kappa(U)).  V is not modified.
 * Synchronises. */
int gsyeig_trsm_lp(gsyeig_ctx *ctx, int64_t n, const float *U, int64_t ldu, int trans, int64_t k,
                   const double *V, int64_t ldv, double *X, int64_t ldx);

/* Dense symmetric eigensolver for the small projected matrices of the
 * refinement (the Rayleigh-Ritz step of Section 2.3, which solves the small
 * projected problem): the nwant smallest (which = 0) or largest (which = 1)
 * eigenpairs of the symmetric N x N matrix H (device, column-major, ldh;
 * only read), N <= 8192, by Householder tridiagonalisation, Sturm bisection,
 * inverse iteration (made orthonormal by Cholesky QR twice; Gram-Schmidt in
 * clusters of near-equal values when that finds near-parallel vectors) and
 * back-transformation.
 * w (device, nwant) ascending; Q (device, N x nwant column-major, ldq)
 * orthonormal.  Synchronises. */
int gsyeig_syev_small(gsyeig_ctx *ctx, int64_t N, const double *H, int64_t ldh, int64_t nwant, int which,
                      double *w, double *Q, int64_t ldq);

/* FP64 refinement of the mixed-precision path (Rayleigh-Ritz on the
 * ORIGINAL pencil of Eq. 1 with correction expansion; the paper ran FP64
 * only, Section 3).  Starting block X0 (device, n x k column-major, k >= s,
 * 2k <= 8192; e.g. U~^-1 times Ritz vectors of the FP32-sweep Lanczos):
 *   repeat: B-orthonormalise; Rayleigh-Ritz with FP64 A X and B X;
 *           R = A X - B X Theta; stop when the wanted s pairs have
 *           eta_i = ||r_i|| / ((||A||_F + |theta_i| ||B||_F) ||x_i||)
 *           <= opts->eta_tol; else opts->refine_inner MINRES steps on the
 *           projected correction equation with the FP32 operator
 *           C~ = U~^-T A~ U~^-1 (A~ = fl32(A)) and expand the basis;
 * at most opts->refine_iters rounds.  U_lowprec: FP32 factor with
 * U~^T U~ ~ B (e.g. from gsyeig_potrf in mixed mode).  Lambda (device, s,
 * ascending) and X (device, n x s, B-orthonormal, sign-normalised as in
 * gsyeig_solve) receive the wanted pairs (s smallest / largest per
 * opts->which).  A, B and X0 are not modified.  *info (host, may be NULL):
 * eta_max (= final max eta), eta_phase1 (after the first Rayleigh-Ritz),
 * refine_iters, block_applies, block_cols, converged, t_refine_ms.
 * Synchronises.  Returns 0 if max eta <= eta_tol, else GSYEIG_ENOCONV. */
int gsyeig_refine(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t k, const double *A, int64_t lda,
                  const double *B, int64_t ldb, const float *U_lowprec, int64_t ldu, const gsyeig_opts *opts,
                  const double *X0, int64_t ldx0, double *Lambda, double *X, int64_t ldx, gsyeig_info *info);

/* BT1 (Eq. 4; Table 1): X = U^-1 Y in place for s column vectors (n x s
 * column-major, ldy >= n).  Asynchronous. */
int gsyeig_backsolve(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *U, int64_t ldu,
                     double *Y_to_X, int64_t ldy);

/* FP64 accuracy check of s pairs (Tables 3/7 metrics + per-pair backward
 * error).  B is read in full storage if Bdiag == NULL; otherwise only B's
 * strict LOWER triangle is read and Bdiag (device, n) supplies its diagonal
 * (the state gsyeig_potrf leaves B in, with the diagonal saved beforehand).
 * Results go to *out (host): eta_max, rho_f, omega, normA_f, normB_f.
 * Synchronises. */
int gsyeig_check(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda,
                 const double *B, int64_t ldb, const double *Bdiag, const double *Lambda,
                 const double *X, int64_t ldx, gsyeig_info *out);

/* The whole path GS1 -> KI1..KI5 -> BT1 -> check (Eq. 1-4).
 * FP64 mode: B is overwritten by U in its upper triangle (Section 2.1: the
 * factor overwrites B); its strict lower triangle is preserved.
 * Mixed mode (opts->prec = GSYEIG_MIXED): B is not modified; GS1 runs with
 * FP32 trailing updates into an internal FP32 factor U~, the Lanczos sweeps
 * read FP32 copies of A and U~ (FP64 vectors, alpha/beta, re-orthogonal-
 * isation and T), s + guard Ritz vectors are back-solved with U~ and
 * refined as by gsyeig_refine; info reports both phases.
 * opts->invert = 1 (A SPD): the pencil (B, A) is solved for its extreme
 * mu = 1/lambda at the other end (Sec. 3.1 used this for the MD problem),
 * then Lambda = 1/mu ascending and X rescaled to X^T B X = I; A and B are not
 * modified (FP64 mode factors a copy of A); a non-SPD A returns +k.  Returns
 * GSYEIG_ENOCONV unless the FP32-sweep Lanczos met tol AND the refinement
 * met eta_tol.  Lambda (device, s)
 * receives the eigenvalues ascending; X (device, n x s column-major,
 * ldx >= n) the B-orthonormal eigenvectors, each signed so that its entry
 * of largest magnitude (lowest index on ties) is positive.  *info (host,
 * may be NULL) receives steps, timings and the check.  Synchronises.
 * Returns 0, +k (B not SPD), GSYEIG_ENOCONV, or an error.  On
 * GSYEIG_ENOCONV *info is filled with what the run reached (in mixed mode,
 * when the Lanczos phase produced no valid Ritz vectors, only the Lanczos
 * fields, with eta_max = HUGE_VAL and no refinement). */
int gsyeig_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, const double *A, int64_t lda, double *B,
                 int64_t ldb, const gsyeig_opts *opts, double *Lambda, double *X, int64_t ldx,
                 gsyeig_info *info);

/* Row a10 of the hot path (batched driver; the 3-5 %-of-the-spectrum regime
 * of the paper's conclusions, Sec. 6): `count` independent pencils, each
 * solved by the method of gsyeig_solve with the same options.  All array
 * arguments are HOST arrays of length count holding per-instance sizes and
 * DEVICE pointers (A[i], B[i], Lambda[i], X[i]; same layouts and in-place
 * behaviour as gsyeig_solve).  Work is spread over `nstreams` (1..16) host
 * threads, each with its own worker context and HIP stream owned by `ctx`
 * (created on first use, freed by gsyeig_destroy), largest instance first.
 * opts->batch_mode 0 (default): the Cholesky factorisation (and, mixed, the
 * FP32 operator data) of each instance runs on the workers; then ONE launch
 * runs the Lanczos phase of every instance with n <= 4096 (KI1-KI4 and the
 * convergence pre-checks of KI5; one workgroup per instance, instances
 * taken from a device-side queue largest first); then the full convergence
 * check, the Ritz vectors, BT1, the refinement (mixed) and the check of
 * each instance run on the workers, an instance whose full check fails
 * going back to the Lanczos launch for more steps.  Same method, own
 * summation order: results agree with gsyeig_solve's to within the
 * convergence tolerance, not bit for bit.  This mode holds every such
 * instance's factor, basis (n x min(n, max_steps) FP64) and, mixed, FP32
 * copies of A and U at once in device memory.  Instances it cannot take
 * (n > 4096, or options other than variant KI, block 1, reorth 2, invert 0,
 * no v0) are solved as in mode 1 in the same call.  batch_mode 1: every
 * instance is a gsyeig_solve on a worker (bit for bit equal to it).
 * status[i] receives instance i's return code; infos (host, may be NULL)
 * its info (batch_mode 0: t_ki_ms is the instance's time in the shared
 * launch, t_total_ms the sum of its phases).  Synchronises.  Returns 0 if
 * every instance succeeded, else the first nonzero status in index order,
 * or a negative code for an illegal batched argument (-9: batch_mode not
 * 0 or 1). */
int gsyeig_solve_batched(gsyeig_ctx *ctx, int64_t count, const int64_t *n, const int64_t *s,
                         const double *const *A, const int64_t *lda, double *const *B,
                         const int64_t *ldb, const gsyeig_opts *opts, double *const *Lambda,
                         double *const *X, const int64_t *ldx, int64_t nstreams, int *status,
                         gsyeig_info *infos);

#ifdef __cplusplus
}
#endif

#endif /* GSYEIG_H */
