// internal.h -- shared declarations of the gfx950 solver library (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <string>
#include <vector>

#include "../../include/gsyeig.h"

// Block size of the triangular factor: diagonal blocks of U are NB x NB.
// One 64-row tile is one wavefront-width of rows and 32 KiB of FP64.
#define NB 64

// Upper bound on polls in a persistent kernel's wait on another workgroup.
// A wait that exceeds it records GSYEIG_ESPIN and the workgroup carries on,
// so a logic error can never hang the GPU.
#define SPIN_LIMIT (1u << 22)

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Control block of one persistent (chained) kernel launch: counters, then a
// staging vector (at byte offset PCTL_STAGE_OFFSET) through which solved
// values are published.  Between launches every staging entry holds
// STAGE_SENTINEL (an all-ones NaN, never produced by arithmetic); the last
// workgroup to finish restores it and resets the counters, so the block is
// ready for the next launch without any host-side memset.
struct PCtl {
    unsigned ticket;
    unsigned done;
    unsigned err;
    unsigned spin;  // bound on the polls of one wait (0 = SPIN_LIMIT); set by the host
};
#define PCTL_STAGE_OFFSET 256
#define STAGE_SENTINEL 0xFFFFFFFFFFFFFFFFull

__host__ __device__ inline double *ctl_stage(PCtl *c)
{
    return reinterpret_cast<double *>(reinterpret_cast<char *>(c) + PCTL_STAGE_OFFSET);
}

enum WsSlot {
    WS_DINV = 0,   // 3 n x NB FP64: Dinv_i = U_ii^-1, M_i, M'_i (chain blocks of the solves)
    WS_TMP1,       // n FP64
    WS_TMP2,       // n FP64
    WS_SYMV_PR,    // SYMV row partials
    WS_SYMV_PC,    // SYMV column partials
    WS_RED,        // partial sums of the Lanczos reductions
    WS_RED2,
    WS_V,          // Lanczos basis, ldv x (max_steps + 1)
    WS_T,          // alpha, beta, theta, last components, scalars
    WS_TRI,        // tridiagonal eigensolver scratch
    WS_S,          // Ritz coefficient matrix S (m x s)
    WS_Y,          // n x s blocks (Ritz vectors / check temporaries)
    WS_Y2,
    WS_BDIAG,      // saved diagonal of B
    WS_SYMVMAP,    // SYMV work list
    WS_SB,         // super-block solve data: Uinv, Uinv^T, N, N' (SB x SB per super-block)
    WS_A32,        // FP32 copy of A (mixed mode)
    WS_U32,        // FP32 Cholesky factor (mixed mode)
    WS_REFINE,     // blocks and small matrices of the FP64 refinement
    WS_RITZ,       // orthonormalisation of the Ritz coefficient matrix
    WS_ACOPY,      // working copy of A factored by the inverse-pencil solve (FP64 mode)
    WS_INV,        // mu and vectors of the inverse-pencil solve
    WS_W,          // W = blockdiag(U_SS)^-1 U_offdiag for the super-block solves (FP64 or FP32)
    WS_BLZ,        // block Lanczos: projected matrix, Ritz coefficients, blocks, kept Ritz vectors
    WS_PRO,        // omega estimates of the partial re-orthogonalisation (3 x (max_steps + 2))
    WS_PROG,       // Gram matrix V_m^T V_m of the semi-orthogonal basis and its Cholesky data
    WS_TRSVQ,      // work queues and sentinel partial buffers of the queue sweeps
    WS_CKE,        // variant KE: the explicit C = U^-T A U^-1 (n x n FP64)
    WS_CKE2,       // variant KE: the second n x n buffer of its formation
    WS_BATCH,      // batched Lanczos phase: every instance's factor data, basis and state
    WS_COUNT
};

struct gsyeig_ctx {
    hipStream_t stream;
    int device;
    void *ws[WS_COUNT];
    size_t ws_bytes[WS_COUNT];
    PCtl *ctl_n;        // persistent-kernel control blocks (+flags)
    PCtl *ctl_t;
    struct LzCtl *ctl_lz;  // the fused Lanczos step's queue (k_lanczos.hip)
    int64_t ctl_rows;   // staging capacity (rows) of each staging vector
    int64_t trsv_block; // 64: chained 64-row solves; 512: super-block solves
    int trsv_sweep;     // super-block solves: 0 = work-queue sweeps, 1 = one workgroup per tile
    int64_t trsvq_n;    // n for which WS_TRSVQ holds the queues (-1: none)
    int trsvq_nitems_n, trsvq_nitems_t;
    size_t trsvq_pbytes;  // byte offset of the partial buffers in WS_TRSVQ
    int64_t symv_map_n; // n for which WS_SYMVMAP is valid
    int64_t symv_items;
    unsigned spin_limit;  // polls per wait of the chained kernels (0 = SPIN_LIMIT)
    void *host_pinned;  // small pinned host staging area
    void *dscal;        // small device scratch (info codes, counters, check results)
    hipEvent_t ev[10];
    hipEvent_t pev[64];   // sampled per-kernel timing (4 per sampled step)
    int npev;             // events recorded since the last harvest
    int64_t prof_samples;
    double prof_ms[3];
    int64_t n_fallback;   // clustered Gram-Schmidt fallbacks of the eigenvector orthonormalisation
    int64_t fallback_why; // last reason: 1 = overlap above the threshold, 2 = Gram not positive definite,
                          // plus 10 x the calling site (syev_site)
    int syev_site;        // caller of the small eigensolver: 1 block Lanczos, 2 SVQB, 3 Rayleigh-Ritz
    gsyeig_ctx *workers[GSYEIG_MAX_STREAMS];  // batched-solve worker contexts
    hipStream_t wstreams[GSYEIG_MAX_STREAMS];
    int nworkers;
};

// ---------------------------------------------------------------- helpers
#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t _e = (expr);                         \
        if (_e != hipSuccess) return GSYEIG_EHIP;       \
    } while (0)

int ws_get(gsyeig_ctx *ctx, int slot, size_t bytes, void **out);
// device address of gsyeig_symv_noalloc's scratch array on the current device
int noalloc_scratch(void **out);
int ctl_reserve(gsyeig_ctx *ctx, int64_t rows);

// ---------------------------------------------------------------- launchers
// Each returns 0 or GSYEIG_EHIP; all are asynchronous on `st`.
// Dense FP64 tiles (MFMA): C = alpha * op(A) op(B) + beta * C.
// Layout codes: 0 = column-major, 1 = row-major, 2 = symmetric taken from the
// strict LOWER triangle of a row-major matrix with diagonal from `diag`.
struct GemmDesc {
    int64_t m, n, k;
    const void *A; int64_t lda; int a_layout;
    const void *B; int64_t ldb; int b_layout;
    void *C; int64_t ldc; int c_layout;
    double alpha, beta;
    const double *a_diag;  // for a_layout == 2
    int upper_only;        // write only C(i, j) with i <= j (logical indices)
    int a_f32, b_f32, c_f32;  // storage of A / B / C is FP32 (else FP64)
    int f32;                  // FP32 compute (MFMA f32, FP32 accumulation); else FP64
    int splitk;               // > 1: split K into chunks summed through `part`
    double *part;             // split-K scratch: gemm_splitk_parts(d) * m * n doubles
    int64_t batch;            // > 1: that many products, operands advanced by the strides
    int64_t stride_a, stride_b, stride_c;  // elements between consecutive products
};
int launch_gemm(const GemmDesc &d, hipStream_t st);
int launch_gemm_f64(const GemmDesc &d, hipStream_t st);
int64_t gemm_splitk_parts(const GemmDesc &d);
// process-wide tile choice of launch_gemm: 128x128 tiles when m and n are
// both >= the given size (0: 64x64 tiles only); set by the autotuner
void gemm_set_big_min(int64_t m);
int64_t gemm_big_min();

// autotuner (autotune.hip): the JSON cache and synthetic operands
struct TuneEntry {
    int prec;
    int64_t n_bucket;
    int trsv_block, trsv_sweep;
    int64_t gemm_big_min;
    double op_ms, gemm_ms;
};
int tune_cache_load(const char *path, const char *arch, std::vector<TuneEntry> *out, std::string *others);
int tune_cache_store(const char *path, const char *arch, const std::vector<TuneEntry> &entries,
                     const std::string &others);
int launch_synth_operands(double *U, double *A, int64_t ld, int64_t n, uint64_t seed, hipStream_t st);

int launch_diag_inv(const double *U, int64_t ldu, int64_t n, double *Dinv, hipStream_t st);
// super-block solves (k_trsv_w.hip): Uinv_SS and its transpose per 512-row super-block
int64_t trsv_sb_rows();  // rows of a diagonal super-block (512)
int launch_sb_inverses(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *Uinv, double *UinvT,
                       hipStream_t st);
int launch_sb_inverses_f32(const float *U, int64_t ldu, int64_t n, const double *Dinv, double *Uinv,
                           double *UinvT, hipStream_t st);
// sweeps on U = D (I + W) (k_trsv_w.hip); sbw = [Uinv | Uinv^T | W_{S-1,S}^T] per super-block
size_t trsv_w_side_bytes(int64_t n);
int launch_make_w(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *sbw, double *W, int64_t ldw,
                  hipStream_t st);
int launch_make_w_f32(const float *U, int64_t ldu, int64_t n, const double *Dinv, double *sbw, float *W,
                      int64_t ldw, hipStream_t st);
int launch_trsv_w_n(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                    PCtl *ctl, hipStream_t st);
int launch_trsv_w_t(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                    PCtl *ctl, hipStream_t st);
int launch_trsv_w_n_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                        PCtl *ctl, hipStream_t st);
int launch_trsv_w_t_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                        PCtl *ctl, hipStream_t st);
int launch_potrf_diag_f32(float *B, int64_t ldb, int64_t n, int64_t kb, double *Dinv, int *info,
                          hipStream_t st);
int launch_diag_inv_f32(const float *U, int64_t ldu, int64_t n, double *Dinv, hipStream_t st);
int launch_backsolve_f32(const float *U, int64_t ldu, int64_t n, int64_t s, const double *Dinv,
                         double *Y, int64_t ldy, hipStream_t st);
int launch_upper_to_f32(const double *B, int64_t ldb, float *W, int64_t ldw, int64_t n, hipStream_t st);
int launch_symv_f32(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x,
                    double *y);
// KI2's tile pass alone (partials Pr / Pc, maxch slots of ch tiles per block
// row) and KI3 taking those partials as its right-hand side
int launch_symv_partials(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x, double **Pr,
                         double **Pc, int *maxch, int *ch);
int launch_symv_partials_f32(gsyeig_ctx *ctx, int64_t n, const float *A, int64_t lda, const double *x, double **Pr,
                             double **Pc, int *maxch, int *ch);
int launch_trsv_w_t_rows(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *Pr,
                         const double *Pc, int maxch, int ch, double *x, PCtl *ctl, hipStream_t st);
int launch_trsv_w_t_rows_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *Pr,
                             const double *Pc, int maxch, int ch, double *x, PCtl *ctl, hipStream_t st);
int launch_to_f32(const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows, int64_t cols,
                  hipStream_t st);
// work-queue sweeps on U = D (I + W) (k_trsv_q.hip); b == nullptr in KI3:
// the right-hand side is the SYMV tile partials Pr / Pc
struct TrsvQ {
    const int2 *items_n; int nitems_n;
    const int2 *items_t; int nitems_t;
    double *P, *Q;         // sentinel-initialised partials, nblk x nsb x 64 each
    int nsb;
};
int trsvq_prepare(gsyeig_ctx *ctx, int64_t n, TrsvQ *q);
int launch_trsvq_n(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x, PCtl *ctl,
                   const TrsvQ &q, hipStream_t st);
int launch_trsvq_n_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, double *x,
                       PCtl *ctl, const TrsvQ &q, hipStream_t st);
int launch_trsvq_t(const double *W, int64_t ldw, int64_t n, const double *sbw, const double *b, const double *Pr,
                   const double *Pc, int maxch, int ch, double *x, PCtl *ctl, const TrsvQ &q, hipStream_t st);
int launch_trsvq_t_f32(const float *W, int64_t ldw, int64_t n, const double *sbw, const double *b, const double *Pr,
                       const double *Pc, int maxch, int ch, double *x, PCtl *ctl, const TrsvQ &q, hipStream_t st);
// M holds [M_i | M'_i] for all blocks (see launch_make_m)
int launch_make_m(const double *U, int64_t ldu, int64_t n, const double *Dinv, double *M,
                  hipStream_t st);
int launch_trsv_n(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *M,
                  const double *b, double *x, PCtl *ctl, hipStream_t st);
int launch_trsv_t(const double *U, int64_t ldu, int64_t n, const double *Dinv, const double *M,
                  const double *b, double *x, PCtl *ctl, hipStream_t st);
int launch_symv(gsyeig_ctx *ctx, int64_t n, const double *A, int64_t lda, const double *x,
                double *y);
int launch_potrf_diag(double *B, int64_t ldb, int64_t n, int64_t kb, double *Dinv, int *info,
                      hipStream_t st);
int launch_copy_diag(const double *B, int64_t ldb, int64_t n, double *d, hipStream_t st);
int launch_backsolve(const double *U, int64_t ldu, int64_t n, int64_t s, const double *Dinv,
                     double *Y, int64_t ldy, hipStream_t st);
int launch_sign_normalise(double *X, int64_t ldx, int64_t n, int64_t s, hipStream_t st);

// Lanczos vector kernels (KI4)
int lz_red_parts(int64_t n);
int lz_norm_parts(int64_t n);
int launch_fill_splitmix(double *v, int64_t n, uint64_t seed, hipStream_t st);
int launch_copy(const double *src, double *dst, int64_t n, hipStream_t st);
int launch_normalize_into(const double *v, double *w, int64_t n, double *part, double *norm_out,
                          hipStream_t st);
// z0part (optional, lz_z0_parts(n) entries): partial sums of the projected z^2
int launch_lz_alpha(double *z, const double *wprev, const double *wk, double *alpha,
                    const double *beta, int64_t k, int64_t n, double *part, hipStream_t st,
                    double *z0part = nullptr);
// run (optional device flag): the pass does nothing when *run == 0
int launch_cgs_pass(const double *V, int64_t ldv, int64_t n, int64_t kcols, double *z, double *part,
                    double *h, double *normpart, hipStream_t st, const int *run = nullptr);
int lz_z0_parts(int64_t n);
// Control block of the fused post-operator Lanczos step (k_lanczos.hip):
// queue ticket, workgroups done, sticky wait-expiry flag, spin bound (0 =
// SPIN_LIMIT), phase counters; zero between launches (the last workgroup
// resets it).
// Batched Lanczos phase (k_lzb.hip): one workgroup per instance, n <= LZB_NMAX.
#define LZB_NMAX 4096
struct LzbDesc {
    // problem and operator (rows contiguous: element (r, c) at M[r * ld + c];
    // U and A 16-byte aligned, ld even, n rows of ld elements below 2^31
    // bytes: the kernel reads them through 32-bit buffer offsets)
    int64_t n, s, nvec, mmax, every;
    int which;
    double tol;
    const void *U; int64_t ldu;   // Cholesky factor, upper triangle (float or double)
    const double *Dinv;           // FP64 inverses of U's 64 x 64 diagonal blocks
    const void *A; int64_t lda;   // symmetric A, upper triangle read (float or double)
    uint64_t seed;                // start vector w_0 = SplitMix64(seed), normalised
    // Lanczos data
    double *V; int64_t ldv;       // w_0 .. w_m, column j at V + j * ldv
    double *alpha, *beta;         // mmax each
    double *om; int64_t ldom;     // three omega columns of ldom >= mmax + 2
    double *chk;                  // lzb_scratch_doubles(n, mmax) doubles
    // state kept between launches (zero before the first)
    int64_t k, next_check, prev_m;
    double prev_rho, anorm;
    int forced, reorth_steps;
    int status;                   // 0 running; 1 the pre-check passed on all s wanted
                                  // values; 2 on the innermost ones (full check due);
                                  // 3 the step cap mmax was reached; 4 the basis lost
                                  // orthogonality (Gram-Schmidt lengthened z)
    int64_t ticks;                // device wall-clock ticks (100 MHz) spent
};
int64_t lzb_scratch_doubles(int64_t n, int64_t mmax);
int launch_lzb(LzbDesc *desc, const int *order, int count, unsigned *next, int f32, hipStream_t st);

struct LzCtl {
    unsigned ticket, done, err, spin;
    unsigned ph[12];
};
// Two launches after the operator on each step with partial
// re-orthogonalisation: alpha_k, the omega recurrence and (when it asks for
// none) beta_k and w_{k+1}; then, only when it asks for them, two
// Gram-Schmidt passes and w_{k+1}.  slots (lz_post_slots doubles) and cgs
// (lz_cgs_doubles(n, kcap), k + 1 <= kcap) all STAGE_SENTINEL before the
// first step of a run; GSYEIG_ETOOBIG for n > 2^21.
int launch_lz_post(double *z, const double *wprev, const double *wk, double *wnext, double *alpha, double *beta,
                   int64_t k, int64_t n, const double *V, int64_t ldv, const double *omP, const double *omC,
                   double *omN, double *anorm, int *flag, double *slots, double *cgs, int64_t kcap, LzCtl *ctl,
                   hipStream_t st);
int lz_post_slots();
int64_t lz_cgs_doubles(int64_t n, int64_t kcap);
// *flag = 1 if the first pass shrank z below 1/sqrt(2) of its norm
int launch_reorth_flag(const double *z0part, int64_t n, const double *z1part, int *flag, hipStream_t st);
int launch_lz_normalize(const double *z, double *wnext, double *beta, int64_t k, int64_t n,
                        const double *normpart, hipStream_t st);
// partial re-orthogonalisation: start of the omega estimates; flag: [0]
// orthogonalise this step, [1] count of such steps, [2] force the next
int launch_pro_init(double *om0, double *anorm, int *flag, hipStream_t st);

// tridiagonal eigensolver (KI5)
int launch_tri_bisect(const double *alpha, const double *beta, int64_t m, int64_t nwant, int which,
                      double *theta, hipStream_t st);
int launch_tri_vectors(const double *alpha, const double *beta, int64_t m, int64_t nwant,
                       const double *theta, double *S, int64_t lds, double *scratch, int clustered,
                       double *lastcomp, hipStream_t st);
int launch_tri_bisect_range(const double *alpha, const double *beta, int64_t m, int64_t first,
                            int64_t count, int which, double *theta, hipStream_t st);
// tn_extra = 1: theta[nwant + 1] also enters the ||T|| estimate
int launch_conv_count(const double *theta, const double *lastcomp, const double *beta_m,
                      int64_t nwant, int64_t i0, int64_t cnt, int tn_extra, double tol, int *nconv,
                      hipStream_t st, double *maxratio = nullptr);

// mixed-precision refinement (k_refine.hip)
struct RefineOp {          // the FP32 operator C~ = U~^-T A~ U~^-1
    const float *U32; int64_t ldu32;
    const double *sb;      // super-block inverses of U~ (FP64)
    const float *A32; int64_t lda32;
};
struct RefineCfg {
    double eta_tol;        // stop when max eta over the wanted pairs <= eta_tol
    int64_t max_iters;     // correction rounds
    int64_t inner;         // MINRES steps per round
};
struct RefineStats {
    int64_t iters, block_applies, kept, nconv;
    double eta0, eta;
};
size_t refine_bytes(int64_t n, int64_t k);
int refine_x0(gsyeig_ctx *ctx, int64_t n, int64_t k, double **X0, int64_t *ld);
int refine_run(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t k, int which, const double *A, int64_t lda,
               const double *B, int64_t ldb, const RefineOp &op, const RefineCfg &cfg, double *Lambda,
               double *X, int64_t ldx, RefineStats *out);
int launch_trsm_sb_f32(int trans, const float *U, int64_t ldu, int64_t n, const double *sb, double *V,
                       int64_t ldv, double *X, int64_t ldx, int64_t k, hipStream_t st);
int launch_trsm_sb(int trans, const void *U, int u_f32, int64_t ldu, int64_t n, const double *sb, double *V,
                   int64_t ldv, double *X, int64_t ldx, int64_t k, int f32, hipStream_t st);
// The same on U = D (I + W) (W from launch_make_w / _f32, FP64 or FP32): the
// diagonal super-blocks as one batched product, the chain only the
// off-diagonal updates.  trans = 0 keeps V; trans = 1 destroys it.
int launch_trsm_w(int trans, const void *W, int w_f32, int64_t ldw, int64_t n, const double *sb, double *V,
                  int64_t ldv, double *X, int64_t ldx, int64_t k, int f32, hipStream_t st);
int launch_blk_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, int64_t k,
                    hipStream_t st);
int launch_identity(double *X, int64_t ld, int64_t r, hipStream_t st);
int launch_invert_pairs(const double *mu, const double *Xin, int64_t ldi, double *lam, double *Xout,
                        int64_t ldo, int64_t n, int64_t s, hipStream_t st);   // r x r identity, column-major
int launch_accum_info(const int *src, int *dst, hipStream_t st);        // *dst = *src if *dst == 0
int launch_flag_offdiag(const double *G, int64_t r, double thresh, int *flag, hipStream_t st);
size_t syev_small_scratch(int64_t N, int64_t nwant);
// ctx != NULL: eigenvectors by independent inverse iteration made orthonormal
// by Cholesky QR twice, the clustered Gram-Schmidt path only when that finds
// near-parallel vectors (synchronises); ctx == NULL: always clustered.
// floor_rel > 0 (which = 0): eigenvectors of eigenvalues with w + floor_shift
// <= floor_rel * (max + floor_shift) are not wanted (computed, but not
// orthonormalised or checked).
int syev_small(gsyeig_ctx *ctx, int64_t N, double *H, int64_t nwant, int which, double *w, double *Q,
               double *scratch, hipStream_t st, double floor_rel = 0.0, double floor_shift = 0.0);
// Cholesky QR twice on the nw columns of S (m x nw, column-major); *info_d
// != 0 when the Gram matrix was not positive definite or two columns
// overlapped by more than 0.5 (two device ints)
int orthonormalise_cols(gsyeig_ctx *ctx, int64_t m, int64_t nw, double *S, int64_t lds, int *info_d);
int64_t syev_small_max();
// syev_small without its order limit (the n x n C of variant TD)
int syev_dense(gsyeig_ctx *ctx, int64_t N, double *H, int64_t nwant, int which, double *w, double *Q,
               double *scratch, hipStream_t st, double floor_rel = 0.0, double floor_shift = 0.0);

// block Lanczos with thick restart (blz.hip)
struct BlkOp {             // C = U^-T A U^-1 on blocks (TRSM, SYMM on the matrix cores)
    const void *U; int u_f32; int64_t ldu;
    const void *W; int w_f32; int64_t ldw;   // U = D (I + W) when W != NULL (then U is not read)
    const double *sb;      // super-block inverses of U (FP64)
    const void *A; int a_f32; int64_t lda;
    int f32;               // FP32 products with FP32 accumulation (else FP64)
};
struct BlzResult {
    int64_t steps;         // operator applications (columns)
    int64_t nconv, restarts, breakdowns, basis, keep;
    float t_loop_ms, t_ritz_ms;
    double t_rr_ms;        // projected eigen-solves (inside the loop)
    int64_t rr_count;
};
size_t blz_bytes(int64_t n, int64_t s, int64_t nvec, const gsyeig_opts *o);
int blz_check_dims(int64_t n, int64_t s, int64_t nvec, const gsyeig_opts *o);
int blz_solve(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t nvec, const BlkOp &op, const gsyeig_opts *o,
              double *theta_out, double *Y, int64_t ldy, BlzResult *res);

// GS2 of variant KE (k_ke.hip): C = U^-T A U^-1, column-major (= row-major,
// C symmetric); W == nullptr: the solves use U with its super-block inverses
int launch_transpose(const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t n, hipStream_t st);
int launch_symmetrise(double *C, int64_t ldc, int64_t n, hipStream_t st);
int form_c(const double *A, int64_t lda, const double *U, int64_t ldu, const double *W, int64_t ldw,
           const double *sb, int64_t n, double *C, int64_t ldc, double *T, int64_t ldt, hipStream_t st);

// accuracy check
int fro_parts(int64_t n);
int launch_fro_norm_parts(const double *A, int64_t lda, int64_t n, int mode, const double *diag,
                          double *part, hipStream_t st);
int launch_check_cols(const double *AX, const double *BX, int64_t ldr, const double *X, int64_t ldx,
                      int64_t n, int64_t s, const double *lam, double *out, hipStream_t st);
int launch_check_finalize(const double *cols, int64_t s, const double *G, int64_t ldg,
                          const double *partA, int PA, const double *partB, int PB,
                          const double *lam, double *res, hipStream_t st);
