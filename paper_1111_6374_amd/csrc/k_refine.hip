// k_refine.hip -- FP64 refinement of the mixed-precision path.
//
// The paper runs KI in FP64 only (Section 2.3, Table 1).  In mixed mode the
// Lanczos sweeps use FP32 copies of A and U, so the Ritz pairs solve a
// nearby pencil; the refinement here wins the FP64 result back on the
// ORIGINAL pencil (A, B) of Eq. 1:
//
//   X <- B-orthonormal basis of the current block (SVQB: scaled Gram
//        matrix, its eigenvectors, small directions dropped);
//   Rayleigh-Ritz: H = Z^T A Z, H Q = Q Theta, X = Z Q            (FP64)
//   R = A X - B X Theta, eta_i = ||r_i|| / ((||A||_F + |theta_i| ||B||_F) ||x_i||)
//   stop when max eta over the wanted pairs <= tol; otherwise
//   correction: with U~ the FP32 factor (B ~ U~^T U~), y-space residual
//   rho_i = U~^-T r_i and the projector P = I - Q_y Q_y^T onto the
//   complement of Q_y = U~ X, a few MINRES steps (Paige and Saunders, 1975)
//   on  P (C~ - theta_i I) P g_i = -P rho_i  for every column at once, with
//   C~ = U~^-T A~ U~^-1 applied as FP32 block products on the matrix cores
//   (TRSM, SYMM, TRSM with FP32 accumulation); d_i = U~^-1 g_i;
//   Z = [X, D] with D made B-orthogonal to X, then Rayleigh-Ritz again.
//
// Accuracy is decided by the FP64 steps (A X, B X, the projected matrices,
// the residual); the FP32 part only changes how fast the loop converges.
//
// The small projected eigenproblems (order <= 8192) are solved by a
// Householder tridiagonalisation (one workgroup up to order 192, the whole
// GPU above), the tridiagonal bisection/inverse-iteration kernels of the
// Lanczos path with Cholesky-QR orthonormalisation, and the reflectors
// applied back.
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace {

constexpr int CHUNK = 4096;        // rows per partial sum in column reductions
constexpr int SYTRD_LDS = 256;     // largest order reduced by the one-workgroup kernel
constexpr int SYTRD_MAX = 8192;    // largest order of the small eigensolver

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

#define RTRY_HIP(expr)           \
    do {                         \
        int _rc = (expr);        \
        if (_rc) return _rc;     \
    } while (0)

__device__ __forceinline__ double block_sum256(double v, double *sb)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sb[0] + sb[1]) + (sb[2] + sb[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum1024(double v, double *sb)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < 16; ++w) r += sb[w];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ column blocks
// Blocks are n x k column-major with leading dimension ld; grid.y = column.

// part[c * nch + b] = sum over the rows of chunk b of X[:, c] * Y[:, c]
__global__ __launch_bounds__(256) void k_col_dot_parts(const double *X, const double *Y, int64_t ld,
                                                       int64_t n, double *part, int nch)
{
    __shared__ double sb[4];
    const int b = blockIdx.x;
    const int64_t c = blockIdx.y;
    const double *x = X + c * ld, *y = Y + c * ld;
    const int64_t r0 = (int64_t)b * CHUNK;
    const int64_t r1 = (r0 + CHUNK < n) ? r0 + CHUNK : n;
    double v = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) v = fma(x[i], y[i], v);
    v = block_sum256(v, sb);
    if (threadIdx.x == 0) part[c * nch + b] = v;
}

// out[c] = sum_b part[c * nch + b] (fixed order), or its square root
__global__ void k_col_reduce(const double *part, int nch, int64_t k, double *out, int sq)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    double s = 0.0;
    for (int b = 0; b < nch; ++b) s += part[c * nch + b];
    out[c] = sq ? sqrt(s) : s;
}

__global__ void k_blk_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) dst[c * ldd + i] = src[c * lds + i];
}

__global__ void k_blk_zero(double *X, int64_t ld, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) X[(int64_t)blockIdx.y * ld + i] = 0.0;
}

// R = AX - theta_c BX
__global__ void k_resid(const double *AX, const double *BX, int64_t ld, int64_t n, const double *theta,
                        double *R)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) R[c * ld + i] = fma(-theta[c], BX[c * ld + i], AX[c * ld + i]);
}

// dst = sgn * scale_c * src
__global__ void k_scale_cols(const double *src, double *dst, int64_t ld, int64_t n, const double *scale,
                             double sgn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) dst[c * ld + i] = sgn * scale[c] * src[c * ld + i];
}

// p -= theta_c v
__global__ void k_shift_sub(double *p, const double *v, int64_t ld, int64_t n, const double *theta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i < n) p[c * ld + i] = fma(-theta[c], v[c * ld + i], p[c * ld + i]);
}

// MINRES state, k entries per field
enum { MR_BETA, MR_C1, MR_S1, MR_C2, MR_S2, MR_PHI, MR_EPS, MR_DELTA, MR_GINV, MR_TAU, MR_VSCALE,
       MR_ALPHA, MR_NRM, MR_FIELDS };

// Lanczos step of MINRES: p -= alpha_c v + beta_c vprev; partial sums of p^2
__global__ __launch_bounds__(256) void k_mr_lanczos(double *p, const double *v, const double *vp,
                                                    int64_t ld, int64_t n, const double *st, int64_t k,
                                                    double *part, int nch)
{
    __shared__ double sb[4];
    const int b = blockIdx.x;
    const int64_t c = blockIdx.y;
    const double al = st[MR_ALPHA * k + c], be = st[MR_BETA * k + c];
    double *pc = p + c * ld;
    const double *vc = v + c * ld, *vpc = vp + c * ld;
    const int64_t r0 = (int64_t)b * CHUNK;
    const int64_t r1 = (r0 + CHUNK < n) ? r0 + CHUNK : n;
    double acc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) {
        const double x = pc[i] - al * vc[i] - be * vpc[i];
        pc[i] = x;
        acc = fma(x, x, acc);
    }
    acc = block_sum256(acc, sb);
    if (threadIdx.x == 0) part[c * nch + b] = acc;
}

// Givens bookkeeping of MINRES for every column (one thread per column):
// column k of the extended tridiagonal is (beta_k, alpha_k, beta_{k+1});
// the two previous rotations are applied, a new one annihilates beta_{k+1}.
__global__ void k_mr_scalars(int64_t k, double *st)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    const double al = st[MR_ALPHA * k + c];
    const double be = st[MR_BETA * k + c];
    const double bn = st[MR_NRM * k + c];   // beta_{k+1} = ||p||
    const double c1 = st[MR_C1 * k + c], s1 = st[MR_S1 * k + c];
    const double c2 = st[MR_C2 * k + c], s2 = st[MR_S2 * k + c];
    const double eps = s2 * be;
    const double dp = c2 * be;
    const double delta = c1 * dp + s1 * al;
    const double gbar = -s1 * dp + c1 * al;
    const double gam = hypot(gbar, bn);
    double cn = 1.0, sn = 0.0, ginv = 0.0;
    if (gam > 0.0) {
        cn = gbar / gam;
        sn = bn / gam;
        ginv = 1.0 / gam;
    }
    const double phi = st[MR_PHI * k + c];
    st[MR_TAU * k + c] = cn * phi;
    st[MR_PHI * k + c] = -sn * phi;
    st[MR_EPS * k + c] = eps;
    st[MR_DELTA * k + c] = delta;
    st[MR_GINV * k + c] = ginv;
    st[MR_C2 * k + c] = c1;
    st[MR_S2 * k + c] = s1;
    st[MR_C1 * k + c] = cn;
    st[MR_S1 * k + c] = sn;
    st[MR_BETA * k + c] = bn;
    st[MR_VSCALE * k + c] = (bn > 0.0) ? 1.0 / bn : 0.0;
}

// w_k = (v_k - delta w_{k-1} - eps w_{k-2}) / gamma  (into the w_{k-2} buffer);
// g += tau w_k;  v_{k+1} = p / beta_{k+1}  (in place in p)
__global__ void k_mr_update(const double *v, const double *w, double *wp, double *g, double *p, int64_t ld,
                            int64_t n, const double *st, int64_t k)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (i >= n) return;
    const int64_t o = c * ld + i;
    const double wn = (v[o] - st[MR_DELTA * k + c] * w[o] - st[MR_EPS * k + c] * wp[o]) * st[MR_GINV * k + c];
    wp[o] = wn;
    g[o] = fma(st[MR_TAU * k + c], wn, g[o]);
    p[o] *= st[MR_VSCALE * k + c];
}

// start of MINRES: beta_1 = ||b|| in st[MR_NRM]; rotations = identity
__global__ void k_mr_init(int64_t k, double *st)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= k) return;
    const double b1 = st[MR_NRM * k + c];
    st[MR_BETA * k + c] = 0.0;
    st[MR_C1 * k + c] = 1.0;
    st[MR_S1 * k + c] = 0.0;
    st[MR_C2 * k + c] = 1.0;
    st[MR_S2 * k + c] = 0.0;
    st[MR_PHI * k + c] = b1;
    st[MR_VSCALE * k + c] = (b1 > 0.0) ? 1.0 / b1 : 0.0;
}

// eta_c = sqrt(r2_c) / ((nA + |theta_c| nB) sqrt(x2_c)) for every column;
// out[0] = max over the wanted columns [w0, w0 + s), out[1] = count <= tol
__global__ __launch_bounds__(256) void k_eta(const double *r2, const double *x2, const double *theta,
                                             int64_t k, int64_t w0, int64_t s, const double *norms,
                                             double tol, double *eta, double *out)
{
    __shared__ double sm[4];
    __shared__ double sc[4];
    double mx = 0.0, cnt = 0.0;
    for (int64_t c = threadIdx.x; c < k; c += 256) {
        const double den = (norms[0] + fabs(theta[c]) * norms[1]) * sqrt(x2[c]);
        const double e = (den > 0.0) ? sqrt(r2[c]) / den : 0.0;
        eta[c] = e;
        if (c >= w0 && c < w0 + s) {
            mx = fmax(mx, e);
            cnt += (e <= tol) ? 1.0 : 0.0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        cnt += __shfl_xor(cnt, o);
    }
    if ((threadIdx.x & 63) == 0) {
        sm[threadIdx.x >> 6] = mx;
        sc[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
        out[1] = (sc[0] + sc[1]) + (sc[2] + sc[3]);
    }
}

__global__ void k_identity(double *X, int64_t ld, int64_t r)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r * r) return;
    const int64_t i = t % r, j = t / r;
    X[j * ld + i] = (i == j) ? 1.0 : 0.0;
}

// *flag = -1 if any |G_ij - delta_ij| > thresh (G: r x r)
__global__ void k_flag_offdiag(const double *G, int64_t r, double thresh, int *flag)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r * r) return;
    const int64_t i = t % r, j = t / r;
    const double d = G[t] - ((i == j) ? 1.0 : 0.0);
    if (fabs(d) > thresh || d != d) atomicCAS(flag, 0, -1);
}

__global__ void k_accum_info(const int *src, int *dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *src != 0 && *dst == 0) *dst = *src;
}

// Pairs (mu_i, x_i) of the inverse pencil, mu ascending, x_i^T A x_i = 1 ->
// pairs of (A, B): lambda_i = 1 / mu_{s-1-i} (ascending when all mu > 0),
// x_i scaled by sqrt(|lambda_i|) so that x_i^T B x_i = 1.
__global__ void k_invert_pairs(const double *mu, const double *Xin, int64_t ldi, double *lam, double *Xout,
                               int64_t ldo, int64_t n, int64_t s)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t c = blockIdx.y;
    const double m = mu[s - 1 - c];
    const double l = 1.0 / m;
    if (i == 0) lam[c] = l;
    if (i < n) Xout[c * ldo + i] = sqrt(fabs(l)) * Xin[(s - 1 - c) * ldi + i];
}

// ||A||_F from the row partials of k_fro_parts
__global__ void k_sum_sqrt(const double *part, int np, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < np; ++i) s += part[i];
    *out = sqrt(s);
}

// H = (H + H^T) / 2 in place (N x N, column-major, leading dimension ld)
__global__ void k_symmetrise(double *H, int64_t ld, int64_t N)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * N) return;
    const int64_t i = t % N, j = t / N;
    if (i >= j) return;
    const double v = 0.5 * (H[j * ld + i] + H[i * ld + j]);
    H[j * ld + i] = v;
    H[i * ld + j] = v;
}

// H(i, i) += a  (N x N, ld)
__global__ void k_diag_shift(double *H, int64_t ld, int64_t N, double a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) H[i * ld + i] += a;
}

// v[i] += a
__global__ void k_vec_shift(double *v, int64_t n, double a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] += a;
}

// Gram matrix G (r x r): dsc_i = G_ii^-1/2 (0 for a non-positive diagonal)
__global__ void k_gram_diag(const double *G, int64_t r, double *dsc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r) return;
    const double gi = G[i * r + i];
    dsc[i] = gi > 0.0 ? 1.0 / sqrt(gi) : 0.0;
}

// G <- diag(dsc) G diag(dsc)
__global__ void k_gram_apply(double *G, int64_t r, const double *dsc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r * r) return;
    const int64_t i = t % r, j = t / r;
    G[t] *= dsc[i] * dsc[j];
}

// W(i, c) = dsc_i V(i, c0 + c) / sqrt(sig_{c0 + c}),  c < rk  (V: r x r, ascending)
__global__ void k_svqb_coef(const double *V, int64_t r, const double *sig, const double *dsc, int64_t c0,
                            int64_t rk, double *W)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= r * rk) return;
    const int64_t i = t % r, c = t / r;
    W[c * r + i] = dsc[i] * V[(c0 + c) * r + i] / sqrt(sig[c0 + c]);
}

// ------------------------------------------------------ small eigensolver
// Householder reduction of a symmetric N x N matrix (column-major, full
// storage, ld) by one workgroup: W = Q T Q^T, Q = H_0 H_1 ... H_{N-3},
// H_j = I - tau_j v_j v_j^T on rows j+1..N-1; v_j (v_j[0] = 1) is left in
// column j below the diagonal.  d = diag(T), e = sub-diagonal of T.
__global__ __launch_bounds__(1024) void k_sytrd(double *W, int64_t ldw, int N, double *d, double *e,
                                                double *tau)
{
    __shared__ double v[SYTRD_LDS];
    __shared__ double q[SYTRD_LDS];
    __shared__ double red[16];
    const int tid = threadIdx.x;
    for (int j = 0; j + 2 < N; ++j) {
        const int m = N - j - 1;
        double *col = W + (int64_t)j * ldw + (j + 1);
        double ss = 0.0;
        for (int t = tid; t < m; t += 1024) {
            const double xv = col[t];
            v[t] = xv;
            if (t > 0) ss = fma(xv, xv, ss);
        }
        ss = block_sum1024(ss, red);
        const double alpha = v[0];
        double tj = 0.0, ej = alpha, scale = 0.0;
        if (ss > 0.0) {
            const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
            tj = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
            ej = beta;
        }
        if (tid == 0) {
            tau[j] = tj;
            e[j] = ej;
        }
        if (tj == 0.0) {
            __syncthreads();
            continue;
        }
        for (int t = tid; t < m; t += 1024) {
            const double vt = (t == 0) ? 1.0 : v[t] * scale;
            v[t] = vt;
            col[t] = vt;
        }
        __syncthreads();
        // p = tau A22 v, K = tau/2 p^T v, q = p - K v
        double *A22 = W + (int64_t)(j + 1) * ldw + (j + 1);
        double pv = 0.0;
        for (int t = tid; t < m; t += 1024) {
            double acc = 0.0;
            for (int l = 0; l < m; ++l) acc = fma(A22[(int64_t)l * ldw + t], v[l], acc);
            const double pt = tj * acc;
            q[t] = pt;
            pv = fma(pt, v[t], pv);
        }
        const double K = 0.5 * tj * block_sum1024(pv, red);
        for (int t = tid; t < m; t += 1024) q[t] = fma(-K, v[t], q[t]);
        __syncthreads();
        // A22 -= v q^T + q v^T
        for (int l = 0; l < m; ++l) {
            const double vl = v[l], ql = q[l];
            for (int t = tid; t < m; t += 1024) {
                double *a = &A22[(int64_t)l * ldw + t];
                *a = *a - v[t] * ql - q[t] * vl;
            }
        }
        __syncthreads();
    }
    for (int j = tid; j < N; j += 1024) d[j] = W[(int64_t)j * ldw + j];
    if (tid == 0 && N >= 2) {
        e[N - 2] = W[(int64_t)(N - 2) * ldw + (N - 1)];
        tau[N - 2] = 0.0;
    }
}

// The same reduction spread over the whole GPU: per column j, one
// workgroup (k_trd_col) finishes q_{j-1}, applies update j-1 to column j
// and forms reflector j; then a grid of tiles (k_trd_upd) applies update
// j-1 to the trailing columns and, in the same pass over the updated
// entries, forms the partial products of p_j = tau_j A22 v_j.  The matrix
// is read and written once per column.  Reflectors, d, e and tau are left
// exactly as k_sytrd leaves them.
//   vbuf: 2 x N (v_j in vbuf[j % 2], absolute row index), qbuf: N,
//   ppart: ceil(N / TRD_TC) x N partial sums of p_j.
constexpr int TRD_TC = 64;  // trailing columns per tile of k_trd_upd

__global__ __launch_bounds__(1024) void k_trd_col(double *W, int64_t ldw, int N, int j, double *d, double *e,
                                                  double *tau, double *vbuf, double *qbuf, const double *ppart,
                                                  int npart, int last)
{
    __shared__ double red[16];
    const int tid = threadIdx.x;
    if (N == 1) {
        if (tid == 0) d[0] = W[0];
        return;
    }
    const double *vprev = vbuf + (int64_t)((j + 1) & 1) * N;
    double *vcur = vbuf + (int64_t)(j & 1) * N;
    const double tp = (j > 0) ? tau[j - 1] : 0.0;
    if (tp != 0.0) {
        // p_{j-1} (tau included) on rows j.., K = tau/2 p^T v, q = p - K v
        double pv = 0.0;
        for (int t = j + tid; t < N; t += 1024) {
            double p = 0.0;
            for (int c = 0; c < npart; ++c) p += ppart[(int64_t)c * N + t];
            qbuf[t] = p;
            pv = fma(p, vprev[t], pv);
        }
        const double K = 0.5 * tp * block_sum1024(pv, red);
        for (int t = j + tid; t < N; t += 1024) qbuf[t] = fma(-K, vprev[t], qbuf[t]);
        __syncthreads();
        // column j (and, at the end, column j + 1) on rows j..: A -= v q^T + q v^T
        const int ncol = last ? 2 : 1;
        for (int c = 0; c < ncol; ++c) {
            const int l = j + c;
            const double ql = qbuf[l], vl = vprev[l];
            for (int t = l + tid; t < N; t += 1024) {
                double *a = &W[(int64_t)l * ldw + t];
                *a = *a - vprev[t] * ql - qbuf[t] * vl;
            }
        }
        __syncthreads();
    }
    if (last) {  // j = N - 2: the trailing 2 x 2 block
        if (tid == 0) {
            d[N - 2] = W[(int64_t)(N - 2) * ldw + (N - 2)];
            d[N - 1] = W[(int64_t)(N - 1) * ldw + (N - 1)];
            e[N - 2] = W[(int64_t)(N - 2) * ldw + (N - 1)];
            tau[N - 2] = 0.0;
        }
        return;
    }
    if (tid == 0) d[j] = W[(int64_t)j * ldw + j];
    // reflector j from x = A[j+1:N, j]
    const int m = N - j - 1;
    double *col = W + (int64_t)j * ldw + (j + 1);
    double ss = 0.0;
    for (int t = 1 + tid; t < m; t += 1024) ss = fma(col[t], col[t], ss);
    ss = block_sum1024(ss, red);
    const double alpha = col[0];
    double tj = 0.0, ej = alpha, scale = 0.0;
    if (ss > 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        ej = beta;
    }
    __syncthreads();
    if (tid == 0) {
        tau[j] = tj;
        e[j] = ej;
    }
    for (int t = tid; t < m; t += 1024) {
        const double vt = (t == 0) ? 1.0 : col[t] * scale;
        vcur[j + 1 + t] = (tj != 0.0) ? vt : 0.0;
        if (tj != 0.0) col[t] = vt;
    }
}

// Trailing columns l >= j+1 on rows t >= j+1: update j-1, then partial
// sums over this tile's columns of tau_j A(t, l) v_j(l).
__global__ __launch_bounds__(256) void k_trd_upd(double *W, int64_t ldw, int N, int j, const double *tau,
                                                 const double *vbuf, const double *qbuf, double *ppart)
{
    __shared__ double s_v[TRD_TC], s_q[TRD_TC], s_w[TRD_TC];
    const double *vprev = vbuf + (int64_t)((j + 1) & 1) * N;
    const double *vcur = vbuf + (int64_t)(j & 1) * N;
    const int r0 = j + 1;
    const int t = r0 + blockIdx.x * 256 + threadIdx.x;
    const int l0 = r0 + blockIdx.y * TRD_TC;
    const double tp = (j > 0) ? tau[j - 1] : 0.0;
    const double tj = tau[j];
    if (threadIdx.x < TRD_TC) {
        const int l = l0 + threadIdx.x;
        const bool in = l < N;
        s_v[threadIdx.x] = (in && tp != 0.0) ? vprev[l] : 0.0;
        s_q[threadIdx.x] = (in && tp != 0.0) ? qbuf[l] : 0.0;
        s_w[threadIdx.x] = in ? vcur[l] : 0.0;
    }
    __syncthreads();
    if (t >= N) return;
    const double vt = (tp != 0.0) ? vprev[t] : 0.0, qt = (tp != 0.0) ? qbuf[t] : 0.0;
    const int lend = min(TRD_TC, N - l0);
    double acc = 0.0;
    double *a = W + (int64_t)l0 * ldw + t;
    if (tp != 0.0) {
        for (int c = 0; c < lend; ++c) {
            const double x = a[(int64_t)c * ldw] - vt * s_q[c] - qt * s_v[c];
            a[(int64_t)c * ldw] = x;
            acc = fma(x, s_w[c], acc);
        }
    } else {
        for (int c = 0; c < lend; ++c) acc = fma(a[(int64_t)c * ldw], s_w[c], acc);
    }
    ppart[(int64_t)blockIdx.y * N + t] = tj * acc;
}

// S <- H_0 H_1 ... H_{N-3} S for the reflectors left by k_sytrd; one
// workgroup per column of S (N x nvec, column-major, lds).
__global__ __launch_bounds__(256) void k_ormtr(const double *W, int64_t ldw, int N, const double *tau,
                                               double *S, int64_t lds)
{
    __shared__ double sb[4];
    double *s = S + (int64_t)blockIdx.x * lds;
    for (int j = N - 3; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        const double *vj = W + (int64_t)j * ldw + (j + 1);
        const int m = N - j - 1;
        double dt = 0.0;
        for (int t = threadIdx.x; t < m; t += 256) dt = fma(vj[t], s[j + 1 + t], dt);
        dt = tj * block_sum256(dt, sb);
        for (int t = threadIdx.x; t < m; t += 256) s[j + 1 + t] = fma(-dt, vj[t], s[j + 1 + t]);
        __syncthreads();
    }
}

// ------------------------------------------------------------ launch helpers
dim3 blk_grid(int64_t n, int64_t k) { return dim3((unsigned)cdiv(n, 256), (unsigned)k); }

int blk_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, int64_t k, hipStream_t st)
{
    if (k <= 0) return 0;
    hipLaunchKernelGGL(k_blk_copy, blk_grid(n, k), dim3(256), 0, st, src, lds, dst, ldd, n);
    return ok();
}

int blk_zero(double *X, int64_t ld, int64_t n, int64_t k, hipStream_t st)
{
    if (k <= 0) return 0;
    hipLaunchKernelGGL(k_blk_zero, blk_grid(n, k), dim3(256), 0, st, X, ld, n);
    return ok();
}

int nchunks(int64_t n) { return (int)cdiv(n, CHUNK); }

// out[c] = X[:, c] . Y[:, c]  (sq: its square root)
int col_dots(const double *X, const double *Y, int64_t ld, int64_t n, int64_t k, double *part, double *out,
             int sq, hipStream_t st)
{
    const int nch = nchunks(n);
    hipLaunchKernelGGL(k_col_dot_parts, dim3((unsigned)nch, (unsigned)k), dim3(256), 0, st, X, Y, ld, n, part,
                       nch);
    if (ok()) return GSYEIG_EHIP;
    hipLaunchKernelGGL(k_col_reduce, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, st, part, nch, k, out, sq);
    return ok();
}

// C (m x nn, column-major, ldc) = alpha X^T Y + beta C, X: n x m, Y: n x nn (FP64, split-K)
int gemm_tn(const double *X, int64_t ldx, const double *Y, int64_t ldy, int64_t n, int64_t m, int64_t nn,
            double *C, int64_t ldc, double alpha, double beta, double *part, int64_t part_elems, hipStream_t st)
{
    GemmDesc d{};
    d.m = m; d.n = nn; d.k = n;
    d.A = X; d.lda = ldx; d.a_layout = 1;   // A(i, t) = X(t, i)
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

// C (n x nn, ldc) = alpha X Q + beta C,  X: n x m (ldx), Q: m x nn (ldq), FP64
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

// C (n x k) = M X with M an n x n row-major matrix (FP64 or FP32 storage)
int gemm_mat(const void *M, int64_t ldm, int m_f32, int f32, const double *X, int64_t ldx, int64_t n,
             int64_t k, double *C, int64_t ldc, hipStream_t st)
{
    GemmDesc d{};
    d.m = n; d.n = k; d.k = n;
    d.A = M; d.lda = ldm; d.a_layout = 1; d.a_f32 = m_f32;
    d.B = X; d.ldb = ldx; d.b_layout = 0;
    d.C = C; d.ldc = ldc; d.c_layout = 0;
    d.alpha = 1.0; d.beta = 0.0;
    d.f32 = f32;
    return launch_gemm(d, st);
}

}  // namespace

// --------------------------------------------------------------- exported

int launch_invert_pairs(const double *mu, const double *Xin, int64_t ldi, double *lam, double *Xout,
                        int64_t ldo, int64_t n, int64_t s, hipStream_t st)
{
    hipLaunchKernelGGL(k_invert_pairs, blk_grid(n, s), dim3(256), 0, st, mu, Xin, ldi, lam, Xout, ldo, n, s);
    return ok();
}

int launch_identity(double *X, int64_t ld, int64_t r, hipStream_t st)
{
    hipLaunchKernelGGL(k_identity, dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, st, X, ld, r);
    return ok();
}

int launch_flag_offdiag(const double *G, int64_t r, double thresh, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_flag_offdiag, dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, st, G, r, thresh, flag);
    return ok();
}

int launch_accum_info(const int *src, int *dst, hipStream_t st)
{
    hipLaunchKernelGGL(k_accum_info, dim3(1), dim3(64), 0, st, src, dst);
    return ok();
}

int launch_blk_copy(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t n, int64_t k,
                    hipStream_t st)
{
    return blk_copy(src, lds, dst, ldd, n, k, st);
}

size_t syev_small_scratch(int64_t N, int64_t nwant)
{
    return sizeof(double) * (size_t)(3 * N + 8 + 7 * N * nwant + 3 * N + cdiv(N, TRD_TC) * N + 64);
}

// Householder tridiagonalisation of H (N x N, ld N): one workgroup for small
// orders, the whole GPU (two launches per column) above.
static int sytrd_launch(int64_t N, double *H, double *d, double *e, double *tau, double *aux, hipStream_t st)
{
    if (N <= 192) {  // <= SYTRD_LDS
        hipLaunchKernelGGL(k_sytrd, dim3(1), dim3(1024), 0, st, H, N, (int)N, d, e, tau);
        return ok();
    }
    double *vbuf = aux, *qbuf = vbuf + 2 * N, *ppart = qbuf + N;
    for (int64_t j = 0; j + 2 < N; ++j) {
        const int64_t m = N - j - 1;
        const int npart_prev = (int)cdiv(m + 1, TRD_TC);  // tiles of the previous column's pass
        hipLaunchKernelGGL(k_trd_col, dim3(1), dim3(1024), 0, st, H, N, (int)N, (int)j, d, e, tau, vbuf, qbuf,
                           ppart, j > 0 ? npart_prev : 0, 0);
        if (ok()) return GSYEIG_EHIP;
        hipLaunchKernelGGL(k_trd_upd, dim3((unsigned)cdiv(m, 256), (unsigned)cdiv(m, TRD_TC)), dim3(256), 0, st, H,
                           N, (int)N, (int)j, tau, vbuf, qbuf, ppart);
        if (ok()) return GSYEIG_EHIP;
    }
    const int64_t jl = N >= 2 ? N - 2 : 0;
    hipLaunchKernelGGL(k_trd_col, dim3(1), dim3(1024), 0, st, H, N, (int)N, (int)jl, d, e, tau, vbuf, qbuf, ppart,
                       (int)cdiv(N - jl, TRD_TC), 1);
    return ok();
}

// Eigenpairs of a symmetric N x N matrix H (column-major, ld N; destroyed):
// the nwant smallest (which = 0) or largest (which = 1), ascending, into
// w[0..nwant) (w[nwant] = the opposite extreme) and Q (N x nwant, ld N).
// *k0 = number of i with w[i] + shift <= floor_rel * (w[n - 1] + shift) (w ascending)
__global__ void k_count_floor(const double *w, int64_t n, double floor_rel, double shift, int *k0)
{
    __shared__ int s_c[256];
    const double thr = floor_rel * (w[n - 1] + shift);
    int c = 0;
    for (int64_t i = threadIdx.x; i < n; i += 256) c += (w[i] + shift <= thr) ? 1 : 0;
    s_c[threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s_c[threadIdx.x] += s_c[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *k0 = s_c[0];
}

int syev_small(gsyeig_ctx *ctx, int64_t N, double *H, int64_t nwant, int which, double *w, double *Q,
               double *scratch, hipStream_t st, double floor_rel, double floor_shift)
{
    if (N < 1 || N > SYTRD_MAX || nwant < 1 || nwant > N) return GSYEIG_EHIP;
    return syev_dense(ctx, N, H, nwant, which, w, Q, scratch, st, floor_rel, floor_shift);
}

// The same for any order N (variant TD's n x n C): the reduction is the
// whole-GPU one above 192, every index product 64-bit.
int syev_dense(gsyeig_ctx *ctx, int64_t N, double *H, int64_t nwant, int which, double *w, double *Q,
               double *scratch, hipStream_t st, double floor_rel, double floor_shift)
{
    if (N < 1 || N > INT32_MAX / 2 || nwant < 1 || nwant > N) return GSYEIG_EHIP;
    double *d = scratch, *e = d + N, *tau = e + N, *tri = tau + N + 8;
    double *aux = tri + 7 * N * nwant;
    if (sytrd_launch(N, H, d, e, tau, aux, st)) return GSYEIG_EHIP;
    int rc = launch_tri_bisect(d, e, N, nwant, which, w, st);
    if (rc) return rc;
    rc = launch_tri_vectors(d, e, N, nwant, w, Q, N, tri, ctx ? 0 : 1, nullptr, st);
    if (rc) return rc;
    if (ctx) {
        // independent inverse-iteration vectors are orthogonal to about
        // u ||T|| / gap; Cholesky QR twice finishes them unless two are
        // near-parallel (tight clusters), which takes the clustered path
        int *info_d = (int *)ctx->dscal + 26;
        int *h = (int *)ctx->host_pinned + 26;
        // eigenvectors at or below the floor are not wanted by the caller:
        // neither made orthonormal nor checked
        int64_t k0 = 0;
        if (floor_rel > 0.0 && which == 0) {
            int *k0_d = (int *)ctx->dscal + 28;
            hipLaunchKernelGGL(k_count_floor, dim3(1), dim3(256), 0, st, w, nwant, floor_rel, floor_shift, k0_d);
            if (ok()) return GSYEIG_EHIP;
            if (hipMemcpyAsync(h + 2, k0_d, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return GSYEIG_EHIP;
            if (hipStreamSynchronize(st) != hipSuccess) return GSYEIG_EHIP;
            k0 = std::min<int64_t>(h[2], nwant);
        }
        if (k0 < nwant) RTRY_HIP(orthonormalise_cols(ctx, N, nwant - k0, Q + k0 * N, N, info_d));
        else if (hipMemsetAsync(info_d, 0, 2 * sizeof(int), st) != hipSuccess) return GSYEIG_EHIP;
        if (hipMemcpyAsync(h, info_d, 2 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) return GSYEIG_EHIP;
        if (hipStreamSynchronize(st) != hipSuccess) return GSYEIG_EHIP;
        if (*h != 0) {
            ctx->n_fallback += 1;
            ctx->fallback_why = ((h[1] != 0) ? 2 : 1) + 10 * ctx->syev_site;
            rc = launch_tri_vectors(d, e, N, nwant, w, Q, N, tri, 1, nullptr, st);
            if (rc) return rc;
        }
    }
    hipLaunchKernelGGL(k_ormtr, dim3((unsigned)nwant), dim3(256), 0, st, H, N, (int)N, tau, Q, N);
    return ok();
}

int64_t syev_small_max() { return SYTRD_MAX; }


// X = U^-1 V (trans = 0) or U^-T V (trans = 1) for a block of k columns, U
// upper triangular stored FP64 or FP32 (u_f32) with its super-block
// inverses in sb (FP64, [Uinv | Uinv^T | ...]); V (n x k, ldv) is
// destroyed.  Right-looking over super-blocks: X_S = Uinv_SS V_S, then the
// rows not yet solved lose U_{.,S} X_S -- matrix-core products, FP32
// (f32 = 1, FP32 accumulation) or FP64.
int launch_trsm_sb(int trans, const void *U, int u_f32, int64_t ldu, int64_t n, const double *sb, double *V,
                   int64_t ldv, double *X, int64_t ldx, int64_t k, int f32, hipStream_t st)
{
    const int64_t SB = trsv_sb_rows();
    const int64_t nsb = cdiv(n, SB), blk = SB * SB;
    const double *Uinv = sb, *UinvT = sb + nsb * blk;
    const size_t esz = u_f32 ? sizeof(float) : sizeof(double);
    const char *Ub = (const char *)U;
    for (int64_t q = 0; q < nsb; ++q) {
        const int64_t S = trans ? q : nsb - 1 - q;
        const int64_t s0 = S * SB;
        const int64_t r = std::min<int64_t>(SB, n - s0);
        GemmDesc d{};
        d.m = r; d.n = k; d.k = r;
        d.A = (trans ? UinvT : Uinv) + S * blk; d.lda = SB; d.a_layout = 1;
        d.B = V + s0; d.ldb = ldv; d.b_layout = 0;
        d.C = X + s0; d.ldc = ldx; d.c_layout = 0;
        d.alpha = 1.0; d.beta = 0.0;
        d.f32 = f32;
        int rc = launch_gemm(d, st);
        if (rc) return rc;
        GemmDesc u{};
        u.n = k; u.k = r;
        u.B = X + s0; u.ldb = ldx; u.b_layout = 0;
        u.ldc = ldv; u.c_layout = 0;
        u.alpha = -1.0; u.beta = 1.0;
        u.a_f32 = u_f32; u.f32 = f32;
        u.lda = ldu;
        if (!trans) {
            if (S == 0) continue;
            u.m = s0;
            u.A = Ub + esz * (size_t)s0; u.a_layout = 1;                  // A(i, t) = U[i, s0 + t]
            u.C = V;
        } else {
            const int64_t s1 = s0 + r;
            if (s1 >= n) continue;
            u.m = n - s1;
            u.A = Ub + esz * (size_t)(s0 * ldu + s1); u.a_layout = 0;     // A(i, t) = U[s0 + t, s1 + i]
            u.C = V + s1;
        }
        rc = launch_gemm(u, st);
        if (rc) return rc;
    }
    return 0;
}

int launch_trsm_sb_f32(int trans, const float *U, int64_t ldu, int64_t n, const double *sb, double *V,
                       int64_t ldv, double *X, int64_t ldx, int64_t k, hipStream_t st)
{
    return launch_trsm_sb(trans, U, 1, ldu, n, sb, V, ldv, X, ldx, k, 1, st);
}

// Y_S = D_SS Z_S for every super-block S (D = Uinv or Uinv^T blocks, FP64
// row-major SB x SB): one batched product for the full super-blocks, one for
// a ragged last one
static int sb_diag_products(const double *D, const double *Z, int64_t ldz, double *Y, int64_t ldy, int64_t n,
                            int64_t k, int f32, hipStream_t st)
{
    const int64_t SB = trsv_sb_rows();
    const int64_t nsb = cdiv(n, SB), nfull = n / SB, blk = SB * SB;
    GemmDesc d{};
    d.n = k;
    d.lda = SB; d.a_layout = 1;
    d.ldb = ldz; d.b_layout = 0;
    d.ldc = ldy; d.c_layout = 0;
    d.alpha = 1.0; d.beta = 0.0;
    d.f32 = f32;
    if (nfull > 0) {
        d.m = SB; d.k = SB;
        d.A = D; d.B = Z; d.C = Y;
        d.batch = nfull;
        d.stride_a = blk; d.stride_b = SB; d.stride_c = SB;
        int rc = launch_gemm(d, st);
        if (rc) return rc;
    }
    if (nsb > nfull) {
        const int64_t s0 = nfull * SB;
        d.m = n - s0; d.k = n - s0;
        d.A = D + nfull * blk; d.B = Z + s0; d.C = Y + s0;
        d.batch = 1;
        return launch_gemm(d, st);
    }
    return 0;
}

int launch_trsm_w(int trans, const void *W, int w_f32, int64_t ldw, int64_t n, const double *sb, double *V,
                  int64_t ldv, double *X, int64_t ldx, int64_t k, int f32, hipStream_t st)
{
    const int64_t SB = trsv_sb_rows();
    const int64_t nsb = cdiv(n, SB), blk = SB * SB;
    const double *Uinv = sb, *UinvT = sb + nsb * blk;
    const size_t esz = w_f32 ? sizeof(float) : sizeof(double);
    const char *Wb = (const char *)W;
    if (!trans) {
        // c = D^-1 V, then from the bottom: X_{<S} -= W_{<S,S} X_S
        int rc = sb_diag_products(Uinv, V, ldv, X, ldx, n, k, f32, st);
        if (rc) return rc;
        for (int64_t S = nsb - 1; S >= 1; --S) {
            const int64_t s0 = S * SB, r = std::min<int64_t>(SB, n - s0);
            GemmDesc u{};
            u.m = s0; u.n = k; u.k = r;
            u.A = Wb + esz * (size_t)s0; u.lda = ldw; u.a_layout = 1; u.a_f32 = w_f32;   // A(i, t) = W[i, s0 + t]
            u.B = X + s0; u.ldb = ldx; u.b_layout = 0;
            u.C = X; u.ldc = ldx; u.c_layout = 0;
            u.alpha = -1.0; u.beta = 1.0;
            u.f32 = f32;
            if ((rc = launch_gemm(u, st))) return rc;
        }
        return 0;
    }
    // y = (I + W)^-T V in V, from the top: V_{>S} -= W_{S,>S}^T V_S; then X = D^-T y
    for (int64_t S = 0; S + 1 < nsb; ++S) {
        const int64_t s0 = S * SB, s1 = s0 + SB;
        GemmDesc u{};
        u.m = n - s1; u.n = k; u.k = SB;
        u.A = Wb + esz * (size_t)(s0 * ldw + s1); u.lda = ldw; u.a_layout = 0; u.a_f32 = w_f32;  // A(i, t) = W[s0 + t, s1 + i]
        u.B = V + s0; u.ldb = ldv; u.b_layout = 0;
        u.C = V + s1; u.ldc = ldv; u.c_layout = 0;
        u.alpha = -1.0; u.beta = 1.0;
        u.f32 = f32;
        const int rc = launch_gemm(u, st);
        if (rc) return rc;
    }
    return sb_diag_products(UinvT, V, ldv, X, ldx, n, k, f32, st);
}

// ------------------------------------------------------------ refinement
namespace {

struct Bump {
    char *base;
    size_t off;
    template <typename T> T *take(size_t count)
    {
        T *p = base ? (T *)(base + off) : nullptr;  // base == nullptr: sizes only
        off += (count * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

struct RefineBufs {
    int64_t ldr, k, K2;
    double *Z[2], *AZ[2], *BZ[2];
    double *Qy, *Rb, *vp, *v, *p, *wp, *w, *g, *t1, *t2;
    double *H, *Qc, *sy, *theta, *C1, *Wc, *st, *colpart, *cols, *cols2, *eta, *part, *scal, *dsc;
    int64_t part_elems;
};

size_t refine_layout(int64_t n, int64_t k, RefineBufs *b, char *base)
{
    Bump m{base, 0};
    const int64_t ldr = cdiv(n, 64) * 64, K2 = 2 * k;
    if (b) {
        b->ldr = ldr;
        b->k = k;
        b->K2 = K2;
    }
    auto blk = [&](int64_t cols) { return m.take<double>((size_t)ldr * (size_t)cols); };
    double *t[32];
    int i = 0;
    for (int z = 0; z < 2; ++z) {
        t[i++] = blk(K2);
        t[i++] = blk(K2);
        t[i++] = blk(K2);
    }
    for (int z = 0; z < 10; ++z) t[i++] = blk(k);
    const int64_t pe = std::min<int64_t>(32 * K2 * K2, std::max<int64_t>(4 * K2 * K2, (int64_t)1 << 22));
    double *H = m.take<double>((size_t)K2 * K2);
    double *Qc = m.take<double>((size_t)K2 * K2);
    double *sy = m.take<double>(syev_small_scratch(K2, K2) / sizeof(double) + 8);
    double *theta = m.take<double>((size_t)K2 + 8);
    double *C1 = m.take<double>((size_t)K2 * K2);
    double *Wc = m.take<double>((size_t)K2 * K2);
    double *st = m.take<double>((size_t)MR_FIELDS * k);
    double *colpart = m.take<double>((size_t)K2 * nchunks(n));
    double *cols = m.take<double>((size_t)K2);
    double *cols2 = m.take<double>((size_t)K2);
    double *eta = m.take<double>((size_t)K2);
    double *part = m.take<double>((size_t)pe);
    double *scal = m.take<double>(64);
    double *dsc = m.take<double>((size_t)K2);
    if (b) {
        for (int z = 0; z < 2; ++z) {
            b->Z[z] = t[3 * z];
            b->AZ[z] = t[3 * z + 1];
            b->BZ[z] = t[3 * z + 2];
        }
        double **vecs[10] = {&b->Qy, &b->Rb, &b->vp, &b->v, &b->p, &b->wp, &b->w, &b->g, &b->t1, &b->t2};
        for (int z = 0; z < 10; ++z) *vecs[z] = t[6 + z];
        b->H = H; b->Qc = Qc; b->sy = sy; b->theta = theta; b->C1 = C1; b->Wc = Wc; b->st = st;
        b->colpart = colpart; b->cols = cols; b->cols2 = cols2; b->eta = eta; b->part = part;
        b->part_elems = pe; b->scal = scal; b->dsc = dsc;
    }
    return m.off + 4096;
}

#define RTRY(expr)               \
    do {                         \
        int _rc = (expr);        \
        if (_rc) return _rc;     \
    } while (0)

struct Ctx {
    gsyeig_ctx *ctx;
    hipStream_t st;
    int64_t n;
    const double *A; int64_t lda;
    const double *B; int64_t ldb;
    const RefineOp *op;
    RefineBufs *b;
};

// B-orthonormalise the r columns of Z/AZ/BZ starting at column c0 in place
// (SVQB); directions with Gram eigenvalue below drop * largest are removed.
// Returns the number of columns kept in *kept.
int svqb(Ctx &c, int z, int64_t c0, int64_t r, double drop, int64_t *kept)
{
    RefineBufs &b = *c.b;
    hipStream_t st = c.st;
    double *Zc = b.Z[z] + c0 * b.ldr, *AZc = b.AZ[z] + c0 * b.ldr, *BZc = b.BZ[z] + c0 * b.ldr;
    const int oz = 1 - z;
    double *Tz = b.Z[oz] + c0 * b.ldr, *TAz = b.AZ[oz] + c0 * b.ldr, *TBz = b.BZ[oz] + c0 * b.ldr;
    // G = Z_c^T B Z_c (symmetrised), scaled to unit diagonal
    RTRY(gemm_tn(Zc, b.ldr, BZc, b.ldr, c.n, r, r, b.C1, r, 1.0, 0.0, b.part, b.part_elems, st));
    hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, st, b.C1, r, r);
    RTRY(ok());
    hipLaunchKernelGGL(k_gram_diag, dim3((unsigned)cdiv(r, 256)), dim3(256), 0, st, b.C1, r, b.dsc);
    RTRY(ok());
    hipLaunchKernelGGL(k_gram_apply, dim3((unsigned)cdiv(r * r, 256)), dim3(256), 0, st, b.C1, r, b.dsc);
    RTRY(ok());
    // decompose G - I (same eigenvectors; the subtraction is exact): for a
    // nearly B-orthonormal block every eigenvalue of G is 1 to working
    // precision, a numerically multiple cluster, while those of G - I are
    // spread relative to its own norm
    hipLaunchKernelGGL(k_diag_shift, dim3((unsigned)cdiv(r, 256)), dim3(256), 0, st, b.C1, r, r, -1.0);
    RTRY(ok());
    c.ctx->syev_site = 2;
    RTRY(syev_small(c.ctx, r, b.C1, r, 0, b.theta, b.Qc, b.sy, st, drop, 1.0));
    hipLaunchKernelGGL(k_vec_shift, dim3((unsigned)cdiv(r, 256)), dim3(256), 0, st, b.theta, r, 1.0);
    RTRY(ok());
    std::vector<double> sig((size_t)r);
    HIP_TRY(hipMemcpyAsync(sig.data(), b.theta, sizeof(double) * (size_t)r, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double smax = sig[(size_t)r - 1];
    int64_t first = 0;
    while (first < r && !(sig[(size_t)first] > drop * smax)) ++first;
    const int64_t rk = r - first;
    *kept = rk;
    if (rk == 0) return 0;
    hipLaunchKernelGGL(k_svqb_coef, dim3((unsigned)cdiv(r * rk, 256)), dim3(256), 0, st, b.Qc, r, b.theta,
                       b.dsc, first, rk, b.Wc);
    RTRY(ok());
    RTRY(gemm_nn(Zc, b.ldr, b.Wc, r, c.n, r, rk, Tz, b.ldr, 1.0, 0.0, st));
    RTRY(gemm_nn(AZc, b.ldr, b.Wc, r, c.n, r, rk, TAz, b.ldr, 1.0, 0.0, st));
    RTRY(gemm_nn(BZc, b.ldr, b.Wc, r, c.n, r, rk, TBz, b.ldr, 1.0, 0.0, st));
    RTRY(blk_copy(Tz, b.ldr, Zc, b.ldr, c.n, rk, st));
    RTRY(blk_copy(TAz, b.ldr, AZc, b.ldr, c.n, rk, st));
    RTRY(blk_copy(TBz, b.ldr, BZc, b.ldr, c.n, rk, st));
    return 0;
}

// Rayleigh-Ritz over the first N columns of Z[z] (B-orthonormal): the nk
// wanted Ritz pairs go to theta and, as X, AX, BX, to the first nk columns
// of the other buffer; returns the index of that buffer.
int rayleigh_ritz(Ctx &c, int z, int64_t N, int64_t nk, int which, int *znew)
{
    RefineBufs &b = *c.b;
    hipStream_t st = c.st;
    RTRY(gemm_tn(b.Z[z], b.ldr, b.AZ[z], b.ldr, c.n, N, N, b.H, N, 1.0, 0.0, b.part, b.part_elems, st));
    hipLaunchKernelGGL(k_symmetrise, dim3((unsigned)cdiv(N * N, 256)), dim3(256), 0, st, b.H, N, N);
    RTRY(ok());
    c.ctx->syev_site = 3;
    RTRY(syev_small(c.ctx, N, b.H, nk, which, b.theta, b.Qc, b.sy, st));
    const int oz = 1 - z;
    RTRY(gemm_nn(b.Z[z], b.ldr, b.Qc, N, c.n, N, nk, b.Z[oz], b.ldr, 1.0, 0.0, st));
    RTRY(gemm_nn(b.AZ[z], b.ldr, b.Qc, N, c.n, N, nk, b.AZ[oz], b.ldr, 1.0, 0.0, st));
    RTRY(gemm_nn(b.BZ[z], b.ldr, b.Qc, N, c.n, N, nk, b.BZ[oz], b.ldr, 1.0, 0.0, st));
    *znew = oz;
    return 0;
}

// y = C~ x = U~^-T A~ U~^-1 x for a block (FP32 matrices, FP32 MFMA);
// x is preserved, t1/t2 are scratch blocks.
int block_op(Ctx &c, const double *x, double *y, int64_t k)
{
    RefineBufs &b = *c.b;
    const RefineOp &op = *c.op;
    hipStream_t st = c.st;
    RTRY(blk_copy(x, b.ldr, b.t1, b.ldr, c.n, k, st));
    RTRY(launch_trsm_sb_f32(0, op.U32, op.ldu32, c.n, op.sb, b.t1, b.ldr, b.t2, b.ldr, k, st));
    RTRY(gemm_mat(op.A32, op.lda32, 1, 1, b.t2, b.ldr, c.n, k, b.t1, b.ldr, st));
    return launch_trsm_sb_f32(1, op.U32, op.ldu32, c.n, op.sb, b.t1, b.ldr, y, b.ldr, k, st);
}

// x <- x - Qy (Qy^T x)
int project_out(Ctx &c, double *x, int64_t k)
{
    RefineBufs &b = *c.b;
    RTRY(gemm_tn(b.Qy, b.ldr, x, b.ldr, c.n, k, k, b.C1, k, 1.0, 0.0, b.part, b.part_elems, c.st));
    return gemm_nn(b.Qy, b.ldr, b.C1, k, c.n, k, k, x, b.ldr, -1.0, 1.0, c.st);
}

}  // namespace

size_t refine_bytes(int64_t n, int64_t k) { return refine_layout(n, k, nullptr, nullptr); }

int refine_x0(gsyeig_ctx *ctx, int64_t n, int64_t k, double **X0, int64_t *ld)
{
    void *p;
    RTRY(ws_get(ctx, WS_REFINE, refine_bytes(n, k), &p));
    RefineBufs b;
    refine_layout(n, k, &b, (char *)p);
    *X0 = b.Z[0];
    *ld = b.ldr;
    return 0;
}

int refine_run(gsyeig_ctx *ctx, int64_t n, int64_t s, int64_t k, int which, const double *A, int64_t lda,
               const double *B, int64_t ldb, const RefineOp &op, const RefineCfg &cfg, double *Lambda,
               double *X, int64_t ldx, RefineStats *out)
{
    if (k < s || 2 * k > SYTRD_MAX) return GSYEIG_EHIP;
    void *p;
    RTRY(ws_get(ctx, WS_REFINE, refine_bytes(n, k), &p));
    RefineBufs b;
    refine_layout(n, k, &b, (char *)p);
    hipStream_t st = ctx->stream;
    Ctx c{ctx, st, n, A, lda, B, ldb, &op, &b};
    memset(out, 0, sizeof(*out));
    double *h = (double *)ctx->host_pinned;

    // ||A||_F, ||B||_F
    RTRY(launch_fro_norm_parts(A, lda, n, 0, nullptr, b.part, st));
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(64), 0, st, b.part, fro_parts(n), b.scal);
    RTRY(ok());
    RTRY(launch_fro_norm_parts(B, ldb, n, 0, nullptr, b.part, st));
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(64), 0, st, b.part, fro_parts(n), b.scal + 1);
    RTRY(ok());

    // start block X0 (in Z[0]): A X0, B X0, B-orthonormalise, Rayleigh-Ritz
    int z = 0;
    RTRY(gemm_mat(A, lda, 0, 0, b.Z[0], b.ldr, n, k, b.AZ[0], b.ldr, st));
    RTRY(gemm_mat(B, ldb, 0, 0, b.Z[0], b.ldr, n, k, b.BZ[0], b.ldr, st));
    int64_t kx = 0, kx2 = 0;
    RTRY(svqb(c, z, 0, k, 1e-10, &kx));
    if (kx < s) return GSYEIG_ENOCONV;
    RTRY(svqb(c, z, 0, kx, 0.0, &kx2));
    if (kx2 < s) return GSYEIG_ENOCONV;
    const int64_t kk = kx2;  // working block width
    const int64_t w0 = which ? kk - s : 0;
    RTRY(rayleigh_ritz(c, z, kk, kk, which, &z));

    for (int64_t it = 0;; ++it) {
        double *Xc = b.Z[z], *AXc = b.AZ[z], *BXc = b.BZ[z];
        // FP64 residual and backward errors
        hipLaunchKernelGGL(k_resid, blk_grid(n, kk), dim3(256), 0, st, AXc, BXc, b.ldr, n, b.theta, b.Rb);
        RTRY(ok());
        RTRY(col_dots(b.Rb, b.Rb, b.ldr, n, kk, b.colpart, b.cols, 0, st));
        RTRY(col_dots(Xc, Xc, b.ldr, n, kk, b.colpart, b.cols2, 0, st));
        hipLaunchKernelGGL(k_eta, dim3(1), dim3(256), 0, st, b.cols, b.cols2, b.theta, kk, w0, s, b.scal,
                           cfg.eta_tol, b.eta, b.scal + 2);
        RTRY(ok());
        HIP_TRY(hipMemcpyAsync(h, b.scal + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (it == 0) out->eta0 = h[0];
        out->eta = h[0];
        out->nconv = (int64_t)h[1];
        if (h[0] <= cfg.eta_tol || it >= cfg.max_iters) break;
        out->iters = it + 1;

        // y-space basis Qy = U~ X and residual rho = U~^-T R (FP32 products)
        RTRY(gemm_mat(op.U32, op.ldu32, 1, 1, Xc, b.ldr, n, kk, b.Qy, b.ldr, st));
        RTRY(launch_trsm_sb_f32(1, op.U32, op.ldu32, n, op.sb, b.Rb, b.ldr, b.t1, b.ldr, kk, st));
        RTRY(project_out(c, b.t1, kk));
        // MINRES on P (C~ - theta I) P g = -P rho, every column at once
        double *mst = b.st;
        RTRY(col_dots(b.t1, b.t1, b.ldr, n, kk, b.colpart, mst + MR_NRM * kk, 1, st));
        hipLaunchKernelGGL(k_mr_init, dim3((unsigned)cdiv(kk, 256)), dim3(256), 0, st, kk, mst);
        RTRY(ok());
        hipLaunchKernelGGL(k_scale_cols, blk_grid(n, kk), dim3(256), 0, st, b.t1, b.v, b.ldr, n,
                           mst + MR_VSCALE * kk, -1.0);
        RTRY(ok());
        RTRY(blk_zero(b.vp, b.ldr, n, kk, st));
        RTRY(blk_zero(b.w, b.ldr, n, kk, st));
        RTRY(blk_zero(b.wp, b.ldr, n, kk, st));
        RTRY(blk_zero(b.g, b.ldr, n, kk, st));
        double *vp = b.vp, *v = b.v, *pp = b.p, *w = b.w, *wp = b.wp;
        const int nch = nchunks(n);
        for (int64_t j = 0; j < cfg.inner; ++j) {
            RTRY(block_op(c, v, pp, kk));
            RTRY(project_out(c, pp, kk));
            hipLaunchKernelGGL(k_shift_sub, blk_grid(n, kk), dim3(256), 0, st, pp, v, b.ldr, n, b.theta);
            RTRY(ok());
            RTRY(col_dots(v, pp, b.ldr, n, kk, b.colpart, mst + MR_ALPHA * kk, 0, st));
            hipLaunchKernelGGL(k_mr_lanczos, dim3((unsigned)nch, (unsigned)kk), dim3(256), 0, st, pp, v, vp,
                               b.ldr, n, mst, kk, b.colpart, nch);
            RTRY(ok());
            hipLaunchKernelGGL(k_col_reduce, dim3((unsigned)cdiv(kk, 256)), dim3(256), 0, st, b.colpart, nch, kk,
                               mst + MR_NRM * kk, 1);
            RTRY(ok());
            hipLaunchKernelGGL(k_mr_scalars, dim3((unsigned)cdiv(kk, 256)), dim3(256), 0, st, kk, mst);
            RTRY(ok());
            hipLaunchKernelGGL(k_mr_update, blk_grid(n, kk), dim3(256), 0, st, v, w, wp, b.g, pp, b.ldr, n, mst,
                               kk);
            RTRY(ok());
            double *ov = vp;
            vp = v;
            v = pp;
            pp = ov;
            std::swap(w, wp);
            out->block_applies += 1;
        }
        // D = U~^-1 g into Z[:, kk:2kk]; A D, B D in FP64
        double *D = Xc + kk * b.ldr, *AD = AXc + kk * b.ldr, *BD = BXc + kk * b.ldr;
        RTRY(launch_trsm_sb_f32(0, op.U32, op.ldu32, n, op.sb, b.g, b.ldr, D, b.ldr, kk, st));
        RTRY(gemm_mat(A, lda, 0, 0, D, b.ldr, n, kk, AD, b.ldr, st));
        RTRY(gemm_mat(B, ldb, 0, 0, D, b.ldr, n, kk, BD, b.ldr, st));
        // D B-orthogonal to X (twice), then B-orthonormal (SVQB, twice)
        for (int pass = 0; pass < 2; ++pass) {
            RTRY(gemm_tn(Xc, b.ldr, BD, b.ldr, n, kk, kk, b.C1, kk, 1.0, 0.0, b.part, b.part_elems, st));
            RTRY(gemm_nn(Xc, b.ldr, b.C1, kk, n, kk, kk, D, b.ldr, -1.0, 1.0, st));
            RTRY(gemm_nn(AXc, b.ldr, b.C1, kk, n, kk, kk, AD, b.ldr, -1.0, 1.0, st));
            RTRY(gemm_nn(BXc, b.ldr, b.C1, kk, n, kk, kk, BD, b.ldr, -1.0, 1.0, st));
        }
        int64_t r1 = 0, r2 = 0;
        RTRY(svqb(c, z, kk, kk, 1e-10, &r1));
        if (r1 > 0) RTRY(svqb(c, z, kk, r1, 0.0, &r2));
        RTRY(rayleigh_ritz(c, z, kk + r2, kk, which, &z));
    }
    out->kept = kk;
    RTRY(launch_copy(b.theta + w0, Lambda, s, st));
    RTRY(blk_copy(b.Z[z] + w0 * b.ldr, b.ldr, X, ldx, n, s, st));
    return 0;
}
