// k_lanczos.hip -- the Lanczos update z_{k+1} -> w_{k+1} (key KI4 of
// variant KI, Section 2.3 and Table 1), in FP64:
//
//   z := z - beta_{k-1} w_{k-1};  alpha_k := w_k^T z;  z := z - alpha_k w_k
//   twice:  h := V_k^T z;  z := z - V_k h      (classical Gram-Schmidt applied
//                                               twice, Kahan's rule)
//   beta_k := ||z||;  w_{k+1} := z / beta_k
//
// The basis V (n x (m+1), column-major, each Lanczos vector contiguous) is
// the dominant traffic: the two Gram-Schmidt passes read it four times per
// step.  Every reduction is two-stage with a fixed summation order, so the
// recurrence is bitwise reproducible.
#include "internal.h"

namespace {

constexpr int RB = 2048;  // rows per partial sum of a vector reduction (256 threads x 8)

__device__ __forceinline__ double wave_sum(double v)
{
    v += __shfl_xor(v, 32);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

// Sum over a 256-thread block; the result is returned to every thread.
__device__ double block_sum(double v, double *sbuf /* >= 4 */)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sbuf[w] = v;
    __syncthreads();
    return ((sbuf[0] + sbuf[1]) + (sbuf[2] + sbuf[3]));
}

// Sum of part[0..P-1] in a fixed tree order, returned to every thread.
__device__ double sum_parts(const double *part, int P, double *sbuf)
{
    double v = 0.0;
    for (int p = threadIdx.x; p < P; p += 256) v += part[p];
    return block_sum(v, sbuf);
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill_splitmix(double *v, int64_t n, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = 2.0 * ((double)(splitmix64(seed, (uint64_t)i) >> 11) * 0x1p-53) - 1.0;
}

__global__ void k_copy(const double *src, double *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// part[p] = sum over rows of chunk p of a[i] * b[i]
__global__ __launch_bounds__(256) void k_dot_parts(const double *a, const double *b, int64_t n,
                                                   double *part)
{
    __shared__ double sbuf[4];
    const int64_t base = (int64_t)blockIdx.x * RB;
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < RB / 256; ++p) {
        const int64_t i = base + threadIdx.x + 256 * p;
        if (i < n) v = fma(a[i], b[i], v);
    }
    v = block_sum(v, sbuf);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// w := v / sqrt(sum(part)); optionally records the norm.
__global__ __launch_bounds__(256) void k_scale_by_norm(const double *v, double *w, int64_t n,
                                                       const double *part, int P, double *norm_out)
{
    __shared__ double sbuf[4];
    const double nrm = sqrt(sum_parts(part, P, sbuf));
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] = v[i] / nrm;
    if (norm_out && blockIdx.x == 0 && threadIdx.x == 0) *norm_out = nrm;
}

// z := z - beta_{k-1} w_{k-1} (k > 0); part = w_k . z over chunks of R rows
template <int R>
__global__ __launch_bounds__(256) void k_lz_three_term(double *z, const double *wprev,
                                                       const double *wk, const double *beta,
                                                       int64_t k, int64_t n, double *part)
{
    __shared__ double sbuf[4];
    const double bp = (k > 0) ? beta[k - 1] : 0.0;
    const int64_t base = (int64_t)blockIdx.x * R;
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < R / 256; ++p) {
        const int64_t i = base + threadIdx.x + 256 * p;
        if (i < n) {
            double zi = z[i];
            if (k > 0) zi = fma(-bp, wprev[i], zi);
            z[i] = zi;
            v = fma(wk[i], zi, v);
        }
    }
    v = block_sum(v, sbuf);
    if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// alpha_k = sum(part); z := z - alpha_k w_k
__global__ __launch_bounds__(256) void k_lz_sub_alpha(double *z, const double *wk, double *alpha,
                                                      int64_t k, int64_t n, const double *part, int P,
                                                      double *z0part)
{
    __shared__ double sbuf[4];
    const double a = sum_parts(part, P, sbuf);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double zz = 0.0;
    if (i < n) {
        zz = fma(-a, wk[i], z[i]);
        z[i] = zz;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) alpha[k] = a;
    if (z0part) {
        const double t = block_sum(zz * zz, sbuf);
        if (threadIdx.x == 0) z0part[blockIdx.x] = t;
    }
}

// Second Gram-Schmidt pass needed?  (Kahan's test as used by Parlett: a
// pass that keeps at least 1/sqrt(2) of the norm leaves z orthogonal to V to
// working accuracy.)  flag = 1 if ||z1||^2 < ||z0||^2 / 2.
// flag[1] counts the steps that took the second pass.
__global__ __launch_bounds__(256) void k_reorth_flag(const double *z0part, int P0, const double *z1part, int P1,
                                                     int *flag)
{
    __shared__ double sbuf[4];
    const double a = sum_parts(z0part, P0, sbuf);
    const double b = sum_parts(z1part, P1, sbuf);
    if (threadIdx.x == 0) {
        const int f = (b < 0.5 * a) ? 1 : 0;
        flag[0] = f;
        flag[1] += f;
    }
}

// Gram-Schmidt projection, stage 1: part[rc * kcols + c] = V(rows of rc, c)^T z(rows of rc)
// for the 8 columns of this workgroup's group.
__global__ __launch_bounds__(256) void k_gemv_t_parts(const double *__restrict__ V, int64_t ldv,
                                                      int64_t n, int64_t kcols,
                                                      const double *__restrict__ z,
                                                      double *__restrict__ part, const int *run)
{
    if (run && *run == 0) return;
    __shared__ double sred[4][8];
    const int64_t c0 = (int64_t)blockIdx.x * 8;
    const int rc = blockIdx.y;
    const int64_t base = (int64_t)rc * RB;
    double zr[RB / 256];
#pragma unroll
    for (int p = 0; p < RB / 256; ++p) {
        const int64_t i = base + threadIdx.x + 256 * p;
        zr[p] = (i < n) ? z[i] : 0.0;
    }
    // every load from a clamped in-bounds address, unconditionally (rows
    // beyond n meet zr = 0; columns beyond kcols are never written out), so
    // all 64 loads of a thread are in flight together
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        acc[c] = 0.0;
        const int64_t cc = (c0 + c < kcols) ? c0 + c : kcols - 1;
        const double *v = V + cc * ldv;
#pragma unroll
        for (int p = 0; p < RB / 256; ++p) {
            const int64_t i = base + threadIdx.x + 256 * p;
            acc[c] = fma(v[i < n ? i : n - 1], zr[p], acc[c]);
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const double s = wave_sum(acc[c]);
        if ((threadIdx.x & 63) == 0) sred[w][c] = s;
    }
    __syncthreads();
    if (threadIdx.x < 8 && c0 + threadIdx.x < kcols)
        part[(int64_t)rc * kcols + c0 + threadIdx.x] =
            (sred[0][threadIdx.x] + sred[1][threadIdx.x]) + (sred[2][threadIdx.x] + sred[3][threadIdx.x]);
}

// stage 2: h[c] = sum over row chunks
__global__ void k_gemv_t_reduce(const double *part, int RC, int64_t kcols, double *h, const int *run)
{
    if (run && *run == 0) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= kcols) return;
    double s = 0.0;
    for (int r = 0; r < RC; ++r) s += part[(int64_t)r * kcols + c];
    h[c] = s;
}

// z := z - V h over 64 rows per workgroup (8 waves split the columns);
// optionally normpart[block] = sum of the updated z^2 over those rows.
__global__ __launch_bounds__(512) void k_gemv_n_update(const double *__restrict__ V, int64_t ldv,
                                                       int64_t n, int64_t kcols,
                                                       const double *__restrict__ h,
                                                       double *__restrict__ z,
                                                       double *__restrict__ normpart, const int *run)
{
    if (run && *run == 0) return;
    __shared__ double s[8][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    const bool ok = r < n;
    // wave w takes a contiguous eighth of the columns, 16 column loads in
    // flight per lane (8 KB per wave), so the streaming of V is not bound by
    // the latency of a few outstanding loads
    double acc = 0.0;
    if (ok) {
        const int64_t per = (kcols + 7) / 8;
        const int wu = __builtin_amdgcn_readfirstlane(w);  // wave-uniform: h is read by scalar loads
        const int64_t cb = wu * per, ce = (cb + per < kcols) ? cb + per : kcols;
        const double *Vr = V + r;
        int64_t c = cb;
        for (; c + 16 <= ce; c += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = Vr[(c + u) * ldv];
            __builtin_amdgcn_sched_barrier(0);  // all 16 loads issued before the first use
#pragma unroll
            for (int u = 0; u < 16; ++u) acc = fma(v[u], h[c + u], acc);
        }
        for (; c < ce; ++c) acc = fma(Vr[c * ldv], h[c], acc);
    }
    s[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        const double sum = ((s[0][lane] + s[1][lane]) + (s[2][lane] + s[3][lane])) +
                           ((s[4][lane] + s[5][lane]) + (s[6][lane] + s[7][lane]));
        double zn = 0.0;
        if (ok) {
            zn = z[r] - sum;
            z[r] = zn;
        }
        if (normpart) {
            const double t = wave_sum(zn * zn);
            if (lane == 0) normpart[blockIdx.x] = t;
        }
    }
}

// beta_k = sqrt(sum(normpart)); w_{k+1} := z / beta_k
__global__ __launch_bounds__(256) void k_lz_normalize(const double *z, double *wnext, double *beta,
                                                      int64_t k, int64_t n, const double *normpart,
                                                      int P)
{
    __shared__ double sbuf[4];
    const double b = sqrt(sum_parts(normpart, P, sbuf));
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) wnext[i] = z[i] / b;
    if (blockIdx.x == 0 && threadIdx.x == 0) beta[k] = b;
}

// Partial re-orthogonalisation (Simon 1984; Section 2.3 asks that the loss
// of orthogonality be watched and repaired): omega_j,k estimates w_j^T w_k.  From
// the Lanczos relation beta_k w_{k+1} = C w_k - alpha_k w_k - beta_{k-1} w_{k-1}
// and the same relation for w_j,
//   beta_k om_{j,k+1} = beta_j om_{j+1,k} + (alpha_j - alpha_k) om_{j,k}
//                       + beta_{j-1} om_{j-1,k} - beta_{k-1} om_{j,k-1} + rounding,
// with om_{k,k} = 1 and om_{k,k+1} at rounding level.  The rounding terms are
// bounded by eps1 ||T||, eps1 = sqrt(n) u / 2, added with the sign of the sum
// (the usual pessimistic choice).  When max_j |om_{j,k+1}| exceeds sqrt(u),
// z is orthogonalised against all of V (two passes) at this step and the
// next one (the first pass leaves the next vector's estimate unreliable),
// and the estimates restart at eps1.  omN[j] = om_{j,k+1}, omC = om_{.,k},
// omP = om_{.,k-1}; beta_k is taken from the unorthogonalised z (z0part).
// flag[0] = this step orthogonalises, flag[1] counts such steps, flag[2] =
// the next step must orthogonalise; *anorm = running estimate of ||T||.
__global__ __launch_bounds__(1024) void k_pro_omega(const double *alpha, const double *beta, int64_t k,
                                                    const double *z0part, int P0, const double *omP,
                                                    const double *omC, double *omN, double *anorm, int *flag,
                                                    double eps1)
{
    __shared__ double s_red[16];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // beta_k before any orthogonalisation: sum of the partials, fixed order
    double v = 0.0;
    for (int p = tid; p < P0; p += 1024) v += z0part[p];
    v = wave_sum(v);
    if (lane == 0) s_red[wv] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += s_red[w];
    const double bk = sqrt(t);
    const double ak = alpha[k];
    const double bkm1 = (k > 0) ? beta[k - 1] : 0.0;
    const double an = fmax(*anorm, fabs(ak) + bk + bkm1);
    const double tau = eps1 * an;
    const double inv = (bk > 0.0) ? 1.0 / bk : 0.0;
    double mx = 0.0;
    for (int64_t j = tid; j < k; j += 1024) {
        double num = beta[j] * omC[j + 1] + (alpha[j] - ak) * omC[j] - bkm1 * omP[j];
        if (j > 0) num += beta[j - 1] * omC[j - 1];
        const double o = (num + copysign(tau, num)) * inv;
        omN[j] = o;
        mx = fmax(mx, fabs(o));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __syncthreads();
    if (lane == 0) s_red[wv] = mx;
    __syncthreads();
    mx = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) mx = fmax(mx, s_red[w]);
    const int forced = flag[2];
    // sqrt(u) = 2^-26.5, with u = 2^-53.  A small beta_k (near breakdown) also
    // loses local orthogonality, om_{k,k+1} = tau / beta_k: orthogonalise then.
    constexpr double thr = 1.0536712127723509e-08;
    const int f = forced || !(mx <= thr) || (bk * thr < tau);
    if (f)  // the two passes restore orthogonality to working accuracy
        for (int64_t j = tid; j < k; j += 1024) omN[j] = eps1;
    __syncthreads();
    if (tid == 0) {
        omN[k] = f ? eps1 : tau * inv;
        omN[k + 1] = 1.0;
        *anorm = an;
        flag[0] = f;
        flag[1] += f;
        flag[2] = f && !forced;
    }
}

__global__ void k_pro_init(double *om0, double *anorm, int *flag)
{
    if (threadIdx.x == 0) {
        om0[0] = 1.0;
        *anorm = 0.0;
        flag[0] = flag[1] = flag[2] = 0;
    }
}

// beta_k = sqrt(sum of the norm partials of the orthogonalised z (flag set)
// or of the unorthogonalised z); w_{k+1} := z / beta_k
__global__ __launch_bounds__(256) void k_lz_normalize_sel(const double *z, double *wnext, double *beta, int64_t k,
                                                          int64_t n, const double *normpart, int P,
                                                          const double *z0part, int P0, const int *flag)
{
    __shared__ double sbuf[4];
    const bool f = *flag != 0;
    const double b = sqrt(f ? sum_parts(normpart, P, sbuf) : sum_parts(z0part, P0, sbuf));
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) wnext[i] = z[i] / b;
    if (blockIdx.x == 0 && threadIdx.x == 0) beta[k] = b;
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

int launch_pro_init(double *om0, double *anorm, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_pro_init, dim3(1), dim3(64), 0, st, om0, anorm, flag);
    return ok();
}

int launch_pro_omega(const double *alpha, const double *beta, int64_t k, const double *z0part, int64_t n,
                     const double *omP, const double *omC, double *omN, double *anorm, int *flag, hipStream_t st)
{
    const double eps1 = 0.5 * sqrt((double)n) * 0x1p-53;
    hipLaunchKernelGGL(k_pro_omega, dim3(1), dim3(1024), 0, st, alpha, beta, k, z0part, lz_z0_parts(n), omP, omC,
                       omN, anorm, flag, eps1);
    return ok();
}

int launch_lz_normalize_sel(const double *z, double *wnext, double *beta, int64_t k, int64_t n,
                            const double *normpart, const double *z0part, const int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_normalize_sel, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, z, wnext, beta, k, n,
                       normpart, lz_norm_parts(n), z0part, lz_z0_parts(n), flag);
    return ok();
}

int lz_red_parts(int64_t n) { return (int)cdiv(n, RB); }
int lz_norm_parts(int64_t n) { return (int)cdiv(n, 64); }

int launch_fill_splitmix(double *v, int64_t n, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_splitmix, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, v, n, seed);
    return ok();
}

int launch_copy(const double *src, double *dst, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, src, dst, n);
    return ok();
}

int launch_normalize_into(const double *v, double *w, int64_t n, double *part, double *norm_out,
                          hipStream_t st)
{
    const int P = lz_red_parts(n);
    hipLaunchKernelGGL(k_dot_parts, dim3(P), dim3(256), 0, st, v, v, n, part);
    if (ok()) return GSYEIG_EHIP;
    hipLaunchKernelGGL(k_scale_by_norm, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, v, w, n,
                       (const double *)part, P, norm_out);
    return ok();
}

int launch_lz_alpha(double *z, const double *wprev, const double *wk, double *alpha,
                    const double *beta, int64_t k, int64_t n, double *part, hipStream_t st, double *z0part)
{
    // 512-row chunks (enough workgroups to stream the three vectors) while
    // the partials fit the 1024 slots; 2048-row chunks beyond
    const bool small = n <= 512 * 1024;
    const int P = (int)cdiv(n, small ? 512 : RB);
    if (small)
        hipLaunchKernelGGL(k_lz_three_term<512>, dim3(P), dim3(256), 0, st, z, wprev, wk, beta, k, n, part);
    else
        hipLaunchKernelGGL(k_lz_three_term<RB>, dim3(P), dim3(256), 0, st, z, wprev, wk, beta, k, n, part);
    if (ok()) return GSYEIG_EHIP;
    hipLaunchKernelGGL(k_lz_sub_alpha, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, z, wk, alpha,
                       k, n, (const double *)part, P, z0part);
    return ok();
}

int launch_cgs_pass(const double *V, int64_t ldv, int64_t n, int64_t kcols, double *z, double *part,
                    double *h, double *normpart, hipStream_t st, const int *run)
{
    const int RC = lz_red_parts(n);
    hipLaunchKernelGGL(k_gemv_t_parts, dim3((unsigned)cdiv(kcols, 8), RC), dim3(256), 0, st, V, ldv,
                       n, kcols, (const double *)z, part, run);
    if (ok()) return GSYEIG_EHIP;
    hipLaunchKernelGGL(k_gemv_t_reduce, dim3((unsigned)cdiv(kcols, 256)), dim3(256), 0, st,
                       (const double *)part, RC, kcols, h, run);
    if (ok()) return GSYEIG_EHIP;
    hipLaunchKernelGGL(k_gemv_n_update, dim3((unsigned)cdiv(n, 64)), dim3(512), 0, st, V, ldv, n,
                       kcols, (const double *)h, z, normpart, run);
    return ok();
}

int lz_z0_parts(int64_t n) { return (int)cdiv(n, 256); }

int launch_reorth_flag(const double *z0part, int64_t n, const double *z1part, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_reorth_flag, dim3(1), dim3(256), 0, st, z0part, lz_z0_parts(n), z1part, lz_norm_parts(n),
                       flag);
    return ok();
}

int launch_lz_normalize(const double *z, double *wnext, double *beta, int64_t k, int64_t n,
                        const double *normpart, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_normalize, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, st, z, wnext,
                       beta, k, n, normpart, lz_norm_parts(n));
    return ok();
}
