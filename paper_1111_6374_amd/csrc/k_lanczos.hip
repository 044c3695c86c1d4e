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

__global__ void k_pro_init(double *om0, double *anorm, int *flag)
{
    if (threadIdx.x == 0) {
        om0[0] = 1.0;
        *anorm = 0.0;
        flag[0] = flag[1] = flag[2] = 0;
    }
}

inline int ok() { return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP; }

}  // namespace

// ---------------------------------------------------------------------------
// The post-operator part of a Lanczos step with partial re-orthogonalisation
// in two launches.
//
// k_lz_step (one 1024-thread workgroup per 2048 rows): the three-term
// update and alpha_k, |z|^2, the omega recurrence and the decision whether
// this step orthogonalises, and -- when it does not -- beta_k and
// w_{k+1} = z / beta_k.  A row chunk stays in registers throughout; the
// two global sums are exchanged through sentinel-initialised slots (each
// workgroup publishes its partial and polls the others', the omega
// recurrence is evaluated identically by every workgroup).  The slots come
// in two sets used by alternate steps, and a workgroup restores its slots
// of the other set, so no launch needs a host memset.  The grid is small
// (n / 2048 workgroups) and every workgroup can be resident at once.
//
// k_lz_cgs (every workgroup that can run): on the steps that orthogonalise,
// two classical Gram-Schmidt passes against w_0..w_k and the normalisation;
// on the others it returns at once.  Its phases are items of one work
// queue taken in order by whichever workgroups are running, and an item
// waits only on counters of earlier phases, so it drains whatever the
// residency: [two passes of (T: V^T z tiles of 8192 rows x 8 columns,
// R: h = sum of the tiles, N: z -= V h over 64 rows)] [E: w_{k+1}].
//
// Summation orders are fixed in both: bitwise reproducible.
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
namespace {

constexpr int PR = 2048;   // rows of a k_lz_step workgroup / an E item (1024 threads x 2)
constexpr int TR = 8192;   // rows of a projection tile (1024 threads x 8)
constexpr int TC = 8;      // columns of a projection tile
constexpr int MAXP = 1024; // k_lz_step workgroups at most (n <= 2^21)

// sum over the 1024 threads, returned to all (fixed order)
__device__ double bsum1024(double v, double *s16)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s16[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += s16[q];
    return t;
}

// sum of part[0..P-1] (fixed order), returned to all
__device__ double sum1024(const double *part, int64_t P, double *s16)
{
    double v = 0.0;
    for (int64_t p = threadIdx.x; p < P; p += 1024) v += part[p];
    return bsum1024(v, s16);
}

// Sum of the P (<= MAXP) published slots (sentinel until written), polled
// by wave 0 (bounded; an expired wait records the error and reads 0) and
// summed in a fixed order; returned to every thread.
__device__ double sum_published(const double *slot, int P, LzCtl *ctl, unsigned lim, double *s1)
{
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        double acc = 0.0;
        for (int p0 = 0; p0 < P; p0 += 64 * 4) {
            unsigned long long v[4];
            unsigned live = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int p = p0 + l + 64 * c;
                live |= (p < P ? 1u : 0u) << c;
                v[c] = (p < P) ? __hip_atomic_load(reinterpret_cast<const unsigned long long *>(slot + p),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : 0ull;
            }
            unsigned it = 0;
            for (;;) {
                bool pend = false;
#pragma unroll
                for (int c = 0; c < 4; ++c) pend |= ((live >> c) & 1u) && v[c] == STAGE_SENTINEL;
                if (!__any(pend)) break;
                if (++it > lim) {
                    __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if (v[c] == STAGE_SENTINEL) v[c] = 0ull;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    if (((live >> c) & 1u) && v[c] == STAGE_SENTINEL)
                        v[c] = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(slot + p0 + l + 64 * c),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if ((live >> c) & 1u) acc += __longlong_as_double((long long)v[c]);
        }
        acc = wave_sum(acc);
        if (l == 0) *s1 = acc;
    }
    __syncthreads();
    const double r = *s1;
    __syncthreads();
    return r;
}

__device__ __forceinline__ void publish(double *slot, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(slot), (unsigned long long)__double_as_longlong(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct LzStep {
    double *z;
    const double *wprev, *wk;
    double *wnext;
    double *alpha, *beta;
    int64_t k, n;
    const double *omP, *omC;
    double *omN, *anorm;
    int *flag;
    double eps1;
    double *slots;  // 2 sets x (apart[MAXP], z0part[MAXP]), sentinel-initialised
    LzCtl *ctl;
};

__global__ __launch_bounds__(1024) void k_lz_step(LzStep a)
{
    __shared__ double s16[16], s1;
    __shared__ double s_in[2];
    __shared__ int s_forced;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t n = a.n, k = a.k;
    const int P = (int)gridDim.x, g = (int)blockIdx.x;
    const unsigned spin = __hip_atomic_load(&a.ctl->spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned lim = spin ? spin : SPIN_LIMIT;
    double *cur = a.slots + (k & 1) * 2 * MAXP, *oth = a.slots + ((k + 1) & 1) * 2 * MAXP;
    // state this step reads and workgroup 0 rewrites at its end: read first
    if (tid == 0) {
        s_forced = a.flag[2];
        s_in[0] = *a.anorm;
        s_in[1] = (k > 0) ? a.beta[k - 1] : 0.0;
        // the other set's slots of this workgroup, for the next step
        publish(oth + g, __longlong_as_double((long long)STAGE_SENTINEL));
        publish(oth + MAXP + g, __longlong_as_double((long long)STAGE_SENTINEL));
    }
    __syncthreads();
    const double bkm1 = s_in[1];
    // the omega recurrence's inputs for j < OMQ * 1024 (earlier steps' alpha,
    // beta and omega columns): loaded now, off the path of the two sums
    constexpr int OMQ = 3;
    double pb[OMQ], pbm[OMQ], pa[OMQ], pc0[OMQ], pc1[OMQ], pcm[OMQ], pp[OMQ];
#pragma unroll
    for (int r = 0; r < OMQ; ++r) {
        const int64_t j = tid + 1024 * r;
        const bool in = j < k;
        pb[r] = in ? a.beta[j] : 0.0;
        pa[r] = in ? a.alpha[j] : 0.0;
        pc0[r] = in ? a.omC[j] : 0.0;
        pc1[r] = in ? a.omC[j + 1] : 0.0;
        pp[r] = in ? a.omP[j] : 0.0;
        pbm[r] = (in && j > 0) ? a.beta[j - 1] : 0.0;
        pcm[r] = (in && j > 0) ? a.omC[j - 1] : 0.0;
    }
    // z := z - beta_{k-1} w_{k-1}; alpha_k = w_k . z
    double zr[PR / 1024], wr[PR / 1024];
    double d = 0.0;
#pragma unroll
    for (int p = 0; p < PR / 1024; ++p) {
        const int64_t i = (int64_t)g * PR + tid + 1024 * p;
        zr[p] = wr[p] = 0.0;
        if (i < n) {
            double zi = a.z[i];
            if (k > 0) zi = fma(-bkm1, a.wprev[i], zi);
            zr[p] = zi;
            wr[p] = a.wk[i];
            d = fma(wr[p], zi, d);
        }
    }
    d = bsum1024(d, s16);
    if (tid == 0) publish(cur + g, d);
    const double ak = sum_published(cur, P, a.ctl, lim, &s1);
    // z := z - alpha_k w_k; beta_k before any orthogonalisation
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < PR / 1024; ++p) {
        zr[p] = fma(-ak, wr[p], zr[p]);
        s = fma(zr[p], zr[p], s);
    }
    s = bsum1024(s, s16);
    if (tid == 0) publish(cur + MAXP + g, s);
    const double bk = sqrt(sum_published(cur + MAXP, P, a.ctl, lim, &s1));
    // the omega recurrence (every workgroup: the same inputs, the same f)
    const double an = fmax(s_in[0], fabs(ak) + bk + bkm1);
    const double tau = a.eps1 * an;
    const double inv = (bk > 0.0) ? 1.0 / bk : 0.0;
    double mx = 0.0;
#pragma unroll
    for (int r = 0; r < OMQ; ++r) {
        const int64_t j = tid + 1024 * r;
        if (j < k) {
            double num = pb[r] * pc1[r] + (pa[r] - ak) * pc0[r] - bkm1 * pp[r];
            if (j > 0) num += pbm[r] * pcm[r];
            const double o = (num + copysign(tau, num)) * inv;
            if (g == 0) a.omN[j] = o;
            mx = fmax(mx, fabs(o));
        }
    }
    for (int64_t j = tid + 1024 * OMQ; j < k; j += 1024) {
        double num = a.beta[j] * a.omC[j + 1] + (a.alpha[j] - ak) * a.omC[j] - bkm1 * a.omP[j];
        if (j > 0) num += a.beta[j - 1] * a.omC[j - 1];
        const double o = (num + copysign(tau, num)) * inv;
        if (g == 0) a.omN[j] = o;
        mx = fmax(mx, fabs(o));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    __syncthreads();
    if (lane == 0) s16[wv] = mx;
    __syncthreads();
    mx = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) mx = fmax(mx, s16[w]);
    // sqrt(u) = 2^-26.5, with u = 2^-53.  A small beta_k (near breakdown)
    // also loses local orthogonality, om_{k,k+1} = tau / beta_k:
    // orthogonalise then.
    const int forced = s_forced;
    constexpr double thr = 1.0536712127723509e-08;
    const int f = forced || !(mx <= thr) || (bk * thr < tau);
#pragma unroll
    for (int p = 0; p < PR / 1024; ++p) {
        const int64_t i = (int64_t)g * PR + tid + 1024 * p;
        if (i < n) {
            if (f) a.z[i] = zr[p];  // for the Gram-Schmidt passes
            else a.wnext[i] = zr[p] / bk;
        }
    }
    if (g == 0) {
        if (f)  // the two passes restore orthogonality to working accuracy
            for (int64_t j = tid; j < k; j += 1024) a.omN[j] = a.eps1;
        __syncthreads();
        if (tid == 0) {
            a.alpha[k] = ak;
            if (!f) a.beta[k] = bk;
            a.omN[k] = f ? a.eps1 : tau * inv;
            a.omN[k + 1] = 1.0;
            *a.anorm = an;
            a.flag[0] = f;
            a.flag[1] += f;
            a.flag[2] = f && !forced;
        }
    }
}

struct LzCgs {
    const double *z;  // z after the three-term update (k_lz_step)
    double *wnext, *beta;
    int64_t k, n;
    const double *V;
    int64_t ldv;
    const int *flag;
    double *sb;       // sentinel buffers: tp[2][rt x kc], hh[2][kc], z1[n], z2[n], np[nn]
    int64_t kcap;     // kc capacity of tp / hh
    LzCtl *ctl;
};

struct CgsPlan {  // item ranges and buffer offsets (derived the same way on every workgroup)
    int64_t rt, nt, nr, nn, ne, pass, e0, end;
    int64_t tp, hh, z1, z2, np, total;
};

__device__ __forceinline__ CgsPlan cgs_plan(int64_t n, int64_t kc, int64_t kcap)
{
    CgsPlan p;
    p.rt = (n + TR - 1) / TR;
    p.nt = p.rt * ((kc + TC - 1) / TC);
    p.nr = (kc + 1023) / 1024;
    p.nn = (n + 63) / 64;
    p.ne = (n + PR - 1) / PR;
    p.pass = p.nt + p.nr + p.nn;
    p.e0 = 2 * p.pass;
    p.end = p.e0 + p.ne;
    p.tp = 0;
    p.hh = 2 * p.rt * kcap;
    p.z1 = p.hh + 2 * kcap;
    p.z2 = p.z1 + n;
    p.np = p.z2 + n;
    p.total = p.np + p.nn;
    return p;
}

// lane `lane`'s v, to every lane (lane wave-uniform)
__device__ __forceinline__ double rdlane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ unsigned long long ldb(const double *p)
{
    return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// One published value per lane (ok lanes), polled until it is not the
// sentinel (bounded: an expired wait records the error and reads 0).
__device__ __forceinline__ double poll1(const double *p, bool ok, LzCtl *ctl, unsigned lim)
{
    unsigned long long v = ok ? ldb(p) : 0ull;
    unsigned it = 0;
    while (__any(ok && v == STAGE_SENTINEL)) {
        if (++it > lim) {
            __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (v == STAGE_SENTINEL) v = 0ull;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
        if (ok && v == STAGE_SENTINEL) v = ldb(p);
    }
    return __longlong_as_double((long long)v);
}

// Up to K published values per lane, base[c * stride] for c < cnt (cnt may
// differ between lanes; out[c] = 0 beyond it): all loads issued at once,
// then the sentinels polled again together (bounded, as poll1).  Called by
// every active lane of the wave.
template <int K>
__device__ __forceinline__ void poll_strided(const double *base, int64_t stride, int cnt, double (&out)[K], LzCtl *ctl,
                                             unsigned lim)
{
    unsigned long long v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = (c < cnt) ? ldb(base + c * stride) : 0ull;
    unsigned it = 0;
    for (;;) {
        bool pend = false;
#pragma unroll
        for (int c = 0; c < K; ++c) pend |= (c < cnt) && v[c] == STAGE_SENTINEL;
        if (!__any(pend)) break;
        if (++it > lim) {
            __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int c = 0; c < K; ++c)
                if (v[c] == STAGE_SENTINEL) v[c] = 0ull;
            break;
        }
        __builtin_amdgcn_s_sleep(2);
#pragma unroll
        for (int c = 0; c < K; ++c)
            if (c < cnt && v[c] == STAGE_SENTINEL) v[c] = ldb(base + c * stride);
    }
#pragma unroll
    for (int c = 0; c < K; ++c) out[c] = __longlong_as_double((long long)v[c]);
}

__global__ __launch_bounds__(1024) void k_lz_cgs(LzCgs a)
{
    if (*(volatile const int *)a.flag == 0) return;  // this step does not orthogonalise
    __shared__ int64_t s_q;
    __shared__ int s_last;
    __shared__ double s16[16];
    __shared__ double s_red[16][64];
    LzCtl *ctl = a.ctl;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t n = a.n, k = a.k, kc = k + 1;
    const CgsPlan P = cgs_plan(n, kc, a.kcap);
    const unsigned spin = __hip_atomic_load(&ctl->spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned lim = spin ? spin : SPIN_LIMIT;
    double *sb = a.sb;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_q = (int64_t)__hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t q = s_q;
        if (q >= P.end) break;
        if (q < P.e0) {
            const int pass = q >= P.pass;
            const int64_t d = q - pass * P.pass;
            double *tp = sb + P.tp + pass * P.rt * a.kcap, *hh = sb + P.hh + pass * a.kcap;
            const double *zin = pass ? sb + P.z1 : a.z;
            double *zout = pass ? sb + P.z2 : sb + P.z1;
            if (d < P.nt) {
                // T: tp[rt][c] = V(rows of rt, c)^T z(rows of rt), TC columns
                const int64_t rt = d % P.rt, c0 = (d / P.rt) * TC;
                double zr[TR / 1024];
                if (pass) {  // z1, published by the previous pass's N items
                    const int64_t i0 = rt * TR + tid;
                    const int cnt = (i0 < n) ? (int)((n - i0 + 1023) / 1024) : 0;
                    poll_strided<TR / 1024>(zin + i0, 1024, cnt < TR / 1024 ? cnt : TR / 1024, zr, ctl, lim);
                } else {
#pragma unroll
                    for (int p = 0; p < TR / 1024; ++p) {
                        const int64_t i = rt * TR + tid + 1024 * p;
                        zr[p] = (i < n) ? zin[i] : 0.0;
                    }
                }
                // every load from a clamped in-bounds address (rows beyond n
                // meet zr = 0; columns beyond kc are never written out)
#pragma unroll 2
                for (int c = 0; c < TC; ++c) {
                    const int64_t cc = (c0 + c < kc) ? c0 + c : kc - 1;
                    const double *v = a.V + cc * a.ldv;
                    double acc = 0.0;
#pragma unroll
                    for (int p = 0; p < TR / 1024; ++p) {
                        const int64_t i = rt * TR + tid + 1024 * p;
                        acc = fma(v[i < n ? i : n - 1], zr[p], acc);
                    }
                    acc = wave_sum(acc);
                    if (lane == 0) s_red[wv][c] = acc;
                }
                __syncthreads();
                if (tid < TC && c0 + tid < kc) {
                    double s = 0.0;
#pragma unroll
                    for (int w = 0; w < 16; ++w) s += s_red[w][tid];
                    publish(tp + rt * a.kcap + c0 + tid, s);
                }
            } else if (d < P.nt + P.nr) {
                // R: hh[c] = sum of the tiles' projections, in tile order
                const int64_t c = (d - P.nt) * 1024 + tid;
                if (c < kc) {
                    double s = 0.0;
                    for (int64_t r0 = 0; r0 < P.rt; r0 += 8) {
                        double v[8];
                        const int64_t left = P.rt - r0;
                        poll_strided<8>(tp + r0 * a.kcap + c, a.kcap, left < 8 ? (int)left : 8, v, ctl, lim);
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            if (q < left) s += v[q];
                    }
                    publish(hh + c, s);
                }
            } else {
                // N: z := z - V hh over 64 rows (16 waves split the columns;
                // a wave polls hh 64 columns at a time and broadcasts lane u's
                // value for column c0 + u); pass 1 also publishes |z|^2 over the rows
                const int64_t r = (d - P.nt - P.nr) * 64 + lane;
                const bool ok = r < n;
                const int64_t rr = ok ? r : n - 1;
                const int64_t per = (((kc + 15) / 16 + 63) / 64) * 64;
                const int64_t cs = wv * per, ce = (cs + per < kc) ? cs + per : kc;
                const double *Vr = a.V + rr;
                double acc = 0.0;
                // the wave's coefficients, 8 chunks of 64 columns per poll
                for (int64_t g0 = cs; g0 < ce; g0 += 8 * 64) {
                    double hq[8];
                    const int64_t rem = ce - g0 - lane;
                    const int cnt = rem > 0 ? (int)((rem + 63) / 64) : 0;
                    poll_strided<8>(hh + g0 + lane, 64, cnt < 8 ? cnt : 8, hq, ctl, lim);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int64_t c0 = g0 + 64 * q;
                        if (c0 >= ce) break;
                        const int64_t cn = (ce - c0 < 64) ? ce - c0 : 64;
                        const double hv = hq[q];
                        int u = 0;
                        for (; u + 8 <= cn; u += 8) {
                            double v[8];
#pragma unroll
                            for (int x = 0; x < 8; ++x) v[x] = Vr[(c0 + u + x) * a.ldv];
#pragma unroll
                            for (int x = 0; x < 8; ++x) acc = fma(v[x], rdlane(hv, u + x), acc);
                        }
                        for (; u < cn; ++u) acc = fma(Vr[(c0 + u) * a.ldv], rdlane(hv, u), acc);
                    }
                }
                s_red[wv][lane] = acc;
                __syncthreads();
                if (wv == 0) {
                    double sum = 0.0;
#pragma unroll
                    for (int w = 0; w < 16; ++w) sum += s_red[w][lane];
                    double zn = 0.0;
                    if (ok) {
                        zn = (pass ? poll1(zin + r, true, ctl, lim) : zin[r]) - sum;
                        publish(zout + r, zn);
                    }
                    if (pass) {
                        const double t2 = wave_sum(zn * zn);
                        if (lane == 0) publish(sb + P.np + r / 64, t2);
                    }
                }
            }
        } else {
            // E: beta_k of the orthogonalised z and w_{k+1} = z / beta_k
            double v = 0.0;
            for (int64_t p0 = 0; p0 < P.nn; p0 += 8 * 1024) {
                double pv[8];
                const int64_t rem = P.nn - p0 - tid;
                const int cnt = rem > 0 ? (int)((rem + 1023) / 1024) : 0;
                poll_strided<8>(sb + P.np + p0 + tid, 1024, cnt < 8 ? cnt : 8, pv, ctl, lim);
#pragma unroll
                for (int c = 0; c < 8; ++c) v += pv[c];
            }
            const double bk = sqrt(bsum1024(v, s16));
            const int64_t e = q - P.e0;
            double zv[PR / 1024];
            const int64_t i0 = e * PR + tid;
            const int cz = (i0 < n) ? (int)((n - i0 + 1023) / 1024) : 0;
            poll_strided<PR / 1024>(sb + P.z2 + i0, 1024, cz < PR / 1024 ? cz : PR / 1024, zv, ctl, lim);
#pragma unroll
            for (int p = 0; p < PR / 1024; ++p) {
                const int64_t i = i0 + 1024 * p;
                if (i < n) a.wnext[i] = zv[p] / bk;
            }
            if (e == 0 && tid == 0) a.beta[k] = bk;
        }
    }
    // count this workgroup out; the last one restores the sentinels and
    // resets the queue for the next step
    __syncthreads();
    if (tid == 0) {
        const unsigned d = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        s_last = (d == gridDim.x - 1);
    }
    __syncthreads();
    if (s_last) {
        const unsigned long long S = STAGE_SENTINEL;
        for (int pass = 0; pass < 2; ++pass) {
            for (int64_t r = 0; r < P.rt; ++r)
                for (int64_t c = tid; c < kc; c += 1024)
                    __hip_atomic_store(reinterpret_cast<unsigned long long *>(sb + P.tp + (pass * P.rt + r) * a.kcap + c),
                                       S, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int64_t c = tid; c < kc; c += 1024)
                __hip_atomic_store(reinterpret_cast<unsigned long long *>(sb + P.hh + pass * a.kcap + c), S,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        for (int64_t i = tid; i < 2 * n + P.nn; i += 1024)
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(sb + P.z1 + i), S, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (tid == 0) {
            __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

int launch_lz_post(double *z, const double *wprev, const double *wk, double *wnext, double *alpha, double *beta,
                   int64_t k, int64_t n, const double *V, int64_t ldv, const double *omP, const double *omC,
                   double *omN, double *anorm, int *flag, double *slots, double *cgs, int64_t kcap, LzCtl *ctl,
                   hipStream_t st)
{
    const int P = (int)cdiv(n, PR);
    if (P > MAXP) return GSYEIG_ETOOBIG;
    LzStep s{z, wprev, wk, wnext, alpha, beta, k, n, omP, omC, omN, anorm, flag, 0.5 * sqrt((double)n) * 0x1p-53,
             slots, ctl};
    hipLaunchKernelGGL(k_lz_step, dim3((unsigned)P), dim3(1024), 0, st, s);
    if (hipGetLastError() != hipSuccess) return GSYEIG_EHIP;
    static int grid = 0;
    if (!grid) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_lz_cgs, 1024, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1, cus = 256;
        grid = per_cu * cus;
    }
    LzCgs c{z, wnext, beta, k, n, V, ldv, flag, cgs, kcap, ctl};
    hipLaunchKernelGGL(k_lz_cgs, dim3((unsigned)grid), dim3(1024), 0, st, c);
    return hipGetLastError() == hipSuccess ? 0 : GSYEIG_EHIP;
}

// buffers launch_lz_post needs, all STAGE_SENTINEL before the first step:
// the partial-sum slots (lz_post_slots doubles) and the Gram-Schmidt
// buffers for k + 1 <= kcap (lz_cgs_doubles)
int lz_post_slots() { return 4 * MAXP; }
int64_t lz_cgs_doubles(int64_t n, int64_t kcap)
{
    return 2 * cdiv(n, TR) * kcap + 2 * kcap + 2 * n + cdiv(n, 64);
}

int launch_pro_init(double *om0, double *anorm, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(k_pro_init, dim3(1), dim3(64), 0, st, om0, anorm, flag);
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
