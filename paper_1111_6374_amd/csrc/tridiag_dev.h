// tridiag_dev.h -- wave-level routines on the Lanczos tridiagonal T_m
// (Sturm bisection, LU with partial pivoting and the inverse-iteration
// solve), shared by the KI5 kernels and the batched Lanczos kernel.  Each
// routine runs on one wavefront (lane = threadIdx.x & 63) and reads T from
// global memory.
#pragma once

#include "internal.h"

namespace tdg {

constexpr double EPS = 0x1p-53;

__device__ __forceinline__ double rdlane(double v, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_min(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Gershgorin interval and the pivot floor, computed by one wave.
static __device__ void gershgorin(const double *alpha, const double *beta, int64_t m, double *gl,
                           double *gu, double *pivmin)
{
    const int lane = threadIdx.x & 63;
    double lo = INFINITY, hi = -INFINITY, b2 = 0.0;
    for (int64_t j = lane; j < m; j += 64) {
        const double bl = (j > 0) ? fabs(beta[j - 1]) : 0.0;
        const double br = (j < m - 1) ? fabs(beta[j]) : 0.0;
        lo = fmin(lo, alpha[j] - bl - br);
        hi = fmax(hi, alpha[j] + bl + br);
        if (j < m - 1) b2 = fmax(b2, beta[j] * beta[j]);
    }
    *gl = wave_min(lo);
    *gu = wave_max(hi);
    *pivmin = 0x1p-1022 * fmax(1.0, wave_max(b2));
}

__device__ __forceinline__ void sturm_step(double a, double b2, double sigma, double pivmin, double &q, int &cnt)
{
    q = (a - sigma) - b2 / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
}

// number of eigenvalues of T below sigma (LDL^T pivots of T - sigma I), one
// sigma per lane.  alpha_j and beta_{j-1}^2 come in chunks of 64 rows, one
// row per lane, read back with readlane; the next chunk's loads are in
// flight while a chunk is processed, so the recurrence never waits on
// memory.  (Row 0 has b2 = 0, so its pivot is alpha_0 - sigma.)
static __device__ int sturm_count(const double *alpha, const double *beta, int64_t m, double sigma,
                           double pivmin)
{
    const int lane = threadIdx.x & 63;
    double an = (lane < m) ? alpha[lane] : 0.0;
    double bn = (lane >= 1 && lane < m) ? beta[lane - 1] * beta[lane - 1] : 0.0;
    double q = 1.0;
    int cnt = 0;
    for (int64_t j0 = 0; j0 < m; j0 += 64) {
        const double ac = an, bc = bn;
        const int64_t jn = j0 + 64 + lane;
        an = (jn < m) ? alpha[jn] : 0.0;
        bn = (jn < m) ? beta[jn - 1] * beta[jn - 1] : 0.0;
        if (m - j0 >= 64) {
#pragma unroll
            for (int t = 0; t < 64; ++t) sturm_step(rdlane(ac, t), rdlane(bc, t), sigma, pivmin, q, cnt);
        } else {
            const int c = (int)(m - j0);
            for (int t = 0; t < c; ++t) sturm_step(rdlane(ac, t), rdlane(bc, t), sigma, pivmin, q, cnt);
        }
    }
    return cnt;
}

// theta[i] for i < nwant: the wanted eigenvalues ascending; theta[nwant]: the
// opposite extreme (used for ||T||).
static __device__ double bisect_index(const double *__restrict__ alpha, const double *__restrict__ beta, int64_t m,
                               int64_t idx)
{
    const int lane = threadIdx.x & 63;
    double gl, gu, pivmin;
    gershgorin(alpha, beta, m, &gl, &gu, &pivmin);
    const double tn = fmax(fabs(gl), fabs(gu));
    double lo = gl - 4.0 * EPS * tn - 2.0 * pivmin;
    double hi = gu + 4.0 * EPS * tn + 2.0 * pivmin;
    for (int round = 0; round < 64; ++round) {
        if (hi - lo <= 4.0 * EPS * fmax(fabs(lo), fabs(hi)) || hi - lo <= 2.0 * EPS * tn) break;
        const double sig = lo + (hi - lo) * (double)(lane + 1) / 65.0;
        const int cnt = sturm_count(alpha, beta, m, sig, pivmin);
        const unsigned long long up = __ballot(cnt > idx);
        if (up == 0ull) {
            lo = rdlane(sig, 63);
        } else {
            const int f = __ffsll((long long)up) - 1;
            const double nhi = rdlane(sig, f);
            const double nlo = (f == 0) ? lo : rdlane(sig, f - 1);
            lo = nlo;
            hi = nhi;
        }
    }
    return 0.5 * (lo + hi);
}

// LU of T - lam I with partial pivoting; factors go to f (5 arrays of m):
// u0 (diagonal of U), u1, u2 (super-diagonals), mult, piv (0/1).
static __device__ void tri_lu(const double *alpha, const double *beta, int64_t m, double lam,
                       double pivtiny, double *f)
{
    double *u0 = f, *u1 = f + m, *u2 = f + 2 * m, *ml = f + 3 * m, *pv = f + 4 * m;
    const int lane = threadIdx.x & 63;
    double a = alpha[0] - lam;
    double b = (m > 1) ? beta[0] : 0.0;
    // operands of rows j0..j0+63 and j0+1..j0+64, one per lane; the next
    // chunk's are loaded while a chunk is eliminated
    double nal1 = (lane + 1 < m) ? alpha[lane + 1] - lam : 0.0;
    double nbe0 = (lane < m - 1) ? beta[lane] : 0.0;
    double nbe1 = (lane + 1 < m - 1) ? beta[lane + 1] : 0.0;
    for (int64_t j0 = 0; j0 < m; j0 += 64) {
        const int64_t jl = j0 + lane;
        const double al1 = nal1, be0 = nbe0, be1 = nbe1;
        {
            const int64_t jn = jl + 64;
            nal1 = (jn + 1 < m) ? alpha[jn + 1] - lam : 0.0;
            nbe0 = (jn < m - 1) ? beta[jn] : 0.0;
            nbe1 = (jn + 1 < m - 1) ? beta[jn + 1] : 0.0;
        }
        double r0 = 0.0, r1 = 0.0, r2 = 0.0, rm = 0.0, rp = 0.0;
        const int cnt = (m - j0 < 64) ? (int)(m - j0) : 64;
        for (int t = 0; t < cnt; ++t) {
            const int64_t j = j0 + t;
            double o0, o1, o2, om, op;
            if (j == m - 1) {
                if (fabs(a) < pivtiny) a = (a < 0.0) ? -pivtiny : pivtiny;
                o0 = a; o1 = 0.0; o2 = 0.0; om = 0.0; op = 0.0;
            } else {
                const double sub = rdlane(be0, t);
                const double d1 = rdlane(al1, t);
                const double e1 = rdlane(be1, t);
                if (fabs(a) >= fabs(sub)) {
                    if (fabs(a) < pivtiny) a = (a < 0.0) ? -pivtiny : pivtiny;
                    const double l = sub / a;
                    o0 = a; o1 = b; o2 = 0.0; om = l; op = 0.0;
                    a = d1 - l * b;
                    b = e1;
                } else {
                    const double l = a / sub;
                    o0 = sub; o1 = d1; o2 = e1; om = l; op = 1.0;
                    a = b - l * d1;
                    b = -l * e1;
                }
            }
            if (lane == t) { r0 = o0; r1 = o1; r2 = o2; rm = om; rp = op; }
        }
        if (jl < m) { u0[jl] = r0; u1[jl] = r1; u2[jl] = r2; ml[jl] = rm; pv[jl] = rp; }
    }
}

// x := (T - lam I)^-1 x using the factors (wave 0 only; x in global memory).
static __device__ void tri_solve(const double *f, int64_t m, double *x)
{
    const double *u0 = f, *u1 = f + m, *u2 = f + 2 * m, *ml = f + 3 * m, *pv = f + 4 * m;
    const int lane = threadIdx.x & 63;
    // forward: y = L^-1 P x (the next chunk's operands are loaded while a
    // chunk is processed; they lie beyond the entries this chunk writes)
    double r = x[0];
    double nmm = (lane < m) ? ml[lane] : 0.0;
    double npp = (lane < m) ? pv[lane] : 0.0;
    double nxn = (lane + 1 < m) ? x[lane + 1] : 0.0;
    for (int64_t j0 = 0; j0 < m; j0 += 64) {
        const int64_t jl = j0 + lane;
        const double mm = nmm, pp = npp, xn = nxn;
        {
            const int64_t jn = jl + 64;
            nmm = (jn < m) ? ml[jn] : 0.0;
            npp = (jn < m) ? pv[jn] : 0.0;
            nxn = (jn + 1 < m) ? x[jn + 1] : 0.0;
        }
        double yout = 0.0;
        const int cnt = (m - j0 < 64) ? (int)(m - j0) : 64;
        for (int t = 0; t < cnt; ++t) {
            const int64_t j = j0 + t;
            double y;
            if (j == m - 1) {
                y = r;
            } else {
                const double l = rdlane(mm, t), xj1 = rdlane(xn, t);
                if (rdlane(pp, t) == 0.0) { y = r; r = xj1 - l * r; }
                else { y = xj1; r = r - l * xj1; }
            }
            if (lane == t) yout = y;
        }
        if (jl < m) x[jl] = yout;
    }
    // back: U z = y, from the bottom
    double z1 = 0.0, z2 = 0.0;  // z[j+1], z[j+2]
    // chunks from the bottom; the one above is loaded while a chunk is solved
    double na0, na1, na2, nyv;
    {
        const int64_t j0 = (m - 64 > 0) ? m - 64 : 0;
        const int64_t jl = j0 + lane;
        const bool in = jl < m;
        na0 = in ? u0[jl] : 1.0;
        na1 = in ? u1[jl] : 0.0;
        na2 = in ? u2[jl] : 0.0;
        nyv = in ? x[jl] : 0.0;
    }
    for (int64_t j1 = m; j1 > 0; j1 -= 64) {
        const int64_t j0 = (j1 - 64 > 0) ? j1 - 64 : 0;
        const int64_t jl = j0 + lane;
        const bool in = jl < j1;
        const double a0 = na0, a1 = na1, a2 = na2, yv = nyv;
        if (j0 > 0) {
            const int64_t p0 = (j0 - 64 > 0) ? j0 - 64 : 0;
            const int64_t pl = p0 + lane;
            const bool pin = pl < j0;
            na0 = pin ? u0[pl] : 1.0;
            na1 = pin ? u1[pl] : 0.0;
            na2 = pin ? u2[pl] : 0.0;
            nyv = pin ? x[pl] : 0.0;
        }
        double zout = 0.0;
        for (int t = (int)(j1 - j0) - 1; t >= 0; --t) {
            const double z = (rdlane(yv, t) - rdlane(a1, t) * z1 - rdlane(a2, t) * z2) / rdlane(a0, t);
            z2 = z1;
            z1 = z;
            if (lane == t) zout = z;
        }
        if (in) x[jl] = zout;
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace tdg
