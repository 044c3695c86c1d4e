// chain.h -- device helpers of the chained (persistent) triangular-solve
// kernels: sentinel-staged publication of solved values, bounded polling,
// chain-ordered tickets and the last-workgroup reset.
#pragma once

#include "internal.h"

namespace chain {

__device__ __forceinline__ unsigned long long ld_bits(const double *p)
{
    return __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_bits(double *p, unsigned long long v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Bound on the polls of one wait: the host may lower it (tests of the
// expiry path force the condition this way); 0 selects SPIN_LIMIT.  It is
// read only once a wait has polled SPIN_FREE times, so a short wait on the
// chain's critical path never pays for the extra load; smaller bounds act
// as SPIN_FREE.
#define SPIN_FREE 32u
__device__ __forceinline__ unsigned spin_bound(PCtl *ctl)
{
    const unsigned s = __hip_atomic_load(&ctl->spin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return s ? (s > SPIN_FREE ? s : SPIN_FREE) : SPIN_LIMIT;
}

// Finish a poll started with ld_bits: spin (bounded) while the value is the
// sentinel.  An expired wait records an error and yields 0.
__device__ __noinline__ double settle_slow(unsigned long long v, const double *p, PCtl *ctl)
{
    unsigned it = 0, lim = 0;
    while (v == STAGE_SENTINEL) {
        if (++it > SPIN_FREE) {
            if (!lim) lim = spin_bound(ctl);
            if (it > lim) {
                __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return 0.0;
            }
        }
        __builtin_amdgcn_s_sleep(2);  // fewer polls on lines every waiting workgroup reads
        v = ld_bits(p);
    }
    return __longlong_as_double((long long)v);
}

__device__ __forceinline__ double settle(unsigned long long v, const double *p, PCtl *ctl)
{
    if (__builtin_expect(v != STAGE_SENTINEL, 1)) return __longlong_as_double((long long)v);
    return settle_slow(v, p, ctl);
}

// The same with a longer sleep between polls, for waits off the chain's
// critical path (values a workgroup needs only several links later): fewer
// requests on the lines the next link is waiting for.
__device__ __noinline__ double settle_lazy_slow(unsigned long long v, const double *p, PCtl *ctl)
{
    unsigned it = 0, lim = 0;
    while (v == STAGE_SENTINEL) {
        if (++it > SPIN_FREE) {
            if (!lim) lim = spin_bound(ctl);
            if (it > lim) {
                __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return 0.0;
            }
        }
        __builtin_amdgcn_s_sleep(16);
        v = ld_bits(p);
    }
    return __longlong_as_double((long long)v);
}

__device__ __forceinline__ double settle_lazy(unsigned long long v, const double *p, PCtl *ctl)
{
    if (__builtin_expect(v != STAGE_SENTINEL, 1)) return __longlong_as_double((long long)v);
    return settle_lazy_slow(v, p, ctl);
}

__device__ __forceinline__ double rdlane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// Chain position of this workgroup.  A counter left inconsistent by an
// earlier failure is reported (GSYEIG_ESPIN) and folded into range, so every
// index stays in bounds.
__device__ int take_ticket(PCtl *ctl, int nblk)
{
    unsigned t = atomicAdd(&ctl->ticket, 1u);
    if (t >= (unsigned)nblk) {
        __hip_atomic_store(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t %= (unsigned)nblk;
    }
    return (int)t;
}

// Count this workgroup out; the last one restores the staging sentinels
// (and those of an optional second staging vector) and resets the counters
// for the next launch.
__device__ void retire(PCtl *ctl, double *stage, int64_t nstage, int nblk, int *s_last,
                       double *stage2 = nullptr)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned d = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        *s_last = (d == (unsigned)nblk - 1u);
    }
    __syncthreads();
    if (*s_last) {
        for (int64_t j = threadIdx.x; j < nstage; j += blockDim.x) {
            st_bits(stage + j, STAGE_SENTINEL);
            if (stage2) st_bits(stage2 + j, STAGE_SENTINEL);
        }
        if (threadIdx.x == 0) {
            __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace chain
