// Helpers of the weakly-synchronous runs of libat.so (1D and 3D): bounded
// polling of per-edge / per-block level counters, the announce after
// device-coherent ring stores, and the idle-time noise.
#pragma once

#include "at_internal.h"

namespace atk {

namespace {

// Pseudo-random idle time before a step (emulated arrival noise): a 32-bit
// integer mix of (seed, tile, step); any mixer serves, it only spreads the
// progress of the tiles.
__device__ __forceinline__ uint32_t ws_mix(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u ^ (c + 0x165667B1u) * 0xC2B2AE3Du;
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    return h;
}

__device__ __forceinline__ void ws_idle(int32_t jitter, uint64_t seed, int64_t who, int64_t n)
{
    if (jitter <= 0) return;
    const uint32_t idle = ws_mix((uint32_t)seed, (uint32_t)who, (uint32_t)n) % (uint32_t)(jitter + 1);
    for (uint32_t i = 0; i < idle; ++i) __builtin_amdgcn_s_sleep(2);
}

// Device-coherent load and store of a double: they read past, and write
// through, the per-XCD L2, so ring values pass between workgroups on
// different XCDs without any cache-wide write-back or invalidate.
__device__ __forceinline__ double ld_coherent(const double *p)
{
    return __longlong_as_double((long long)__hip_atomic_load(
        reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
        __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void st_coherent(double *p, double v)
{
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                       (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t load_relaxed(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Announce level v on a counter: the device-coherent ring stores issued
// before it have completed (vmcnt 0) when the counter store is issued, so a
// reader that sees v and then loads the ring sees the values.
__device__ __forceinline__ void announce(int32_t *p, int32_t v)
{
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until the counter announces at least level `need`; returns the newest
// announced level, or -2 when the spin limit passed or another workgroup
// raised the error flag (the flag is then set).  The polls are relaxed
// device-scope loads; the ring reads that follow are issued after the last
// poll has returned.
__device__ int32_t ws_wait(const int32_t *cnt, int32_t need, int32_t *err, int64_t spin_limit)
{
    int32_t t = load_relaxed(cnt);
    int64_t spins = 0;
    while (t < need) {
        if (++spins > spin_limit) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -2;
        }
        if ((spins & 63) == 0 && load_relaxed(err) != 0) return -2;
        __builtin_amdgcn_s_sleep(1);
        t = load_relaxed(cnt);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return t;
}

}  // namespace

}  // namespace atk
