// Device-side helpers shared by the libabm kernels: the fixed set of
// right-hand sides f(t, y) of the Caputo problem (eq. fde) and wavefront
// reductions.  Included only by libabm's own .hip files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm.h"

namespace abm {

constexpr int kWave = 64;

// f(t, y) for the right-hand side R (enum abm_rhs) of dimension D.
template <int R, int D>
__device__ __forceinline__ void rhs_eval(const double* __restrict__ p, double t, const double* y,
                                         double* f)
{
    if constexpr (R == ABM_RHS_LINEAR) {
        f[0] = -p[0] * y[0];
    } else if constexpr (R == ABM_RHS_DUFFING) {
        f[0] = y[1];
        f[1] = -p[0] * y[1] - y[0] - y[0] * y[0] * y[0] + p[1] * cos(p[2] * t);
    } else if constexpr (R == ABM_RHS_LORENZ) {
        f[0] = p[0] * (y[1] - y[0]);
        f[1] = y[0] * (p[1] - y[2]) - y[1];
        f[2] = y[0] * y[1] - p[2] * y[2];
    } else if constexpr (R == ABM_RHS_POLY) {
        f[0] = p[0] + p[1] * t;
    } else if constexpr (R == ABM_RHS_LCR) {
        const double x = y[0];
        double g;
        if (x <= -1.0)
            g = p[3] * x - p[2] + p[3];
        else if (x >= 1.0)
            g = p[3] * x + p[2] - p[3];
        else
            g = p[2] * x;
        f[0] = y[1] - g;
        f[1] = -p[0] * y[1] - y[0] + p[4] * sin(p[1] * t);
    }
}

// Butterfly sum over the 64 lanes of a wavefront.  Every lane ends with the
// same bits: each stage adds a value and its partner's (x + y == y + x).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, kWave);
    return v;
}

__device__ __forceinline__ void spin_pause() { __builtin_amdgcn_s_sleep(1); }

template <typename T>
__device__ __forceinline__ T ld_acquire(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_release(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Device status word bits (written with atomic OR, read by the host).
constexpr uint32_t kStatusTimeout = 1u;   // a bounded device-side wait gave up
constexpr uint32_t kStatusNonFinite = 2u; // a state became NaN/Inf

__device__ __forceinline__ void raise_status(uint32_t* st, uint32_t bit)
{
    __hip_atomic_fetch_or(st, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace abm
