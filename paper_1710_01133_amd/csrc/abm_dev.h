// Device-side helpers shared by the libabm kernels: the fixed set of
// right-hand sides f(t, y) of the Caputo problem (eq. fde) and wavefront
// reductions.  Included only by libabm's own .hip files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "abm.h"

namespace abm {

constexpr int kWave = 64;

// Pointers into device memory that the kernels read from descriptors are
// generic to the compiler, which then emits flat memory instructions; flat
// loads also count against the LDS wait counter, so every wait for an LDS
// operand would wait for the HBM prefetch in flight as well.  Kernels
// therefore access such memory through global-address-space pointers.
#define ABM_GLOBAL __attribute__((address_space(1)))
template <typename T>
using gptr = ABM_GLOBAL T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p)
{
    return (gptr<T>)p;
}

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
    } else if constexpr (R == ABM_RHS_DIAG) {
        f[0] = -p[0] * y[0] + p[2];
        f[1] = -p[1] * y[1] + p[3];
    }
}

// The part of f(t, y) that depends on t only (the forcing), so that it can be
// evaluated ahead of a sequential chain: rhs_eval_forced(p, y, force, f)
// equals rhs_eval(p, t, y, f) when force = forcing<R>(p, t).
template <int R>
__device__ __forceinline__ double forcing(const double* __restrict__ p, double t)
{
    if constexpr (R == ABM_RHS_DUFFING) return p[1] * cos(p[2] * t);
    else if constexpr (R == ABM_RHS_POLY) return p[0] + p[1] * t;
    else if constexpr (R == ABM_RHS_LCR) return p[4] * sin(p[1] * t);
    else return 0.0;
}

template <int R, int D>
__device__ __forceinline__ void rhs_eval_forced(const double* __restrict__ p, const double* y,
                                                double force, double* f)
{
    if constexpr (R == ABM_RHS_LINEAR) {
        f[0] = -p[0] * y[0];
    } else if constexpr (R == ABM_RHS_DUFFING) {
        f[0] = y[1];
        f[1] = -p[0] * y[1] - y[0] - y[0] * y[0] * y[0] + force;
    } else if constexpr (R == ABM_RHS_LORENZ) {
        f[0] = p[0] * (y[1] - y[0]);
        f[1] = y[0] * (p[1] - y[2]) - y[1];
        f[2] = y[0] * y[1] - p[2] * y[2];
    } else if constexpr (R == ABM_RHS_POLY) {
        f[0] = force;
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
        f[1] = -p[0] * y[1] - y[0] + force;
    } else if constexpr (R == ABM_RHS_DIAG) {
        f[0] = -p[0] * y[0] + p[2];
        f[1] = -p[1] * y[1] + p[3];
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

// bf16 helpers: round-to-nearest-even of a finite float, and back.
__device__ __forceinline__ uint16_t bf16_rn(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f(uint16_t h)
{
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}
// Split x (rounded once to float) into bf16 terms t0 + t1 + t2 that carry its
// 24 significant bits; t0 + t1 alone keep 16 of them.
__device__ __forceinline__ void bf16_split3(double x, uint16_t* t)
{
    const float x32 = (float)x;
    t[0] = bf16_rn(x32);
    const float r1 = x32 - bf16_f(t[0]);
    t[1] = bf16_rn(r1);
    t[2] = bf16_rn(r1 - bf16_f(t[1]));
}

// Index of history row k >= 1, column col, in the k-blocked layout of the
// bf16 history copies: 8 consecutive rows of one column are contiguous.
__device__ __forceinline__ int64_t kblocked_index(int64_t k, int64_t col, int64_t ld)
{
    return (((k - 1) >> 3) * ld + col) * 8 + ((k - 1) & 7);
}

// Index of history row k >= 1, column col, in the layout of the int8 history
// limbs: 16 consecutive rows of one column are contiguous (one 16-byte operand
// of the int8 matrix product).
__device__ __forceinline__ int64_t q16_index(int64_t k, int64_t col, int64_t ld)
{
    return (((k - 1) >> 4) * ld + col) * 16 + ((k - 1) & 15);
}

// Index of history row k, column col, in the column-blocked layout of the
// float history copy: 16 columns form a block and each block stores its rows
// contiguously (rows * 16 floats), so a far-field workgroup reading one block
// streams whole cache lines.
__device__ __forceinline__ int64_t colblocked_index(int64_t k, int64_t col, int64_t rows)
{
    return ((col >> 4) * rows + k) * 16 + (col & 15);
}

// Device status word bits (written with atomic OR, read by the host).
constexpr uint32_t kStatusTimeout = 1u;   // a bounded device-side wait gave up
constexpr uint32_t kStatusNonFinite = 2u; // a state became NaN/Inf

__device__ __forceinline__ void raise_status(uint32_t* st, uint32_t bit)
{
    __hip_atomic_fetch_or(st, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace abm
