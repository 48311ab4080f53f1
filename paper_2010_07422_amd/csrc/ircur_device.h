// Device helpers shared by the IRCUR kernel files: element loads, the fma
// chain of an entry of L_k, the exact threshold test of eq. (4) and the
// rank dispatch.
#pragma once

#include "ircur_internal.h"

namespace ircur {

// ---------------------------------------------------------------- types ---

struct bf16_t { uint16_t bits; };

template <typename T, typename F> __device__ __forceinline__ F ld(const T* p);
template <> __device__ __forceinline__ double ld<double, double>(const double* p) { return *p; }
template <> __device__ __forceinline__ float ld<float, float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float ld<bf16_t, float>(const bf16_t* p) {
    return __uint_as_float(((uint32_t)p->bits) << 16);
}

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// |x| > zeta evaluated exactly: in float, against the largest float <= zeta.
__device__ __forceinline__ bool above(double ax, double z, float) { return ax > z; }
__device__ __forceinline__ bool above(float ax, double, float zf) { return ax > zf; }

template <typename F>
__device__ __forceinline__ F entry_value(F d, F dot, double zeta, float zeta_f, bool* is_out) {
    const F x = d - dot;
    const bool o = above(x < F(0) ? -x : x, zeta, zeta_f);
    *is_out = o;
    return o ? d - x : d;
}

__device__ __forceinline__ double wave_sum(double v) {
    // Fixed butterfly over the 64 lanes: every lane ends with the same sum,
    // formed in the same order on every run.
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Round a float to the nearest bfloat16 (ties to even); NaN stays NaN.
__device__ __forceinline__ bf16_t to_bf16(float v) {
    uint32_t u = __float_as_uint(v);
    bf16_t b;
    if ((u & 0x7fffffffu) > 0x7f800000u) { b.bits = (uint16_t)((u >> 16) | 0x40u); return b; }
    u += 0x7fffu + ((u >> 16) & 1u);
    b.bits = (uint16_t)(u >> 16);
    return b;
}

template <typename T> __device__ __forceinline__ T from_f(double v);
template <> __device__ __forceinline__ double from_f<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16_t from_f<bf16_t>(double v) { return to_bf16((float)v); }

#define IRCUR_RANK_SWITCH(FN, T, F, R, ...)                     \
    switch (R) {                                                \
        case 1: return FN<T, F, 1>(__VA_ARGS__);                \
        case 2: return FN<T, F, 2>(__VA_ARGS__);                \
        case 3: return FN<T, F, 3>(__VA_ARGS__);                \
        case 4: return FN<T, F, 4>(__VA_ARGS__);                \
        case 5: return FN<T, F, 5>(__VA_ARGS__);                \
        case 6: return FN<T, F, 6>(__VA_ARGS__);                \
        case 8: return FN<T, F, 8>(__VA_ARGS__);                \
        case 10: return FN<T, F, 10>(__VA_ARGS__);              \
        case 12: return FN<T, F, 12>(__VA_ARGS__);              \
        case 16: return FN<T, F, 16>(__VA_ARGS__);              \
        case 20: return FN<T, F, 20>(__VA_ARGS__);              \
        case 24: return FN<T, F, 24>(__VA_ARGS__);              \
        case 32: return FN<T, F, 32>(__VA_ARGS__);              \
        default: return hipErrorInvalidValue;                   \
    }


}  // namespace ircur
