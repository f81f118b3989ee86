// Storage codecs of the distributions.
//
// FP64 and FP32 store values as they are.  FP16 and BF16 store shifted and
// scaled populations, (f - shift) * scale, rounded to nearest-even; loads
// invert that in FP32.  Shift removes the part every node shares (w_j * phi_ref
// for h); scale (a power of two) lifts small populations out of the FP16
// subnormal range.  BF16 rounding is written out from the IEEE-754 binary32
// layout: keep the upper 16 bits, round half to even, keep NaNs quiet.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pulbm {

struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

template <class S> struct Codec;

template <> struct Codec<double> {
    using CT = double;  // compute type
    static constexpr int BYTES = 8;
    __device__ static __forceinline__ double load(const double* p, size_t i, double, double) { return p[i]; }
    __device__ static __forceinline__ void store(double* p, size_t i, double v, double, double) { p[i] = v; }
};

template <> struct Codec<float> {
    using CT = float;
    static constexpr int BYTES = 4;
    __device__ static __forceinline__ float load(const float* p, size_t i, float, float) { return p[i]; }
    __device__ static __forceinline__ void store(float* p, size_t i, float v, float, float) { p[i] = v; }
};

template <> struct Codec<_Float16> {
    using CT = float;
    static constexpr int BYTES = 2;
    __device__ static __forceinline__ float load(const _Float16* p, size_t i, float inv_scale, float shift)
    {
        return fmaf((float)p[i], inv_scale, shift);
    }
    __device__ static __forceinline__ void store(_Float16* p, size_t i, float v, float scale, float shift)
    {
        p[i] = (_Float16)((v - shift) * scale);
    }
};

template <> struct Codec<bf16_t> {
    using CT = float;
    static constexpr int BYTES = 2;
    __device__ static __forceinline__ float load(const bf16_t* p, size_t i, float inv_scale, float shift)
    {
        return fmaf(bf16_to_f32(p[i].bits), inv_scale, shift);
    }
    __device__ static __forceinline__ void store(bf16_t* p, size_t i, float v, float scale, float shift)
    {
        p[i].bits = f32_to_bf16_rne((v - shift) * scale);
    }
};

}  // namespace pulbm
