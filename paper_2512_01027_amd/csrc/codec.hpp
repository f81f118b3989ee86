// Storage codecs of the distributions.
//
// FP64 and FP32 store values as they are.  FP16 and BF16 store shifted and
// scaled populations, (f - shift) * scale, rounded to nearest-even; loads
// invert that in FP32.  The shift removes the large part of a population that
// its reader can rebuild on its own (w_j times its own phi of the step before,
// for h); the scale (a power of two) lifts the small remainder out of the
// FP16 subnormal range.  BF16 rounding is written out from the IEEE-754 binary32
// layout: keep the upper 16 bits, round half to even, keep NaNs quiet.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pulbm {

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

#define PULBM_GLB __attribute__((address_space(1)))
#define PULBM_CST __attribute__((address_space(4)))

template <class S> struct Codec;

template <> struct Codec<double> {
    using CT = double;  // compute type
    static constexpr int BYTES = 8;
    __device__ static __forceinline__ double dec(double v, double, double) { return v; }
    __device__ static __forceinline__ double enc(double v, double, double) { return v; }
};

template <> struct Codec<float> {
    using CT = float;
    static constexpr int BYTES = 4;
    __device__ static __forceinline__ float dec(float v, float, float) { return v; }
    __device__ static __forceinline__ float enc(float v, float, float) { return v; }
};

template <> struct Codec<_Float16> {
    using CT = float;
    static constexpr int BYTES = 2;
    __device__ static __forceinline__ float dec(_Float16 v, float inv_scale, float shift)
    {
        return fmaf((float)v, inv_scale, shift);
    }
    __device__ static __forceinline__ _Float16 enc(float v, float scale, float shift)
    {
        return (_Float16)((v - shift) * scale);
    }
};

// BF16 storage: the upper 16 bits of a binary32, held in a uint16_t.
template <> struct Codec<uint16_t> {
    using CT = float;
    static constexpr int BYTES = 2;
    __device__ static __forceinline__ float dec(uint16_t v, float inv_scale, float shift)
    {
        return fmaf(bf16_to_f32(v), inv_scale, shift);
    }
    __device__ static __forceinline__ uint16_t enc(float v, float scale, float shift)
    {
        return f32_to_bf16_rne((v - shift) * scale);
    }
};

}  // namespace pulbm
