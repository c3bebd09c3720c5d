// Storage / compute precision traits shared by the device kernels.
//   double : stored double, computed double
//   float  : stored float,  computed float
//   bf16   : stored bfloat16 (round-to-nearest-even), computed float
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dwf {

struct bf16s {            // one bfloat16 value, raw bits
    uint16_t bits;
};

template <class S> struct Traits;

template <> struct Traits<double> {
    using R = double;      // compute type
    using C = double2;     // stored complex
    static __device__ __forceinline__ double2 load(const void* base, long i) {
        return reinterpret_cast<const double2*>(base)[i];
    }
    static __device__ __forceinline__ void store(void* base, long i, double re, double im) {
        reinterpret_cast<double2*>(base)[i] = make_double2(re, im);
    }
};

template <> struct Traits<float> {
    using R = float;
    using C = float2;
    static __device__ __forceinline__ double2 load(const void* base, long i) {
        float2 v = reinterpret_cast<const float2*>(base)[i];
        return make_double2(v.x, v.y);
    }
    static __device__ __forceinline__ void store(void* base, long i, float re, float im) {
        reinterpret_cast<float2*>(base)[i] = make_float2(re, im);
    }
};

__device__ __forceinline__ float bf16_to_f32(uint32_t b) {
    return __uint_as_float(b << 16);
}

// Round-to-nearest-even conversion of a finite float to bfloat16 bits;
// NaN is kept quiet.
__device__ __forceinline__ uint32_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return u >> 16;
}

template <> struct Traits<bf16s> {
    using R = float;
    using C = uint32_t;    // (re bits) | (im bits << 16)
    static __device__ __forceinline__ double2 load(const void* base, long i) {
        uint32_t v = reinterpret_cast<const uint32_t*>(base)[i];
        return make_double2(bf16_to_f32(v & 0xffffu), bf16_to_f32(v >> 16));
    }
    static __device__ __forceinline__ void store(void* base, long i, float re, float im) {
        reinterpret_cast<uint32_t*>(base)[i] = f32_to_bf16(re) | (f32_to_bf16(im) << 16);
    }
};

// Load a complex as a pair of compute-type values.
template <class S>
__device__ __forceinline__ void cload(const void* base, long i, typename Traits<S>::R& re,
                                      typename Traits<S>::R& im) {
    if constexpr (sizeof(S) == 8) {
        double2 v = reinterpret_cast<const double2*>(base)[i];
        re = v.x;
        im = v.y;
    } else if constexpr (sizeof(S) == 4) {
        float2 v = reinterpret_cast<const float2*>(base)[i];
        re = v.x;
        im = v.y;
    } else {
        uint32_t v = reinterpret_cast<const uint32_t*>(base)[i];
        re = bf16_to_f32(v & 0xffffu);
        im = bf16_to_f32(v >> 16);
    }
}

template <class S>
__device__ __forceinline__ void cstore(void* base, long i, typename Traits<S>::R re,
                                       typename Traits<S>::R im) {
    Traits<S>::store(base, i, re, im);
}

inline size_t complex_bytes(int kind) { return kind == 0 ? 16 : kind == 1 ? 8 : 4; }

}  // namespace dwf
