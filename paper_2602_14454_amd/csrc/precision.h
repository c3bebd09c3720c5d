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

// Loads/stores addressed as (wave-uniform base pointer, 32-bit per-lane byte
// offset).  Kernels keep the uniform part (field, right-hand side, component
// row) in scalar registers and only a 32-bit offset per lane, so the
// compiler can use the scalar-base form of global loads instead of keeping
// 64-bit addresses in vector registers.
template <class S>
__device__ __forceinline__ void cload_b(const void* base, unsigned boff, typename Traits<S>::R& re,
                                        typename Traits<S>::R& im) {
    const char* p = static_cast<const char*>(base) + boff;
    if constexpr (sizeof(S) == 8) {
        double2 v = *reinterpret_cast<const double2*>(p);
        re = v.x;
        im = v.y;
    } else if constexpr (sizeof(S) == 4) {
        float2 v = *reinterpret_cast<const float2*>(p);
        re = v.x;
        im = v.y;
    } else {
        uint32_t v = *reinterpret_cast<const uint32_t*>(p);
        re = bf16_to_f32(v & 0xffffu);
        im = bf16_to_f32(v >> 16);
    }
}

template <class S>
__device__ __forceinline__ void cstore_b(void* base, unsigned boff, typename Traits<S>::R re,
                                         typename Traits<S>::R im) {
    char* p = static_cast<char*>(base) + boff;
    if constexpr (sizeof(S) == 8) {
        *reinterpret_cast<double2*>(p) = make_double2(re, im);
    } else if constexpr (sizeof(S) == 4) {
        *reinterpret_cast<float2*>(p) = make_float2(re, im);
    } else {
        *reinterpret_cast<uint32_t*>(p) = f32_to_bf16(re) | (f32_to_bf16(im) << 16);
    }
}

// Buffer-resource access (raw buffers, stride 0): a 128-bit descriptor in
// scalar registers holds the base and the byte range; each access adds a
// 32-bit per-lane byte offset (vector register) and a 32-bit wave-uniform
// byte offset (scalar register).  Accesses outside the range read zero and
// drop writes.  The last descriptor word is the gfx9-family default.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)nbytes, 0x00020000);
}

template <class S>
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                      typename Traits<S>::R& re, typename Traits<S>::R& im) {
    if constexpr (sizeof(S) == 8) {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        re = __hiloint2double(v.y, v.x);
        im = __hiloint2double(v.w, v.z);
    } else if constexpr (sizeof(S) == 4) {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        re = __uint_as_float(v.x);
        im = __uint_as_float(v.y);
    } else {
        unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
        re = bf16_to_f32(v & 0xffffu);
        im = bf16_to_f32(v >> 16);
    }
}

template <class S>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                       typename Traits<S>::R re, typename Traits<S>::R im) {
    if constexpr (sizeof(S) == 8) {
        u32x4 v;
        v.x = (unsigned)__double2loint(re);
        v.y = (unsigned)__double2hiint(re);
        v.z = (unsigned)__double2loint(im);
        v.w = (unsigned)__double2hiint(im);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, 0);
    } else if constexpr (sizeof(S) == 4) {
        u32x2 v;
        v.x = __float_as_uint(re);
        v.y = __float_as_uint(im);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, 0);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(f32_to_bf16(re) | (f32_to_bf16(im) << 16), r, voff, soff, 0);
    }
}

// bytes of one stored complex
template <class S> constexpr unsigned cbytes() { return sizeof(S) == 8 ? 16u : sizeof(S) == 4 ? 8u : 4u; }

inline size_t complex_bytes(int kind) { return kind == 0 ? 16 : kind == 1 ? 8 : 4; }

}  // namespace dwf
