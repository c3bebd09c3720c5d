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

// Two floats to a pair of bfloat16 (lo = re, hi = im), round to nearest
// even, NaN stays NaN: one gfx950 v_cvt_pk_bf16_f32.  Checked against the
// bit-level rounding rule over every 32-bit pattern.
typedef __bf16 bf16x2_v __attribute__((ext_vector_type(2)));
typedef float f32x2_v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float re, float im) {
    const f32x2_v f = {re, im};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_v));
}

template <> struct Traits<bf16s> {
    using R = float;
    using C = uint32_t;    // (re bits) | (im bits << 16)
    static __device__ __forceinline__ double2 load(const void* base, long i) {
        uint32_t v = reinterpret_cast<const uint32_t*>(base)[i];
        return make_double2(bf16_to_f32(v & 0xffffu), bf16_to_f32(v >> 16));
    }
    static __device__ __forceinline__ void store(void* base, long i, float re, float im) {
        reinterpret_cast<uint32_t*>(base)[i] = pack_bf16(re, im);
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
        *reinterpret_cast<uint32_t*>(p) = pack_bf16(re, im);
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

template <class S, int AUX = 0>
__device__ __forceinline__ void bload(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                      typename Traits<S>::R& re, typename Traits<S>::R& im) {
    if constexpr (sizeof(S) == 8) {
        u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX);
        re = __hiloint2double(v.y, v.x);
        im = __hiloint2double(v.w, v.z);
    } else if constexpr (sizeof(S) == 4) {
        u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
        re = __uint_as_float(v.x);
        im = __uint_as_float(v.y);
    } else {
        unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX);
        re = bf16_to_f32(v & 0xffffu);
        im = bf16_to_f32(v >> 16);
    }
}

template <class S, int AUX = 0>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                       typename Traits<S>::R re, typename Traits<S>::R im) {
    if constexpr (sizeof(S) == 8) {
        u32x4 v;
        v.x = (unsigned)__double2loint(re);
        v.y = (unsigned)__double2hiint(re);
        v.z = (unsigned)__double2loint(im);
        v.w = (unsigned)__double2hiint(im);
        __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, AUX);
    } else if constexpr (sizeof(S) == 4) {
        u32x2 v;
        v.x = __float_as_uint(re);
        v.y = __float_as_uint(im);
        __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, AUX);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(pack_bf16(re, im), r, voff, soff, AUX);
    }
}

// bytes of one stored complex
template <class S> constexpr unsigned cbytes() { return sizeof(S) == 8 ? 16u : sizeof(S) == 4 ? 8u : 4u; }

// ---------------------------------------------------------------------
// Internal layouts.
//
// Fields: element (row, site), row = s * 12 + comp (further right-hand sides
// and channels continue the row count), at complex index
//   ((row / P) * Vhp + site) * P + row % P
// with P = 1 for FP64, 2 for FP32 and 4 for BF16: P consecutive spin-colour
// components of a site are contiguous (16 bytes) and consecutive sites follow
// each other, so a wave's load of one group for 16 consecutive sites reads one
// contiguous 256-byte run with a single 128-bit load per lane.  Kernels that
// mix storage kinds element by element (conversions, CG updates with FP32 x, r
// and BF16 p, w) index each operand in its own layout (blas.hip).
//
// Links: LP = 16 / (complex bytes) elements of one site's 3x3 matrix share
// a 16-byte group; direction d has NG = ceil(9 / LP) groups:
//   element (d, e, site) at ((d * NG + e / LP) * Vhp + site) * LP + e % LP.
// ---------------------------------------------------------------------
// Compile-time layout switches (measured on MI355X, see the hop kernel):
// DWF_FIELD_PAIRS groups FP32/BF16 components in pairs, DWF_LINK_PACK packs
// link elements in 16-byte groups.
#ifndef DWF_FIELD_PAIRS
#define DWF_FIELD_PAIRS 1
#endif
#ifndef DWF_LINK_PACK
#define DWF_LINK_PACK 1
#endif
__host__ __device__ __forceinline__ long fidx(long row, long site, long Vhp, int P) {
    return P == 1 ? row * Vhp + site : (P == 2 ? ((row >> 1) * Vhp + site) * 2 + (row & 1)
                                               : ((row >> 2) * Vhp + site) * 4 + (row & 3));
}
// components per group: FP64 1, FP32 2, BF16 4 (16 bytes per site and group)
template <class S> constexpr int fpack() {
    return (sizeof(S) == 8 || !DWF_FIELD_PAIRS) ? 1 : (sizeof(S) == 4 ? 2 : 4);
}
inline int fpack_of(int kind) { return (kind == 0 || !DWF_FIELD_PAIRS) ? 1 : (kind == 1 ? 2 : 4); }
__host__ __device__ constexpr int link_lp(int cb) { return DWF_LINK_PACK ? 16 / cb : 1; }
__host__ __device__ constexpr int link_ng(int cb) { return (9 + link_lp(cb) - 1) / link_lp(cb); }
__host__ __device__ __forceinline__ long lidx(int d, int e, long site, long Vhp, int cb) {
    return (((long)d * link_ng(cb) + e / link_lp(cb)) * Vhp + site) * link_lp(cb) + e % link_lp(cb);
}
// complex elements of the link table of one parity
inline long link_elems_parity(long Vhp, int cb) { return 8L * link_ng(cb) * link_lp(cb) * Vhp; }

// Components 4g .. 4g+3 of one site with whole-group accesses (16 bytes per
// access when the layout packs 16 bytes per group): v = re0, im0, ..., re3, im3.
template <class S>
__device__ __forceinline__ void load4(const void* base, long g, long site, long Vhp,
                                      typename Traits<S>::R (&v)[8]) {
    constexpr int P = fpack<S>();
    if constexpr (P == 4) {   // BF16 quads
        const uint4 w = reinterpret_cast<const uint4*>(base)[g * Vhp + site];
        const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = bf16_to_f32(u[k] & 0xffffu);
            v[2 * k + 1] = bf16_to_f32(u[k] >> 16);
        }
    } else if constexpr (P == 2 && sizeof(S) == 4) {   // FP32 pairs
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float4 w = reinterpret_cast<const float4*>(base)[(2 * g + j) * Vhp + site];
            v[4 * j] = w.x;
            v[4 * j + 1] = w.y;
            v[4 * j + 2] = w.z;
            v[4 * j + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) cload<S>(base, fidx(4 * g + k, site, Vhp, P), v[2 * k], v[2 * k + 1]);
    }
}

template <class S>
__device__ __forceinline__ void store4(void* base, long g, long site, long Vhp,
                                       const typename Traits<S>::R (&v)[8]) {
    constexpr int P = fpack<S>();
    if constexpr (P == 4) {
        uint4 w;
        w.x = pack_bf16(v[0], v[1]);
        w.y = pack_bf16(v[2], v[3]);
        w.z = pack_bf16(v[4], v[5]);
        w.w = pack_bf16(v[6], v[7]);
        reinterpret_cast<uint4*>(base)[g * Vhp + site] = w;
    } else if constexpr (P == 2 && sizeof(S) == 4) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
            reinterpret_cast<float4*>(base)[(2 * g + j) * Vhp + site] =
                make_float4(v[4 * j], v[4 * j + 1], v[4 * j + 2], v[4 * j + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) cstore<S>(base, fidx(4 * g + k, site, Vhp, P), v[2 * k], v[2 * k + 1]);
    }
}

// One group of fpack<S>() complex (voff = site * group bytes, soff = the
// group row's byte offset).  v = re0, im0, re1, im1, ...
template <class S>
__device__ __forceinline__ void bload_group(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff,
                                            typename Traits<S>::R (&v)[8]) {
    if constexpr (fpack<S>() == 1) {
        bload<S>(r, voff, soff, v[0], v[1]);
    } else if constexpr (sizeof(S) == 4) {
        u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        v[0] = __uint_as_float(w.x);
        v[1] = __uint_as_float(w.y);
        v[2] = __uint_as_float(w.z);
        v[3] = __uint_as_float(w.w);
    } else if constexpr (fpack<S>() == 2) {
        u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        v[0] = bf16_to_f32(w.x & 0xffffu);
        v[1] = bf16_to_f32(w.x >> 16);
        v[2] = bf16_to_f32(w.y & 0xffffu);
        v[3] = bf16_to_f32(w.y >> 16);
    } else {
        u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = bf16_to_f32(u[k] & 0xffffu);
            v[2 * k + 1] = bf16_to_f32(u[k] >> 16);
        }
    }
}

// Decode one 16-byte link group g (elements LP*g .. LP*g+LP-1) into U.
template <class S>
__device__ __forceinline__ void decode_link_group(u32x4 w, int g, typename Traits<S>::R (&U)[18]) {
    constexpr int LP = link_lp(cbytes<S>());
    static_assert(LP * cbytes<S>() == 16, "16-byte link groups expected");
    if constexpr (sizeof(S) == 8) {
        U[2 * g] = __hiloint2double(w.y, w.x);
        U[2 * g + 1] = __hiloint2double(w.w, w.z);
    } else if constexpr (sizeof(S) == 4) {
        U[4 * g] = __uint_as_float(w.x);
        U[4 * g + 1] = __uint_as_float(w.y);
        if (2 * g + 1 < 9) {
            U[4 * g + 2] = __uint_as_float(w.z);
            U[4 * g + 3] = __uint_as_float(w.w);
        }
    } else {
        const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (LP * g + k < 9) {
                U[2 * (LP * g + k)] = bf16_to_f32(u[k] & 0xffffu);
                U[2 * (LP * g + k) + 1] = bf16_to_f32(u[k] >> 16);
            }
    }
}

// The 3x3 link of direction d at one site: voff = site * group bytes,
// soff = d * NG * group row bytes, gstride = group row bytes.  U = re, im of
// elements 0..8.
template <class S>
__device__ __forceinline__ void bload_link(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, unsigned gstride,
                                           typename Traits<S>::R (&U)[18]) {
    constexpr int CB = cbytes<S>(), LP = link_lp(CB), NG = link_ng(CB);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if constexpr (LP == 1) {
            bload<S>(r, voff, soff + (unsigned)g * gstride, U[2 * g], U[2 * g + 1]);
        } else {
            u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff + (unsigned)g * gstride, 0);
            if constexpr (sizeof(S) == 8) {
                U[2 * g] = __hiloint2double(w.y, w.x);
                U[2 * g + 1] = __hiloint2double(w.w, w.z);
            } else if constexpr (sizeof(S) == 4) {
                U[4 * g] = __uint_as_float(w.x);
                U[4 * g + 1] = __uint_as_float(w.y);
                if (2 * g + 1 < 9) {
                    U[4 * g + 2] = __uint_as_float(w.z);
                    U[4 * g + 3] = __uint_as_float(w.w);
                }
            } else {
                const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (LP * g + k < 9) {
                        U[2 * (LP * g + k)] = bf16_to_f32(u[k] & 0xffffu);
                        U[2 * (LP * g + k) + 1] = bf16_to_f32(u[k] >> 16);
                    }
            }
        }
    }
}

inline size_t complex_bytes(int kind) { return kind == 0 ? 16 : kind == 1 ? 8 : 4; }

}  // namespace dwf
