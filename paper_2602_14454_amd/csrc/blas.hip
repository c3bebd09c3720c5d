// Vector kernels on internal half fields: layout conversion, precision
// conversion, CG updates and deterministic FP64 reductions.
//
// Reductions: every kernel that reduces writes one FP64 partial per block
// (wavefront __shfl_xor tree, then the block's waves in order); a single
// block then sums the partials in a fixed order.  No floating-point atomics,
// so results are bit-reproducible run to run.
#include <type_traits>

#include "blas.h"
#include "dwf_internal.h"
#include "precision.h"

namespace dwf {

constexpr int BLAS_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------
// canonical complex128 <-> internal layout
// ---------------------------------------------------------------------
// Full 5D canonical: src[((r*Ls + s)*V + lex)*12 + comp]
template <class S>
__global__ void pack_full_kernel(void* dst, const double2* src, const int* lex_of_site, long Vh, long Vhp,
                                 long V, long nslices) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nslices * Vh) return;
    const long rs = idx / Vh, eo = idx % Vh;
    const long lex = lex_of_site[eo];
    const double2* in = src + (rs * V + lex) * 12;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        double2 v = in[cp];
        cstore<S>(dst, fidx(rs * 12 + cp, eo, Vhp, fpack<S>()), (typename Traits<S>::R)v.x, (typename Traits<S>::R)v.y);
    }
}

template <class S>
__global__ void unpack_full_kernel(double2* dst, const void* src, const int* lex_of_site, long Vh, long Vhp,
                                   long V, long nslices) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nslices * Vh) return;
    const long rs = idx / Vh, eo = idx % Vh;
    const long lex = lex_of_site[eo];
    double2* out = dst + (rs * V + lex) * 12;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        typename Traits<S>::R re, im;
        cload<S>(src, fidx(rs * 12 + cp, eo, Vhp, fpack<S>()), re, im);
        out[cp] = make_double2((double)re, (double)im);
    }
}

// Even canonical: src[((r*Ls + s)*Vh + eo)*12 + comp], eo = lex >> 1;
// internal site i holds lex_of_site[i].
template <class S>
__global__ void pack_half_kernel(void* dst, const double2* src, const int* lex_of_site, long Vh, long Vhp,
                                 long nslices) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nslices * Vh) return;
    const long rs = idx / Vh, i = idx % Vh;
    const long eo = lex_of_site[i] >> 1;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        double2 v = src[(rs * Vh + eo) * 12 + cp];
        cstore<S>(dst, fidx(rs * 12 + cp, i, Vhp, fpack<S>()), (typename Traits<S>::R)v.x, (typename Traits<S>::R)v.y);
    }
}

template <class S>
__global__ void unpack_half_kernel(double2* dst, const void* src, const int* lex_of_site, long Vh, long Vhp,
                                   long nslices) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nslices * Vh) return;
    const long rs = idx / Vh, i = idx % Vh;
    const long eo = lex_of_site[i] >> 1;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        typename Traits<S>::R re, im;
        cload<S>(src, fidx(rs * 12 + cp, i, Vhp, fpack<S>()), re, im);
        dst[(rs * Vh + eo) * 12 + cp] = make_double2((double)re, (double)im);
    }
}

// 4D canonical -> two-slice half field of one parity: slice 0 = P+ b4, slice 1 = P- b4
template <class S>
__global__ void pack_chiral_pair_kernel(void* dst, const double2* b4, const int* lex_of_site, long Vh, long Vhp) {
    const long eo = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (eo >= Vh) return;
    const long lex = lex_of_site[eo];
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        double2 v = b4[lex * 12 + cp];
        const bool up = cp < 6;
        cstore<S>(dst, fidx(cp, eo, Vhp, fpack<S>()), up ? v.x : 0.0, up ? v.y : 0.0);
        cstore<S>(dst, fidx(12 + cp, eo, Vhp, fpack<S>()), up ? 0.0 : v.x, up ? 0.0 : v.y);
    }
}

// x4[lex] = P_- x5(s=0)[lex] + P_+ x5(s=Ls-1)[lex], canonical complex128
__global__ void project4d_kernel(double2* x4, const double2* x5, long V, int Ls) {
    const long lex = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= V) return;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        const bool up = cp < 6;   // P_+ components come from s = Ls-1, P_- from s = 0
        x4[lex * 12 + cp] = up ? x5[((long)(Ls - 1) * V + lex) * 12 + cp] : x5[lex * 12 + cp];
    }
}

// e5 = P (y, 0, ..., 0): the first block column of the paper's projector
// matrix, (P_- y at s = 0, P_+ y at s = Ls-1, zero elsewhere); canonical.
__global__ void embed4d_kernel(double2* e5, const double2* y, long V, int Ls) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)Ls * V) return;
    const int s = (int)(idx / V);
    const long lex = idx % V;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        const bool up = cp < 6;
        const bool keep = (s == 0 && !up) || (s == Ls - 1 && up);
        e5[idx * 12 + cp] = keep ? y[lex * 12 + cp] : make_double2(0.0, 0.0);
    }
}

// ---------------------------------------------------------------------
// elementwise / CG kernels on flat complex arrays of n elements
// ---------------------------------------------------------------------
template <class SD, class SS>
__global__ void convert_kernel(void* dst, const void* src, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<SS>::R re, im;
        cload<SS>(src, i, re, im);
        cstore<SD>(dst, i, (typename Traits<SD>::R)re, (typename Traits<SD>::R)im);
    }
}

// The same copy between layouts with different component grouping (FP64
// single components, FP32 pairs, BF16 quads): thread t handles rows 4g..4g+3
// of site t % Vhp, g = t / Vhp.
template <class SD, class SS>
__global__ void convert_remap_kernel(void* dst, const void* src, long nquads, long Vhp) {
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        typename Traits<SS>::R a[8];
        typename Traits<SD>::R c[8];
        load4<SS>(src, g, site, Vhp, a);
#pragma unroll
        for (int k = 0; k < 8; ++k) c[k] = (typename Traits<SD>::R)a[k];
        store4<SD>(dst, g, site, Vhp, c);
    }
}

// y = a x + b y between layouts with different grouping (no reduction)
template <class SY, class SX>
__global__ void axpby_remap_kernel(void* y, const void* x, long nquads, long Vhp, const double* sa, double ha,
                                   const double* sb, double hb) {
    const double a = sa ? *sa : ha;
    const double bb = sb ? *sb : hb;
    using RY = typename Traits<SY>::R;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        typename Traits<SX>::R xv[8];
        RY yv[8];
        load4<SX>(x, g, site, Vhp, xv);
        load4<SY>(y, g, site, Vhp, yv);
#pragma unroll
        for (int k = 0; k < 8; ++k) yv[k] = RY(a) * RY(xv[k]) + RY(bb) * yv[k];
        store4<SY>(y, g, site, Vhp, yv);
    }
}

// CG updates whose operands differ in layout (FP32 x, r with BF16 p, w):
// same arithmetic as cg_xr_kernel / cg_p_kernel, each operand read in its own
// layout with whole-group accesses, four components of one site per thread.
template <class SX, class SP>
__global__ void cg_xr_remap_kernel(void* x, void* r, const void* p, const void* w, long nquads, long Vhp,
                                   const double* alpha, double* partial) {
    __shared__ double red[BLAS_THREADS / 64];
    using RX = typename Traits<SX>::R;
    const RX a = RX(*alpha);
    double acc = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        typename Traits<SP>::R pv[8], wv[8];
        RX xv[8], rv[8];
        load4<SP>(p, g, site, Vhp, pv);
        load4<SP>(w, g, site, Vhp, wv);
        load4<SX>(x, g, site, Vhp, xv);
        load4<SX>(r, g, site, Vhp, rv);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xv[k] += a * RX(pv[k]);
            rv[k] -= a * RX(wv[k]);
            acc += double(rv[k]) * double(rv[k]);
        }
        store4<SX>(x, g, site, Vhp, xv);
        store4<SX>(r, g, site, Vhp, rv);
    }
    double tt = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = tt;
}

template <class SR, class SP>
__global__ void cg_p_remap_kernel(void* p, const void* r, long nquads, long Vhp, const double* beta) {
    using RP = typename Traits<SP>::R;
    const RP b = RP(*beta);
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        typename Traits<SR>::R rv[8];
        RP pv[8];
        load4<SR>(r, g, site, Vhp, rv);
        load4<SP>(p, g, site, Vhp, pv);
#pragma unroll
        for (int k = 0; k < 8; ++k) pv[k] = RP(rv[k]) + b * pv[k];
        store4<SP>(p, g, site, Vhp, pv);
    }
}

// p_dst = r + beta p_src
template <class SR, class SP>
__global__ void cg_p2_kernel(void* pd, const void* ps, const void* r, long n, const double* beta) {
    using RP = typename Traits<SP>::R;
    const RP b = RP(*beta);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<SR>::R rr, ri;
        RP pr, pi;
        cload<SR>(r, i, rr, ri);
        cload<SP>(ps, i, pr, pi);
        cstore<SP>(pd, i, RP(rr) + b * pr, RP(ri) + b * pi);
    }
}
template <class SR, class SP>
__global__ void cg_p2_remap_kernel(void* pd, const void* ps, const void* r, long nquads, long Vhp,
                                   const double* beta) {
    using RP = typename Traits<SP>::R;
    const RP b = RP(*beta);
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        typename Traits<SR>::R rv[8];
        RP pv[8];
        load4<SR>(r, g, site, Vhp, rv);
        load4<SP>(ps, g, site, Vhp, pv);
#pragma unroll
        for (int k = 0; k < 8; ++k) pv[k] = RP(rv[k]) + b * pv[k];
        store4<SP>(pd, g, site, Vhp, pv);
    }
}

// x += sum_i alpha_i p_i in order, x rounded to its storage after every term
// (x is FP32 or FP64, whose compute type is the storage type)
template <class SX, class SP>
__global__ void cg_accx_kernel(void* x, const void* ring, const double* alpha, int cnt, long n) {
    using RX = typename Traits<SX>::R;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        RX xr, xi;
        cload<SX>(x, i, xr, xi);
        for (int q = 0; q < cnt; ++q) {
            typename Traits<SP>::R pr, pi;
            cload<SP>(static_cast<const char*>(ring) + (size_t)q * n * cbytes<SP>(), i, pr, pi);
            const RX a = RX(alpha[q]);
            xr = xr + a * RX(pr);   // x is FP32 or FP64: stored in its compute type
            xi = xi + a * RX(pi);
        }
        cstore<SX>(x, i, xr, xi);
    }
}
// FP32 x and FP32 ring: two complex numbers (16 bytes) per lane, the loads of
// every ring term issued before the updates, which then run in the order of
// cg_accx_kernel (x rounded after each term: the same bits).  One step per
// lane (no grid-stride loop).
__global__ __launch_bounds__(256) void cg_accx_f32_kernel(float4* __restrict__ x, const float4* __restrict__ ring,
                                                          const double* __restrict__ alpha, int cnt, long n2) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n2) return;
    constexpr int QMAX = 16;
    float4 p[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
        if (q < cnt) p[q] = ring[(long)q * n2 + i];
    float4 v = x[i];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
        if (q < cnt) {
            const float a = (float)alpha[q];
            v.x = v.x + a * p[q].x;
            v.y = v.y + a * p[q].y;
            v.z = v.z + a * p[q].z;
            v.w = v.w + a * p[q].w;
        }
    }
    x[i] = v;
}

// FP32 p_dst = r + beta p_src, 2 x 16 bytes per lane, all loads first
__global__ __launch_bounds__(256) void cg_p2_f32_kernel(float4* __restrict__ pd, const float4* __restrict__ ps,
                                                        const float4* __restrict__ r, long n2, const double* beta) {
    const long i0 = (long)blockIdx.x * 512 + threadIdx.x;
    const float b = (float)*beta;
    float4 rv[2], pv[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const long i = i0 + k * 256;
        if (i < n2) {
            rv[k] = r[i];
            pv[k] = ps[i];
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const long i = i0 + k * 256;
        if (i < n2)
            pd[i] = make_float4(rv[k].x + b * pv[k].x, rv[k].y + b * pv[k].y, rv[k].z + b * pv[k].z,
                                rv[k].w + b * pv[k].w);
    }
}

template <class SX, class SP>
__global__ void cg_accx_remap_kernel(void* x, const void* ring, const double* alpha, int cnt, long n, long nquads,
                                     long Vhp) {
    using RX = typename Traits<SX>::R;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        RX xv[8];
        load4<SX>(x, g, site, Vhp, xv);
        for (int q = 0; q < cnt; ++q) {
            typename Traits<SP>::R pv[8];
            load4<SP>(static_cast<const char*>(ring) + (size_t)q * n * cbytes<SP>(), g, site, Vhp, pv);
            const RX a = RX(alpha[q]);
#pragma unroll
            for (int k = 0; k < 8; ++k) xv[k] = xv[k] + a * RX(pv[k]);
        }
        store4<SX>(x, g, site, Vhp, xv);
    }
}

// x += alpha p; p = r + beta p (the x update of a CG step deferred to the
// kernel that reads p anyway), operands in different layouts
template <class SX, class SP>
__global__ void cg_px_remap_kernel(void* x, void* p, const void* r, long nquads, long Vhp, const double* alpha,
                                   const double* beta) {
    using RX = typename Traits<SX>::R;
    using RP = typename Traits<SP>::R;
    const RX a = RX(*alpha);
    const RP b = RP(*beta);
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < nquads; t += (long)gridDim.x * blockDim.x) {
        const long g = t / Vhp, site = t - g * Vhp;
        RX xv[8], rv[8];
        RP pv[8];
        load4<SP>(p, g, site, Vhp, pv);
        load4<SX>(x, g, site, Vhp, xv);
        load4<SX>(r, g, site, Vhp, rv);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            xv[k] += a * RX(pv[k]);
            pv[k] = RP(rv[k]) + b * pv[k];
        }
        store4<SX>(x, g, site, Vhp, xv);
        store4<SP>(p, g, site, Vhp, pv);
    }
}

template <class S>
__global__ void norm2_kernel(const void* x, long n, double* partial) {
    __shared__ double red[BLAS_THREADS / 64];
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<S>::R re, im;
        cload<S>(x, i, re, im);
        acc += double(re) * double(re) + double(im) * double(im);
    }
    double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// <x, y> = sum conj(x) y, partial[2*block] = re, partial[2*block+1] = im
template <class S>
__global__ void dot_kernel(const void* x, const void* y, long n, double* partial) {
    __shared__ double red[BLAS_THREADS / 64];
    double ar = 0.0, ai = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<S>::R xr, xi, yr, yi;
        cload<S>(x, i, xr, xi);
        cload<S>(y, i, yr, yi);
        ar += double(xr) * double(yr) + double(xi) * double(yi);
        ai += double(xr) * double(yi) - double(xi) * double(yr);
    }
    double tr = block_sum(ar, red);
    double ti = block_sum(ai, red);
    if (threadIdx.x == 0) { partial[2 * blockIdx.x] = tr; partial[2 * blockIdx.x + 1] = ti; }
}

// y = a*x + b*y with real scalars a = sa[0] (or ha if sa null), b likewise
template <class SY, class SX>
__global__ void axpby_kernel(void* y, const void* x, long n, const double* sa, double ha,
                             const double* sb, double hb, double* partial) {
    __shared__ double red[BLAS_THREADS / 64];
    const double a = sa ? *sa : ha;
    const double b = sb ? *sb : hb;
    using RY = typename Traits<SY>::R;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<SX>::R xr, xi;
        RY yr, yi;
        cload<SX>(x, i, xr, xi);
        cload<SY>(y, i, yr, yi);
        RY nr = RY(a) * RY(xr) + RY(b) * yr;
        RY ni = RY(a) * RY(xi) + RY(b) * yi;
        cstore<SY>(y, i, nr, ni);
        acc += double(nr) * double(nr) + double(ni) * double(ni);
    }
    if (partial) {
        double t = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = t;
    }
}

// y += (ar + i ai) x  (complex scalar from the host), one storage type
template <class S>
__global__ void caxpy_kernel(void* y, const void* x, long n, double ar, double ai) {
    using R = typename Traits<S>::R;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        R xr, xi, yr, yi;
        cload<S>(x, i, xr, xi);
        cload<S>(y, i, yr, yi);
        cstore<S>(y, i, yr + R(ar) * xr - R(ai) * xi, yi + R(ar) * xi + R(ai) * xr);
    }
}

// Deterministic pseudo-random fill in [-1, 1) (SplitMix64 of seed and index)
// on the valid sites of each row; padding stays zero.
__global__ void random_fill_kernel(double2* v, long rows, long Vh, long Vhp, unsigned long long seed) {
    const long n = rows * Vh;
    for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const long row = k / Vh, site = k % Vh;
        double out[2];
        for (int h = 0; h < 2; ++h) {
            unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(2 * k + h + 1);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            out[h] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        }
        v[fidx(row, site, Vhp, 1)] = make_double2(out[0], out[1]);
    }
}

// CG update: x += alpha p; r -= alpha w; partial |r|^2.  x, r of type SX; p, w of type SP.
template <class SX, class SP>
__global__ void cg_xr_kernel(void* x, void* r, const void* p, const void* w, long n,
                             const double* alpha, double* partial) {
    __shared__ double red[BLAS_THREADS / 64];
    using RX = typename Traits<SX>::R;
    const RX a = RX(*alpha);
    double acc = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<SP>::R pr, pi, wr, wi;
        RX xr, xi, rr, ri;
        cload<SP>(p, i, pr, pi);
        cload<SP>(w, i, wr, wi);
        cload<SX>(x, i, xr, xi);
        cload<SX>(r, i, rr, ri);
        xr += a * RX(pr); xi += a * RX(pi);
        rr -= a * RX(wr); ri -= a * RX(wi);
        cstore<SX>(x, i, xr, xi);
        cstore<SX>(r, i, rr, ri);
        acc += double(rr) * double(rr) + double(ri) * double(ri);
    }
    double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// p = r + beta p
template <class SR, class SP>
__global__ void cg_p_kernel(void* p, const void* r, long n, const double* beta) {
    using RP = typename Traits<SP>::R;
    const RP b = RP(*beta);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        typename Traits<SR>::R rr, ri;
        RP pr, pi;
        cload<SR>(r, i, rr, ri);
        cload<SP>(p, i, pr, pi);
        cstore<SP>(p, i, RP(rr) + b * pr, RP(ri) + b * pi);
    }
}

// x += alpha p; p = r + beta p, operands in the same layout
template <class SX, class SP>
__global__ void cg_px_kernel(void* x, void* p, const void* r, long n, const double* alpha, const double* beta) {
    using RX = typename Traits<SX>::R;
    using RP = typename Traits<SP>::R;
    const RX a = RX(*alpha);
    const RP b = RP(*beta);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        RX xr, xi, rr, ri;
        RP pr, pi;
        cload<SP>(p, i, pr, pi);
        cload<SX>(x, i, xr, xi);
        cload<SX>(r, i, rr, ri);
        cstore<SX>(x, i, xr + a * RX(pr), xi + a * RX(pi));
        cstore<SP>(p, i, RP(rr) + b * pr, RP(ri) + b * pi);
    }
}

// Sum nparts partials in a fixed order; store according to mode:
//  mode 0: out[0] = sum
//  mode 1 (alpha): s[QQ] = sum; s[ALPHA] = s[RR] / sum (0 if sum <= 0)
//  mode 2 (beta):  s[RRNEW] = sum; s[BETA] = sum / s[RR]; s[RROLD] = s[RR]; s[RR] = sum
//  mode 3 (beta after replacing r): s[RRNEW] = s[RR] = sum; s[BETA] = sum / s[RROLD]
// In modes 1-3 a non-finite sum sets s[NANFLAG] = 1.
// alpha_copy (mode 1, or nullptr): also receives the new alpha.
// One block of FIN_THREADS sums the partials in a fixed order (four
// interleaved accumulators per thread, so that four loads per thread are in
// flight, then wave shuffles and one wave over the per-wave sums): the same
// bits on every run, no atomics.  With one accumulator per thread and 256
// threads the loop issued its loads one after another (32 us for 20 736
// partials on MI355X).
constexpr int FIN_THREADS = 1024;
__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(const double* partial, int nparts, int stride,
                                                               double* out, int mode, double* alpha_copy) {
    __shared__ double red[FIN_THREADS / 64];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * FIN_THREADS < nparts; i += 4 * FIN_THREADS) {
        a0 += partial[(long)i * stride];
        a1 += partial[(long)(i + FIN_THREADS) * stride];
        a2 += partial[(long)(i + 2 * FIN_THREADS) * stride];
        a3 += partial[(long)(i + 3 * FIN_THREADS) * stride];
    }
    for (; i < nparts; i += FIN_THREADS) a0 += partial[(long)i * stride];
    double acc = (a0 + a1) + (a2 + a3);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x < 64) {
        double w = threadIdx.x < FIN_THREADS / 64 ? red[threadIdx.x] : 0.0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) w += __shfl_xor(w, off, 64);
        acc = w;
    }
    if (threadIdx.x == 0) {
        const double sum = acc;
        // modes 1-3 address a whole CG scalar block; mode 0 writes out[0] only
        // (a non-finite sum is visible in the value itself)
        if (mode != 0 && !isfinite(sum)) out[CG_NANFLAG] = 1.0;
        if (mode == 0) {
            out[0] = sum;
        } else if (mode == 1) {
            out[CG_QQ] = sum;
            out[CG_ALPHA] = (sum > 0.0 && isfinite(sum)) ? out[CG_RR] / sum : 0.0;
            if (alpha_copy) *alpha_copy = out[CG_ALPHA];
        } else if (mode == 2) {
            out[CG_RRNEW] = sum;
            out[CG_BETA] = out[CG_RR] > 0.0 ? sum / out[CG_RR] : 0.0;
            out[CG_RROLD] = out[CG_RR];
            out[CG_RR] = sum;
        } else if (mode == 3) {
            out[CG_RRNEW] = sum;
            out[CG_BETA] = out[CG_RROLD] > 0.0 ? sum / out[CG_RROLD] : 0.0;
            out[CG_RR] = sum;
        }
    }
}

// ---------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------
static int blocks_for(long work, int threads) {
    long b = (work + threads - 1) / threads;
    return (int)(b < 1 ? 1 : b);
}

int blas_grid(long n) {
    long b = (n + BLAS_THREADS - 1) / BLAS_THREADS;
    if (b > 2048) b = 2048;
    return (int)(b < 1 ? 1 : b);
}

#define DISPATCH1(kind, F, ...)                                              \
    switch (kind) {                                                          \
        case ST_F64: F<double>(__VA_ARGS__); break;                          \
        case ST_F32: F<float>(__VA_ARGS__); break;                           \
        case ST_BF16: F<bf16s>(__VA_ARGS__); break;                          \
        default: throw Error{DWF_EINVAL, "bad storage kind"};                \
    }

template <class S>
static void pack_full_t(void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long ns,
                        hipStream_t st) {
    hipLaunchKernelGGL(pack_full_kernel<S>, dim3(blocks_for(ns * Vh, 256)), dim3(256), 0, st, dst,
                       (const double2*)src, lex, Vh, Vhp, V, ns);
}
void pack_full(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long ns,
               hipStream_t st) {
    DISPATCH1(kind, pack_full_t, dst, src, lex, Vh, Vhp, V, ns, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void unpack_full_t(void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long ns,
                          hipStream_t st) {
    hipLaunchKernelGGL(unpack_full_kernel<S>, dim3(blocks_for(ns * Vh, 256)), dim3(256), 0, st,
                       (double2*)dst, src, lex, Vh, Vhp, V, ns);
}
void unpack_full(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long ns,
                 hipStream_t st) {
    DISPATCH1(kind, unpack_full_t, dst, src, lex, Vh, Vhp, V, ns, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void pack_half_t(void* dst, const void* src, const int* lex, long Vh, long Vhp, long ns, hipStream_t st) {
    hipLaunchKernelGGL(pack_half_kernel<S>, dim3(blocks_for(ns * Vh, 256)), dim3(256), 0, st, dst,
                       (const double2*)src, lex, Vh, Vhp, ns);
}
void pack_half(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long ns, hipStream_t st) {
    DISPATCH1(kind, pack_half_t, dst, src, lex, Vh, Vhp, ns, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void unpack_half_t(void* dst, const void* src, const int* lex, long Vh, long Vhp, long ns, hipStream_t st) {
    hipLaunchKernelGGL(unpack_half_kernel<S>, dim3(blocks_for(ns * Vh, 256)), dim3(256), 0, st,
                       (double2*)dst, src, lex, Vh, Vhp, ns);
}
void unpack_half(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long ns, hipStream_t st) {
    DISPATCH1(kind, unpack_half_t, dst, src, lex, Vh, Vhp, ns, st);
    DWF_HIP(hipGetLastError());
}

void pack_chiral_pair_f64(void* dst, const void* b4, const int* lex, long Vh, long Vhp, hipStream_t st) {
    hipLaunchKernelGGL(pack_chiral_pair_kernel<double>, dim3(blocks_for(Vh, 256)), dim3(256), 0, st, dst,
                       (const double2*)b4, lex, Vh, Vhp);
    DWF_HIP(hipGetLastError());
}

void project_4d(void* x4, const void* x5, long V, int Ls, hipStream_t st) {
    hipLaunchKernelGGL(project4d_kernel, dim3(blocks_for(V, 256)), dim3(256), 0, st, (double2*)x4,
                       (const double2*)x5, V, Ls);
    DWF_HIP(hipGetLastError());
}

void embed_4d(void* e5, const void* y, long V, int Ls, hipStream_t st) {
    hipLaunchKernelGGL(embed4d_kernel, dim3(blocks_for((long)Ls * V, 256)), dim3(256), 0, st, (double2*)e5,
                       (const double2*)y, V, Ls);
    DWF_HIP(hipGetLastError());
}

template <class SD, class SS>
static void convert_t2(void* dst, const void* src, long n, long Vhp, hipStream_t st) {
    if (fpack<SD>() == fpack<SS>())
        hipLaunchKernelGGL((convert_kernel<SD, SS>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, dst, src, n);
    else
        hipLaunchKernelGGL((convert_remap_kernel<SD, SS>), dim3(blas_grid(n / 4)), dim3(BLAS_THREADS), 0, st, dst,
                           src, n / 4, Vhp);
}
template <class SD>
static void convert_t1(int ks, void* dst, const void* src, long n, long Vhp, hipStream_t st) {
    switch (ks) {
        case ST_F64: convert_t2<SD, double>(dst, src, n, Vhp, st); break;
        case ST_F32: convert_t2<SD, float>(dst, src, n, Vhp, st); break;
        case ST_BF16: convert_t2<SD, bf16s>(dst, src, n, Vhp, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void convert(int kd, int ks, void* dst, const void* src, long n, hipStream_t st, long Vhp) {
    if (fpack_of(kd) != fpack_of(ks))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kd, convert_t1, ks, dst, src, n, Vhp, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void norm2_t(const void* x, long n, double* partial, hipStream_t st) {
    hipLaunchKernelGGL(norm2_kernel<S>, dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, n, partial);
}
void norm2_partial(int kind, const void* x, long n, double* partial, hipStream_t st) {
    DISPATCH1(kind, norm2_t, x, n, partial, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void dot_t(const void* x, const void* y, long n, double* partial, hipStream_t st) {
    hipLaunchKernelGGL(dot_kernel<S>, dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, y, n, partial);
}
void dot_partial(int kind, const void* x, const void* y, long n, double* partial, hipStream_t st) {
    DISPATCH1(kind, dot_t, x, y, n, partial, st);
    DWF_HIP(hipGetLastError());
}

template <class SY, class SX>
static void axpby_t2(void* y, const void* x, long n, const double* sa, double ha, const double* sb,
                     double hb, double* partial, hipStream_t st) {
    hipLaunchKernelGGL((axpby_kernel<SY, SX>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, y, x, n, sa, ha,
                       sb, hb, partial);
}
template <class SY, class SX>
static void axpby_remap_t(void* y, const void* x, long n, long Vhp, const double* sa, double ha, const double* sb,
                          double hb, hipStream_t st) {
    hipLaunchKernelGGL((axpby_remap_kernel<SY, SX>), dim3(blas_grid(n / 4)), dim3(BLAS_THREADS), 0, st, y, x, n / 4,
                       Vhp, sa, ha, sb, hb);
}
template <class SY>
static void axpby_t1(int kx, void* y, const void* x, long n, const double* sa, double ha, const double* sb,
                     double hb, double* partial, hipStream_t st) {
    switch (kx) {
        case ST_F64: axpby_t2<SY, double>(y, x, n, sa, ha, sb, hb, partial, st); break;
        case ST_F32: axpby_t2<SY, float>(y, x, n, sa, ha, sb, hb, partial, st); break;
        case ST_BF16: axpby_t2<SY, bf16s>(y, x, n, sa, ha, sb, hb, partial, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void axpby(int ky, int kx, void* y, const void* x, long n, const double* sa, double ha, const double* sb,
           double hb, double* partial, hipStream_t st, long Vhp) {
    if (fpack_of(ky) != fpack_of(kx)) {
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0 && !partial, DWF_EINVAL, "layout change needs the row stride");
        switch (ky * 3 + kx) {
            case ST_F64 * 3 + ST_F32: axpby_remap_t<double, float>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
            case ST_F64 * 3 + ST_BF16: axpby_remap_t<double, bf16s>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
            case ST_F32 * 3 + ST_F64: axpby_remap_t<float, double>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
            case ST_F32 * 3 + ST_BF16: axpby_remap_t<float, bf16s>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
            case ST_BF16 * 3 + ST_F64: axpby_remap_t<bf16s, double>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
            default: axpby_remap_t<bf16s, float>(y, x, n, Vhp, sa, ha, sb, hb, st); break;
        }
        DWF_HIP(hipGetLastError());
        return;
    }
    DISPATCH1(ky, axpby_t1, kx, y, x, n, sa, ha, sb, hb, partial, st);
    DWF_HIP(hipGetLastError());
}

template <class SX, class SP>
static void cg_xr_t2(void* x, void* r, const void* p, const void* w, long n, long Vhp, const double* alpha,
                     double* partial, hipStream_t st) {
    // same block count in both forms: callers reduce blas_grid(n) partials
    if (fpack<SX>() == fpack<SP>())
        hipLaunchKernelGGL((cg_xr_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, r, p, w, n,
                           alpha, partial);
    else
        hipLaunchKernelGGL((cg_xr_remap_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, r, p, w,
                           n / 4, Vhp, alpha, partial);
}
template <class SX>
static void cg_xr_t1(int kp, void* x, void* r, const void* p, const void* w, long n, long Vhp, const double* alpha,
                     double* partial, hipStream_t st) {
    switch (kp) {
        case ST_F64: cg_xr_t2<SX, double>(x, r, p, w, n, Vhp, alpha, partial, st); break;
        case ST_F32: cg_xr_t2<SX, float>(x, r, p, w, n, Vhp, alpha, partial, st); break;
        case ST_BF16: cg_xr_t2<SX, bf16s>(x, r, p, w, n, Vhp, alpha, partial, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void cg_update_xr(int kx, int kp, void* x, void* r, const void* p, const void* w, long n,
                  const double* alpha, double* partial, hipStream_t st, long Vhp) {
    if (fpack_of(kx) != fpack_of(kp))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kx, cg_xr_t1, kp, x, r, p, w, n, Vhp, alpha, partial, st);
    DWF_HIP(hipGetLastError());
}

template <class SR, class SP>
static void cg_p_t2(void* p, const void* r, long n, long Vhp, const double* beta, hipStream_t st) {
    if (fpack<SR>() == fpack<SP>())
        hipLaunchKernelGGL((cg_p_kernel<SR, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, p, r, n, beta);
    else
        hipLaunchKernelGGL((cg_p_remap_kernel<SR, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, p, r, n / 4,
                           Vhp, beta);
}
template <class SR>
static void cg_p_t1(int kp, void* p, const void* r, long n, long Vhp, const double* beta, hipStream_t st) {
    switch (kp) {
        case ST_F64: cg_p_t2<SR, double>(p, r, n, Vhp, beta, st); break;
        case ST_F32: cg_p_t2<SR, float>(p, r, n, Vhp, beta, st); break;
        case ST_BF16: cg_p_t2<SR, bf16s>(p, r, n, Vhp, beta, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void cg_update_p(int kr, int kp, void* p, const void* r, long n, const double* beta, hipStream_t st, long Vhp) {
    if (fpack_of(kr) != fpack_of(kp))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kr, cg_p_t1, kp, p, r, n, Vhp, beta, st);
    DWF_HIP(hipGetLastError());
}

template <class SX, class SP>
static void cg_px_t2(void* x, void* p, const void* r, long n, long Vhp, const double* alpha, const double* beta,
                     hipStream_t st) {
    if (fpack<SX>() == fpack<SP>())
        hipLaunchKernelGGL((cg_px_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, p, r, n, alpha,
                           beta);
    else
        hipLaunchKernelGGL((cg_px_remap_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, p, r,
                           n / 4, Vhp, alpha, beta);
}
template <class SX>
static void cg_px_t1(int kp, void* x, void* p, const void* r, long n, long Vhp, const double* alpha,
                     const double* beta, hipStream_t st) {
    switch (kp) {
        case ST_F64: cg_px_t2<SX, double>(x, p, r, n, Vhp, alpha, beta, st); break;
        case ST_F32: cg_px_t2<SX, float>(x, p, r, n, Vhp, alpha, beta, st); break;
        case ST_BF16: cg_px_t2<SX, bf16s>(x, p, r, n, Vhp, alpha, beta, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void cg_update_px(int kx, int kp, void* x, void* p, const void* r, long n, const double* alpha, const double* beta,
                  hipStream_t st, long Vhp) {
    if (fpack_of(kx) != fpack_of(kp))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kx, cg_px_t1, kp, x, p, r, n, Vhp, alpha, beta, st);
    DWF_HIP(hipGetLastError());
}

template <class SR, class SP>
static void cg_p2_t2(void* pd, const void* ps, const void* r, long n, long Vhp, const double* beta, hipStream_t st) {
    if constexpr (std::is_same<SR, float>::value && std::is_same<SP, float>::value) {
        if (n % 2 == 0) {
            const long n2 = n / 2;
            hipLaunchKernelGGL(cg_p2_f32_kernel, dim3((unsigned)((n2 + 511) / 512)), dim3(256), 0, st,
                               static_cast<float4*>(pd), static_cast<const float4*>(ps), static_cast<const float4*>(r),
                               n2, beta);
            return;
        }
    }
    if (fpack<SR>() == fpack<SP>())
        hipLaunchKernelGGL((cg_p2_kernel<SR, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, pd, ps, r, n, beta);
    else
        hipLaunchKernelGGL((cg_p2_remap_kernel<SR, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, pd, ps, r,
                           n / 4, Vhp, beta);
}
template <class SR>
static void cg_p2_t1(int kp, void* pd, const void* ps, const void* r, long n, long Vhp, const double* beta,
                     hipStream_t st) {
    switch (kp) {
        case ST_F64: cg_p2_t2<SR, double>(pd, ps, r, n, Vhp, beta, st); break;
        case ST_F32: cg_p2_t2<SR, float>(pd, ps, r, n, Vhp, beta, st); break;
        case ST_BF16: cg_p2_t2<SR, bf16s>(pd, ps, r, n, Vhp, beta, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void cg_update_p2(int kr, int kp, void* p_dst, const void* p_src, const void* r, long n, const double* beta,
                  hipStream_t st, long Vhp) {
    if (fpack_of(kr) != fpack_of(kp))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kr, cg_p2_t1, kp, p_dst, p_src, r, n, Vhp, beta, st);
    DWF_HIP(hipGetLastError());
}

template <class SX, class SP>
static void cg_accx_t2(void* x, const void* ring, const double* alpha, int cnt, long n, long Vhp, hipStream_t st) {
    if constexpr (std::is_same<SX, float>::value && std::is_same<SP, float>::value) {
        if (n % 2 == 0 && cnt <= 16) {
            const long n2 = n / 2;
            hipLaunchKernelGGL(cg_accx_f32_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st,
                               static_cast<float4*>(x), static_cast<const float4*>(ring), alpha, cnt, n2);
            return;
        }
    }
    if (fpack<SX>() == fpack<SP>())
        hipLaunchKernelGGL((cg_accx_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, ring, alpha,
                           cnt, n);
    else
        hipLaunchKernelGGL((cg_accx_remap_kernel<SX, SP>), dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, x, ring,
                           alpha, cnt, n, n / 4, Vhp);
}
template <class SX>
static void cg_accx_t1(int kp, void* x, const void* ring, const double* alpha, int cnt, long n, long Vhp,
                       hipStream_t st) {
    switch (kp) {
        case ST_F64: cg_accx_t2<SX, double>(x, ring, alpha, cnt, n, Vhp, st); break;
        case ST_F32: cg_accx_t2<SX, float>(x, ring, alpha, cnt, n, Vhp, st); break;
        case ST_BF16: cg_accx_t2<SX, bf16s>(x, ring, alpha, cnt, n, Vhp, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void cg_accumulate_x(int kx, int kp, void* x, const void* p_ring, const double* alpha, int cnt, long n,
                     hipStream_t st, long Vhp) {
    if (cnt <= 0) return;
    if (fpack_of(kx) != fpack_of(kp))
        DWF_REQUIRE(Vhp > 0 && n % (4 * Vhp) == 0, DWF_EINVAL, "layout change needs the row stride");
    DISPATCH1(kx, cg_accx_t1, kp, x, p_ring, alpha, cnt, n, Vhp, st);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void caxpy_t(void* y, const void* x, long n, double ar, double ai, hipStream_t st) {
    hipLaunchKernelGGL(caxpy_kernel<S>, dim3(blas_grid(n)), dim3(BLAS_THREADS), 0, st, y, x, n, ar, ai);
}
void caxpy(int kind, void* y, const void* x, long n, double ar, double ai, hipStream_t st) {
    DISPATCH1(kind, caxpy_t, y, x, n, ar, ai, st);
    DWF_HIP(hipGetLastError());
}

void random_fill_f64(void* v, long rows, long Vh, long Vhp, unsigned long long seed, hipStream_t st) {
    hipLaunchKernelGGL(random_fill_kernel, dim3(blas_grid(rows * Vh)), dim3(BLAS_THREADS), 0, st, (double2*)v, rows,
                       Vh, Vhp, seed);
    DWF_HIP(hipGetLastError());
}

void finalize(const double* partial, int nparts, int stride, double* out, int mode, hipStream_t st,
              double* alpha_copy) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(FIN_THREADS), 0, st, partial, nparts, stride, out, mode,
                       alpha_copy);
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
