// Slot-aware vector kernels for batched solves; see slot_blas.h.
#include <type_traits>

#include "slot_blas.h"
#include "blas.h"
#include "dwf_internal.h"
#include "precision.h"

namespace dwf {

constexpr int BT = 256;

__device__ __forceinline__ double bsum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BT / 64; ++i) t += red[i];
    return t;
}

// slot of a block (binary search over block0, wave-uniform)
__device__ __forceinline__ int find_slot(const SlotDesc* __restrict__ slots, int nslots, int b) {
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class S>
__global__ __launch_bounds__(BT) void bnorm2_kernel(const void* x, const SlotDesc* __restrict__ slots, int nslots,
                                                    double* partial, long pstride, const double* scal) {
    __shared__ double red[BT / 64];
    const int v = find_slot(slots, nslots, blockIdx.x);
    const SlotDesc d = slots[v];
    const int b = blockIdx.x - d.block0;
    double acc = 0.0;
    for (long i = (long)b * BT + threadIdx.x; i < d.n; i += (long)d.nb * BT) {
        typename Traits<S>::R re, im;
        cload<S>(x, d.off + i, re, im);
        acc += double(re) * double(re) + double(im) * double(im);
    }
    const double t = bsum(acc, red);
    if (threadIdx.x == 0) partial[(long)v * pstride + b] = t;
}

template <class SR, class SP>
__global__ __launch_bounds__(BT) void bcg_p2_kernel(void* pd, const void* ps, const void* r,
                                                    const SlotDesc* __restrict__ slots, int nslots,
                                                    const double* scal) {
    const int v = find_slot(slots, nslots, blockIdx.x);
    const SlotDesc d = slots[v];
    const int b = blockIdx.x - d.block0;
    const double* sv = scal + (long)v * CG_NSLOTS;
    if (sv[CG_DONE] != 0.0) return;   // block-uniform
    using RP = typename Traits<SP>::R;
    const RP be = RP(sv[CG_BETA]);
    if constexpr (std::is_same<SR, float>::value && std::is_same<SP, float>::value) {
        // FP32: two complex numbers (16 bytes) per lane, two steps with all
        // loads issued first (slot offsets and sizes are even)
        const float4* r4 = reinterpret_cast<const float4*>(static_cast<const float2*>(r) + d.off);
        const float4* s4 = reinterpret_cast<const float4*>(static_cast<const float2*>(ps) + d.off);
        float4* d4 = reinterpret_cast<float4*>(static_cast<float2*>(pd) + d.off);
        const long n2 = d.n / 2, stride = (long)d.nb * BT;
        for (long i = (long)b * BT + threadIdx.x; i < n2; i += 2 * stride) {
            const long i1 = i + stride;
            const bool two = i1 < n2;
            const float4 ra = r4[i], pa = s4[i];
            float4 rb = ra, pb = pa;
            if (two) {
                rb = r4[i1];
                pb = s4[i1];
            }
            d4[i] = make_float4(ra.x + be * pa.x, ra.y + be * pa.y, ra.z + be * pa.z, ra.w + be * pa.w);
            if (two) d4[i1] = make_float4(rb.x + be * pb.x, rb.y + be * pb.y, rb.z + be * pb.z, rb.w + be * pb.w);
        }
    } else if constexpr (fpack<SR>() == fpack<SP>()) {
        for (long i = (long)b * BT + threadIdx.x; i < d.n; i += (long)d.nb * BT) {
            const long k = d.off + i;
            typename Traits<SR>::R rr, ri;
            RP pr, pi;
            cload<SR>(r, k, rr, ri);
            cload<SP>(ps, k, pr, pi);
            cstore<SP>(pd, k, RP(rr) + be * pr, RP(ri) + be * pi);
        }
    } else {
        // operands in different layouts: four components of one site per step
        // (slot offsets are multiples of 4 * Vhp complex, whole groups)
        const char* rb = static_cast<const char*>(r) + d.off * cbytes<SR>();
        const char* sb = static_cast<const char*>(ps) + d.off * cbytes<SP>();
        char* db = static_cast<char*>(pd) + d.off * cbytes<SP>();
        for (long t = (long)b * BT + threadIdx.x; t < d.n / 4; t += (long)d.nb * BT) {
            const long g = t / d.Vhp, site = t - g * d.Vhp;
            typename Traits<SR>::R rv[8];
            RP pv[8];
            load4<SR>(rb, g, site, d.Vhp, rv);
            load4<SP>(sb, g, site, d.Vhp, pv);
#pragma unroll
            for (int q = 0; q < 8; ++q) pv[q] = RP(rv[q]) + be * pv[q];
            store4<SP>(db, g, site, d.Vhp, pv);
        }
    }
}

template <class SX, class SP>
__global__ __launch_bounds__(BT) void bcg_accx_kernel(void* x, const void* ring, long N, const double* alpha,
                                                      int astride, int cnt, const SlotDesc* __restrict__ slots,
                                                      int nslots) {
    const int v = find_slot(slots, nslots, blockIdx.x);
    const SlotDesc d = slots[v];
    const int b = blockIdx.x - d.block0;
    const double* al = alpha + (long)v * astride;
    bool any = false;
    for (int q = 0; q < cnt; ++q) any = any || al[q] != 0.0;
    if (!any) return;   // block-uniform: the slot was done for the whole ring
    using RX = typename Traits<SX>::R;
    using RP = typename Traits<SP>::R;
    const size_t qb = (size_t)N * cbytes<SP>();   // bytes of one ring slot
    if constexpr (std::is_same<SX, float>::value && std::is_same<SP, float>::value) {
        // FP32: 16 bytes per lane, the loads of every ring term first, the
        // updates in ring order (x rounded after each term: the same bits)
        constexpr int QMAX = 16;
        float4* x4 = reinterpret_cast<float4*>(static_cast<float2*>(x) + d.off);
        const float4* p4 = reinterpret_cast<const float4*>(static_cast<const float2*>(ring) + d.off);
        const long n2 = d.n / 2, q2 = N / 2;
        for (long i = (long)b * BT + threadIdx.x; i < n2; i += (long)d.nb * BT) {
            float4 p[QMAX];
#pragma unroll
            for (int q = 0; q < QMAX; ++q)
                if (q < cnt && al[q] != 0.0) p[q] = p4[(long)q * q2 + i];
            float4 v = x4[i];
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
                if (q < cnt && al[q] != 0.0) {
                    const float a = (float)al[q];
                    v.x = v.x + a * p[q].x;
                    v.y = v.y + a * p[q].y;
                    v.z = v.z + a * p[q].z;
                    v.w = v.w + a * p[q].w;
                }
            }
            x4[i] = v;
        }
    } else if constexpr (fpack<SX>() == fpack<SP>()) {
        for (long i = (long)b * BT + threadIdx.x; i < d.n; i += (long)d.nb * BT) {
            const long k = d.off + i;
            RX xr, xi;
            cload<SX>(x, k, xr, xi);
            for (int q = 0; q < cnt; ++q) {
                if (al[q] == 0.0) continue;
                RP pr, pi;
                cload<SP>(static_cast<const char*>(ring) + q * qb, k, pr, pi);
                const RX a = RX(al[q]);
                xr = xr + a * RX(pr);
                xi = xi + a * RX(pi);
            }
            cstore<SX>(x, k, xr, xi);
        }
    } else {
        char* xb = static_cast<char*>(x) + d.off * cbytes<SX>();
        const char* pb = static_cast<const char*>(ring) + d.off * cbytes<SP>();
        for (long t = (long)b * BT + threadIdx.x; t < d.n / 4; t += (long)d.nb * BT) {
            const long g = t / d.Vhp, site = t - g * d.Vhp;
            RX xv[8];
            load4<SX>(xb, g, site, d.Vhp, xv);
            for (int q = 0; q < cnt; ++q) {
                if (al[q] == 0.0) continue;
                RP pv[8];
                load4<SP>(pb + q * qb, g, site, d.Vhp, pv);
                const RX a = RX(al[q]);
#pragma unroll
                for (int k = 0; k < 8; ++k) xv[k] = xv[k] + a * RX(pv[k]);
            }
            store4<SX>(xb, g, site, d.Vhp, xv);
        }
    }
}

__global__ __launch_bounds__(BT) void bfinalize_kernel(const double* partial, long pstride,
                                                       const SlotDesc* __restrict__ slots, double* scal, int mode,
                                                       int from_hop, const double* tol2, double* alpha_out,
                                                       int astride, int check_every) {
    __shared__ double red[BT];
    const int v = blockIdx.x;
    const SlotDesc d = slots[v];
    double* sv = scal + (long)v * CG_NSLOTS;
    if ((mode == 1 || mode == 2) && sv[CG_DONE] != 0.0) {
        if (mode == 1 && alpha_out && threadIdx.x == 0) alpha_out[(long)v * astride] = 0.0;
        return;
    }
    if (mode == 0 && tol2 && tol2[v] == 0.0) return;   // block-uniform: the slot keeps its state
    if (mode == 0 && tol2 && tol2[v] < 0.0) {
        // retired: done without reading its partials (its r may never have been written)
        if (threadIdx.x == 0) {
            sv[CG_RR] = sv[CG_RR0] = sv[CG_STOP] = 0.0;
            sv[CG_ITERS] = 0.0;
            sv[CG_NANFLAG] = 0.0;
            sv[CG_DONE] = 1.0;
        }
        return;
    }
    const int np = from_hop ? d.nhop : d.nb;
    const double* pp = partial + (long)v * pstride;
    // four interleaved accumulators (four loads in flight per thread), fixed order
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * BT < np; i += 4 * BT) {
        a0 += pp[i];
        a1 += pp[i + BT];
        a2 += pp[i + 2 * BT];
        a3 += pp[i + 3 * BT];
    }
    for (; i < np; i += BT) a0 += pp[i];
    red[threadIdx.x] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    for (int h = BT / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double sum = red[0];
    const bool fin = isfinite(sum);
    if (mode == 0) {
        sv[CG_RR] = sum;
        sv[CG_RR0] = sum;
        const double t2 = tol2 ? tol2[v] : 0.0;
        sv[CG_STOP] = t2 * sum;
        sv[CG_ITERS] = 0.0;
        sv[CG_NANFLAG] = fin ? 0.0 : 1.0;
        sv[CG_DONE] = (!fin || sum == 0.0 || t2 < 0.0) ? 1.0 : 0.0;
    } else if (mode == 1) {
        sv[CG_QQ] = sum;
        const double a = (sum > 0.0 && fin) ? sv[CG_RR] / sum : 0.0;
        sv[CG_ALPHA] = a;
        if (alpha_out) alpha_out[(long)v * astride] = a;
        if (!fin) { sv[CG_NANFLAG] = 1.0; sv[CG_DONE] = 1.0; }
    } else if (mode == 2) {
        sv[CG_RRNEW] = sum;
        sv[CG_BETA] = sv[CG_RR] > 0.0 ? sum / sv[CG_RR] : 0.0;
        sv[CG_RROLD] = sv[CG_RR];
        sv[CG_RR] = sum;
        sv[CG_ITERS] += 1.0;
        const long it = (long)sv[CG_ITERS];
        if (!fin) { sv[CG_NANFLAG] = 1.0; sv[CG_DONE] = 1.0; }
        else if (sum <= sv[CG_STOP] && it % check_every == 0) sv[CG_DONE] = 1.0;
    } else {
        sv[CG_TMP] = sum;
        if (!fin) sv[CG_NANFLAG] = 1.0;
    }
}

// ---------------------------------------------------------------------
int slot_blocks(long n) {
    long b = (n + BT * 4 - 1) / (BT * 4);   // about 4 elements per thread
    if (b > 1024) b = 1024;
    return (int)(b < 1 ? 1 : b);
}

#define BDISPATCH1(kind, F, ...)                                             \
    switch (kind) {                                                          \
        case ST_F64: F<double>(__VA_ARGS__); break;                          \
        case ST_F32: F<float>(__VA_ARGS__); break;                           \
        case ST_BF16: F<bf16s>(__VA_ARGS__); break;                          \
        default: throw Error{DWF_EINVAL, "bad storage kind"};                \
    }

template <class S>
static void bnorm2_t(const void* x, const SlotDesc* slots, int nslots, int blocks, double* partial, long pstride,
                     const double* scal, hipStream_t st) {
    hipLaunchKernelGGL(bnorm2_kernel<S>, dim3(blocks), dim3(BT), 0, st, x, slots, nslots, partial, pstride, scal);
}
void bnorm2(int kind, const void* x, const SlotDesc* slots, int nslots, int blocks, double* partial, long pstride,
            const double* scal, hipStream_t st) {
    BDISPATCH1(kind, bnorm2_t, x, slots, nslots, blocks, partial, pstride, scal, st);
    DWF_HIP(hipGetLastError());
}

template <class SR, class SP>
static void bcg_p2_t2(void* pd, const void* ps, const void* r, const SlotDesc* slots, int nslots, int blocks,
                      const double* scal, hipStream_t st) {
    hipLaunchKernelGGL((bcg_p2_kernel<SR, SP>), dim3(blocks), dim3(BT), 0, st, pd, ps, r, slots, nslots, scal);
}
template <class SR>
static void bcg_p2_t1(int kp, void* pd, const void* ps, const void* r, const SlotDesc* slots, int nslots, int blocks,
                      const double* scal, hipStream_t st) {
    switch (kp) {
        case ST_F64: bcg_p2_t2<SR, double>(pd, ps, r, slots, nslots, blocks, scal, st); break;
        case ST_F32: bcg_p2_t2<SR, float>(pd, ps, r, slots, nslots, blocks, scal, st); break;
        case ST_BF16: bcg_p2_t2<SR, bf16s>(pd, ps, r, slots, nslots, blocks, scal, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void bcg_p2(int kx, int kp, void* p_dst, const void* p_src, const void* r, const SlotDesc* slots, int nslots,
            int blocks, const double* scal, hipStream_t st) {
    BDISPATCH1(kx, bcg_p2_t1, kp, p_dst, p_src, r, slots, nslots, blocks, scal, st);
    DWF_HIP(hipGetLastError());
}

template <class SX, class SP>
static void bcg_accx_t2(void* x, const void* ring, long N, const double* alpha, int astride, int cnt,
                        const SlotDesc* slots, int nslots, int blocks, hipStream_t st) {
    hipLaunchKernelGGL((bcg_accx_kernel<SX, SP>), dim3(blocks), dim3(BT), 0, st, x, ring, N, alpha, astride, cnt,
                       slots, nslots);
}
template <class SX>
static void bcg_accx_t1(int kp, void* x, const void* ring, long N, const double* alpha, int astride, int cnt,
                        const SlotDesc* slots, int nslots, int blocks, hipStream_t st) {
    switch (kp) {
        case ST_F64: bcg_accx_t2<SX, double>(x, ring, N, alpha, astride, cnt, slots, nslots, blocks, st); break;
        case ST_F32: bcg_accx_t2<SX, float>(x, ring, N, alpha, astride, cnt, slots, nslots, blocks, st); break;
        case ST_BF16: bcg_accx_t2<SX, bf16s>(x, ring, N, alpha, astride, cnt, slots, nslots, blocks, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}
void bcg_accx(int kx, int kp, void* x, const void* ring, long N, const double* alpha, int astride, int cnt,
              const SlotDesc* slots, int nslots, int blocks, hipStream_t st) {
    DWF_REQUIRE(cnt >= 1 && cnt <= astride && cnt <= 16, DWF_EINVAL, "ring count out of range");
    DWF_REQUIRE(N % 2 == 0, DWF_EINVAL, "batch vectors hold an even number of complex numbers");
    BDISPATCH1(kx, bcg_accx_t1, kp, x, ring, N, alpha, astride, cnt, slots, nslots, blocks, st);
    DWF_HIP(hipGetLastError());
}

void bfinalize(const double* partial, long pstride, const SlotDesc* slots, int nslots, double* scal, int mode,
               int from_hop, const double* tol2, hipStream_t st, double* alpha_out, int astride,
               int check_every) {
    DWF_REQUIRE(check_every >= 1, DWF_EINVAL, "check period must be >= 1");
    hipLaunchKernelGGL(bfinalize_kernel, dim3(nslots), dim3(BT), 0, st, partial, pstride, slots, scal, mode,
                       from_hop, tol2, alpha_out, astride, check_every);
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
