// Kernels of the learned preconditioner: a linear, gauge-equivariant
// parallel-transport convolution (PTC) network (layers, weight gradients,
// loss, Adam).  Fields are FP32 internal half fields, channel-major:
// element (ch, s, comp, site) at ((ch * Ls + s) * 12 + comp) * Vhp + site.
//
// One layer, for the sites x of one parity p:
//   out^a(x, s) = sum_b [ sum_{q in 0, +s, -s} W_q^{ab} in_loc^b(x, s + shift_q)
//                       + sum_{d = 0..7}     W_{1+d}^{ab} L_d(x) in_hop^b(nbr_d(x), s) ]
// where L_d(x) is the hop link of direction d (U_mu(x) forward, U_mu(x-mu)^dag
// backward, boundary phase folded; the same tables as the Wilson hop), W is
// a complex 4x4 spin matrix and in_loc / in_hop live on parity p / 1 - p.
// Path numbering: 0 identity, 1..8 = direction d + 1, 9 = +s, 10 = -s.
#include "dwf_internal.h"
#include "precision.h"
#include "ptc.h"

namespace dwf {

constexpr int PT = 256;
#ifndef DWF_PTC_COMMUTE
#define DWF_PTC_COMMUTE 1
#endif

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

// v (12 complex, spin-major) of the slice whose first row is row0, at internal
// site i (FP32 field layout: pairs of components, or single components)
__device__ __forceinline__ void load12(const float2* f, long row0, long i, long Vhp, float2 (&v)[12]) {
    if constexpr (fpack<float>() == 2) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const float4 a = *reinterpret_cast<const float4*>(f + fidx(row0 + 2 * q, i, Vhp, 2));
            v[2 * q] = make_float2(a.x, a.y);
            v[2 * q + 1] = make_float2(a.z, a.w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = f[fidx(row0 + k, i, Vhp, 1)];
    }
}

__device__ __forceinline__ void store12(float2* f, long row0, long i, long Vhp, const float2 (&v)[12]) {
    if constexpr (fpack<float>() == 2) {
#pragma unroll
        for (int q = 0; q < 6; ++q)
            *reinterpret_cast<float4*>(f + fidx(row0 + 2 * q, i, Vhp, 2)) =
                make_float4(v[2 * q].x, v[2 * q].y, v[2 * q + 1].x, v[2 * q + 1].y);
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) f[fidx(row0 + k, i, Vhp, 1)] = v[k];
    }
}

// t = L v on every spin (L: 9 complex of direction d at site i; FP32 links
// in pairs, one 16-byte load per pair)
__device__ __forceinline__ void transport(const float2* links, int d, long i, long Vhp, const float2 (&v)[12],
                                          float2 (&t)[12]) {
    float2 L[10];
    if constexpr (link_lp(8) == 2) {
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            const float4 a = *reinterpret_cast<const float4*>(links + lidx(d, 2 * g, i, Vhp, 8));
            L[2 * g] = make_float2(a.x, a.y);
            L[2 * g + 1] = make_float2(a.z, a.w);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) L[e] = links[lidx(d, e, i, Vhp, 8)];
    }
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int b = 0; b < 3; ++b) cfma(acc, L[a * 3 + b], v[sp * 3 + b]);
            t[sp * 3 + a] = acc;
        }
}

// acc += W v  (W: 4x4 complex on spin, row-major; v, acc: 12 complex)
__device__ __forceinline__ void spin_apply(const float2* __restrict__ W, const float2 (&v)[12], float2 (&acc)[12]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float2 w = W[i * 4 + j];
#pragma unroll
            for (int c = 0; c < 3; ++c) cfma(acc[i * 3 + c], w, v[j * 3 + c]);
        }
}

// Input of path q for channel b at (site i, slice s): true if nonzero.
__device__ __forceinline__ bool path_input(const PtcLayerParams& P, int q, int b, int s, long i, float2 (&t)[12]) {
    const long Vhp = P.Vhp;
    if (q == 0 || q >= 9) {
        if (!P.in_loc) return false;
        const int ss = q == 0 ? s : (q == 9 ? s + 1 : s - 1);
        if (ss < 0 || ss >= P.Ls) return false;
        load12(P.in_loc, ((long)b * P.Ls + ss) * 12, i, Vhp, t);
        return true;
    }
    if (!P.in_hop) return false;
    const int d = q - 1;
    const long y = P.nbr[(long)d * Vhp + i];
    float2 v[12];
    load12(P.in_hop, ((long)b * P.Ls + s) * 12, y, Vhp, v);
    transport(P.links, d, i, Vhp, v, t);
    return true;
}

// grid (ceil(Vh / PT), Ls, A / AC); AC output channels per thread.  The
// path loop is outside the channel loop: a hop path's link (9 complex) and
// neighbour index are loaded once per thread and serve every input channel,
// and the weights of a path are read with wave-uniform addresses.
// COMMUTE: the spin weights act on spin and the link on colour, so
//   sum_b W^{ab} L v^b = L (sum_b W^{ab} v^b);
// with more input than output channels (the second layer, 8 -> 1) the
// channels are combined first and transported once per output channel.
template <int AC, bool COMMUTE>
__global__ __launch_bounds__(PT) void ptc_layer_kernel(PtcLayerParams P) {
    const long i = (long)blockIdx.x * PT + threadIdx.x;
    if (i >= P.Vh) return;
    const int s = blockIdx.y;
    const int a0 = blockIdx.z * AC;
    const long Vhp = P.Vhp;
    float2 acc[AC][12];
#pragma unroll
    for (int a = 0; a < AC; ++a)
#pragma unroll
        for (int k = 0; k < 12; ++k) acc[a][k] = make_float2(0.f, 0.f);
    // local paths: 0 (same slice), 9 (s + 1), 10 (s - 1)
    if (P.in_loc) {
        for (int qi = 0; qi < 3; ++qi) {
            const int q = qi == 0 ? 0 : 8 + qi;
            const int ss = qi == 0 ? s : (qi == 1 ? s + 1 : s - 1);
            if (ss < 0 || ss >= P.Ls) continue;
            for (int b = 0; b < P.B; ++b) {
                float2 t[12];
                load12(P.in_loc, ((long)b * P.Ls + ss) * 12, i, Vhp, t);
#pragma unroll
                for (int a = 0; a < AC; ++a)
                    spin_apply(P.W + (((long)q * P.A + a0 + a) * P.B + b) * 16, t, acc[a]);
            }
        }
    }
    // link paths 1..8: the link and neighbour of direction d once for all channels
    if (P.in_hop) {
        for (int d = 0; d < 8; ++d) {
            const long y = P.nbr[(long)d * Vhp + i];
            float2 L[10];
            if constexpr (link_lp(8) == 2) {
#pragma unroll
                for (int g = 0; g < 5; ++g) {
                    const float4 v4 = *reinterpret_cast<const float4*>(P.links + lidx(d, 2 * g, i, Vhp, 8));
                    L[2 * g] = make_float2(v4.x, v4.y);
                    L[2 * g + 1] = make_float2(v4.z, v4.w);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 9; ++e) L[e] = P.links[lidx(d, e, i, Vhp, 8)];
            }
            if constexpr (COMMUTE) {
                float2 m[AC][12];
#pragma unroll
                for (int a = 0; a < AC; ++a)
#pragma unroll
                    for (int k = 0; k < 12; ++k) m[a][k] = make_float2(0.f, 0.f);
                for (int b = 0; b < P.B; ++b) {
                    float2 v[12];
                    load12(P.in_hop, ((long)b * P.Ls + s) * 12, y, Vhp, v);
#pragma unroll
                    for (int a = 0; a < AC; ++a)
                        spin_apply(P.W + (((long)(1 + d) * P.A + a0 + a) * P.B + b) * 16, v, m[a]);
                }
#pragma unroll
                for (int a = 0; a < AC; ++a)
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                        for (int c3 = 0; c3 < 3; ++c3)
#pragma unroll
                            for (int bb = 0; bb < 3; ++bb) cfma(acc[a][sp * 3 + c3], L[c3 * 3 + bb], m[a][sp * 3 + bb]);
            } else {
                for (int b = 0; b < P.B; ++b) {
                    float2 v[12], t[12];
                    load12(P.in_hop, ((long)b * P.Ls + s) * 12, y, Vhp, v);
#pragma unroll
                    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            float2 c = make_float2(0.f, 0.f);
#pragma unroll
                            for (int bb = 0; bb < 3; ++bb) cfma(c, L[a * 3 + bb], v[sp * 3 + bb]);
                            t[sp * 3 + a] = c;
                        }
#pragma unroll
                    for (int a = 0; a < AC; ++a)
                        spin_apply(P.W + (((long)(1 + d) * P.A + a0 + a) * P.B + b) * 16, t, acc[a]);
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < AC; ++a) {
        const long row0 = ((long)(a0 + a) * P.Ls + s) * 12;
        if (P.accumulate) {
            float2 o[12];
            load12(P.out, row0, i, P.Vhp, o);
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                acc[a][k].x += o[k].x;
                acc[a][k].y += o[k].y;
            }
        }
        store12(P.out, row0, i, P.Vhp, acc[a]);
    }
}

// Weight gradient rows: row = (path index in `paths`, b, a-group); each block
// sums over its PT (site, slice) pairs
//   G[a][i][j] = sum_c g^a_i conj(t^b_j)   (t = path input of channel b)
// and writes AC * 16 complex partials.  The per-block order is fixed, so the
// result is deterministic.
template <int AC>
__global__ __launch_bounds__(PT) void ptc_wgrad_kernel(PtcLayerParams P, const float2* __restrict__ g,
                                                       const int* __restrict__ rows, float* __restrict__ partial) {
    __shared__ float red[PT / 64][AC * 32];
    const int row = blockIdx.y;
    const int q = rows[3 * row], b = rows[3 * row + 1], a0 = rows[3 * row + 2];
    const long t_id = (long)blockIdx.x * PT + threadIdx.x;
    const long Vh = P.Vh, Vhp = P.Vhp;
    float2 acc[AC][16];
#pragma unroll
    for (int a = 0; a < AC; ++a)
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[a][k] = make_float2(0.f, 0.f);
    if (t_id < Vh * P.Ls) {
        const int s = (int)(t_id / Vh);
        const long i = t_id % Vh;
        float2 t[12];
        if (path_input(P, q, b, s, i, t)) {
#pragma unroll
            for (int a = 0; a < AC; ++a) {
                float2 gv[12];
                load12(g, ((long)(a0 + a) * P.Ls + s) * 12, i, Vhp, gv);
#pragma unroll
                for (int ii = 0; ii < 4; ++ii)
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const float2 pr = cmulc(gv[ii * 3 + c], t[jj * 3 + c]);
                            acc[a][ii * 4 + jj].x += pr.x;
                            acc[a][ii * 4 + jj].y += pr.y;
                        }
            }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < AC; ++a)
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float x = acc[a][k].x, y = acc[a][k].y;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                x += __shfl_xor(x, off, 64);
                y += __shfl_xor(y, off, 64);
            }
            if (lane == 0) {
                red[w][(a * 16 + k) * 2] = x;
                red[w][(a * 16 + k) * 2 + 1] = y;
            }
        }
    __syncthreads();
    if (threadIdx.x < AC * 32) {
        float sum = 0.f;
        for (int ww = 0; ww < PT / 64; ++ww) sum += red[ww][threadIdx.x];
        partial[((long)row * gridDim.x + blockIdx.x) * (AC * 32) + threadIdx.x] = sum;
    }
}

// grad[(q, a0 + a, b)] += sum over blocks (FP64), one block per row
template <int AC>
__global__ __launch_bounds__(PT) void ptc_wgrad_finalize(const float* __restrict__ partial, int nblocks,
                                                         const int* __restrict__ rows, int A, int B,
                                                         float2* __restrict__ grad) {
    const int row = blockIdx.x;
    const int q = rows[3 * row], b = rows[3 * row + 1], a0 = rows[3 * row + 2];
    if (threadIdx.x >= AC * 32) return;
    double sum = 0.0;
    for (int k = 0; k < nblocks; ++k) sum += partial[((long)row * nblocks + k) * (AC * 32) + threadIdx.x];
    const int v = threadIdx.x >> 1, a = v / 16, e = v % 16;
    float* gp = reinterpret_cast<float*>(grad + (((long)q * A + a0 + a) * B + b) * 16 + e) + (threadIdx.x & 1);
    *gp += (float)sum;
}

// partial sums of |y - e|^2 and |e|^2 (FP64) over one half field
__global__ __launch_bounds__(PT) void ptc_loss_partial(const float2* y, const float2* e, long n, double* partial) {
    __shared__ double red[2][PT / 64];
    double d2 = 0.0, e2 = 0.0;
    for (long k = (long)blockIdx.x * PT + threadIdx.x; k < n; k += (long)gridDim.x * PT) {
        const float2 a = y[k], b = e[k];
        const double dx = (double)a.x - b.x, dy = (double)a.y - b.y;
        d2 += dx * dx + dy * dy;
        e2 += (double)b.x * b.x + (double)b.y * b.y;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        d2 += __shfl_xor(d2, off, 64);
        e2 += __shfl_xor(e2, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[0][w] = d2; red[1][w] = e2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int k = 0; k < PT / 64; ++k) { a += red[0][k]; b += red[1][k]; }
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

// out[0] = |y-e|^2 / |e|^2 (loss), out[1] = |e|^2, out[2] = |y-e|^2
__global__ void ptc_loss_finalize(const double* partial, int nparts, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0, b = 0;
    for (int k = 0; k < nparts; ++k) { a += partial[2 * k]; b += partial[2 * k + 1]; }
    out[0] = b > 0 ? a / b : 0.0;
    out[1] = b;
    out[2] = a;
}

// g = 2 (y - e) / |e|^2
__global__ __launch_bounds__(PT) void ptc_loss_grad(const float2* y, const float2* e, long n, const double* stats,
                                                    float2* g) {
    const double e2 = stats[1];
    const float sc = e2 > 0 ? (float)(2.0 / e2) : 0.f;
    for (long k = (long)blockIdx.x * PT + threadIdx.x; k < n; k += (long)gridDim.x * PT) {
        const float2 a = y[k], b = e[k];
        g[k] = make_float2(sc * (a.x - b.x), sc * (a.y - b.y));
    }
}

// residual loss: out[0] = |u|^2 / |r|^2, out[1] = |r|^2, out[2] = |u|^2 (partials as ptc_loss_partial)
__global__ __launch_bounds__(PT) void ptc_norms_partial(const float2* u, const float2* r, long n, double* partial) {
    __shared__ double red[2][PT / 64];
    double u2 = 0.0, r2 = 0.0;
    for (long k = (long)blockIdx.x * PT + threadIdx.x; k < n; k += (long)gridDim.x * PT) {
        const float2 a = u[k], b = r[k];
        u2 += (double)a.x * a.x + (double)a.y * a.y;
        r2 += (double)b.x * b.x + (double)b.y * b.y;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        u2 += __shfl_xor(u2, off, 64);
        r2 += __shfl_xor(r2, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[0][w] = u2; red[1][w] = r2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0;
        for (int k2 = 0; k2 < PT / 64; ++k2) { a += red[0][k2]; b += red[1][k2]; }
        partial[2 * blockIdx.x] = a;
        partial[2 * blockIdx.x + 1] = b;
    }
}

// d = y - e
__global__ __launch_bounds__(PT) void ptc_sub(const float2* y, const float2* e, long n, float2* d) {
    for (long k = (long)blockIdx.x * PT + threadIdx.x; k < n; k += (long)gridDim.x * PT) {
        const float2 a = y[k], b = e[k];
        d[k] = make_float2(a.x - b.x, a.y - b.y);
    }
}

// g = (2 / stats[1]) w
__global__ __launch_bounds__(PT) void ptc_scale_grad(const float2* w, long n, const double* stats, float2* g) {
    const double r2 = stats[1];
    const float sc = r2 > 0 ? (float)(2.0 / r2) : 0.f;
    for (long k = (long)blockIdx.x * PT + threadIdx.x; k < n; k += (long)gridDim.x * PT) {
        const float2 a = w[k];
        g[k] = make_float2(sc * a.x, sc * a.y);
    }
}

// Adam on n real parameters (Kingma and Ba); bc1 = 1 - b1^t, bc2 = 1 - b2^t
__global__ __launch_bounds__(PT) void ptc_adam_kernel(float* w, const float* g, float* m, float* v, int n, float lr,
                                                      float b1, float b2, float eps, float bc1, float bc2) {
    const int k = blockIdx.x * PT + threadIdx.x;
    if (k >= n) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    w[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + eps);
}

// Wt[rev(q)][b][a] = W[q][a][b]^dag (weights of the adjoint layer)
__global__ __launch_bounds__(PT) void ptc_adjoint_weights(const float2* W, float2* Wt, int A, int B) {
    const int k = blockIdx.x * PT + threadIdx.x;
    if (k >= 11 * A * B * 16) return;
    const int e = k % 16, rest = k / 16;
    const int b = rest % B, a = (rest / B) % A, q = rest / (A * B);
    const int i = e / 4, j = e % 4;
    const int rq = q == 0 ? 0 : (q <= 4 ? q + 4 : (q <= 8 ? q - 4 : 19 - q));
    const float2 w = W[(((long)q * A + a) * B + b) * 16 + i * 4 + j];
    Wt[(((long)rq * B + b) * A + a) * 16 + j * 4 + i] = make_float2(w.x, -w.y);
}

// ---------------------------------------------------------------------
void ptc_layer(const PtcLayerParams& P, hipStream_t st) {
    DWF_REQUIRE(P.A >= 1 && P.B >= 1 && P.Ls >= 1 && P.Vh >= 1, DWF_EINVAL, "bad PTC layer shape");
    const int ac = P.A % 4 == 0 ? 4 : (P.A % 2 == 0 ? 2 : 1);
    dim3 grid((unsigned)((P.Vh + PT - 1) / PT), (unsigned)P.Ls, (unsigned)(P.A / ac));
    const bool commute = DWF_PTC_COMMUTE && P.B > ac;   // fewer transports when the channels are combined first
    if (ac == 4) {
        if (commute) hipLaunchKernelGGL((ptc_layer_kernel<4, true>), grid, dim3(PT), 0, st, P);
        else hipLaunchKernelGGL((ptc_layer_kernel<4, false>), grid, dim3(PT), 0, st, P);
    } else if (ac == 2) {
        if (commute) hipLaunchKernelGGL((ptc_layer_kernel<2, true>), grid, dim3(PT), 0, st, P);
        else hipLaunchKernelGGL((ptc_layer_kernel<2, false>), grid, dim3(PT), 0, st, P);
    } else {
        if (commute) hipLaunchKernelGGL((ptc_layer_kernel<1, true>), grid, dim3(PT), 0, st, P);
        else hipLaunchKernelGGL((ptc_layer_kernel<1, false>), grid, dim3(PT), 0, st, P);
    }
    DWF_HIP(hipGetLastError());
}

int ptc_wgrad_blocks(const PtcLayerParams& P) { return (int)((P.Vh * P.Ls + PT - 1) / PT); }

void ptc_wgrad(const PtcLayerParams& P, const float2* g, const int* rows_dev, int nrows, float* partial,
               float2* grad, hipStream_t st) {
    if (nrows == 0) return;
    const int nb = ptc_wgrad_blocks(P);
    const int ac = P.A % 2 == 0 ? 2 : 1;
    if (ac == 2) {
        hipLaunchKernelGGL(ptc_wgrad_kernel<2>, dim3(nb, nrows), dim3(PT), 0, st, P, g, rows_dev, partial);
        hipLaunchKernelGGL(ptc_wgrad_finalize<2>, dim3(nrows), dim3(PT), 0, st, partial, nb, rows_dev, P.A, P.B,
                           grad);
    } else {
        hipLaunchKernelGGL(ptc_wgrad_kernel<1>, dim3(nb, nrows), dim3(PT), 0, st, P, g, rows_dev, partial);
        hipLaunchKernelGGL(ptc_wgrad_finalize<1>, dim3(nrows), dim3(PT), 0, st, partial, nb, rows_dev, P.A, P.B,
                           grad);
    }
    DWF_HIP(hipGetLastError());
}

int ptc_wgrad_ac(int A) { return A % 2 == 0 ? 2 : 1; }

int ptc_loss_blocks(long n) {
    long b = (n + PT - 1) / PT;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

void ptc_loss(const float2* y, const float2* e, long n, double* partial, double* stats, float2* g, hipStream_t st) {
    const int nb = ptc_loss_blocks(n);
    hipLaunchKernelGGL(ptc_loss_partial, dim3(nb), dim3(PT), 0, st, y, e, n, partial);
    hipLaunchKernelGGL(ptc_loss_finalize, dim3(1), dim3(64), 0, st, partial, nb, stats);
    if (g) hipLaunchKernelGGL(ptc_loss_grad, dim3(nb), dim3(PT), 0, st, y, e, n, stats, g);
    DWF_HIP(hipGetLastError());
}

void ptc_sub(const float2* y, const float2* e, long n, float2* d, hipStream_t st) {
    hipLaunchKernelGGL(ptc_sub, dim3(ptc_loss_blocks(n)), dim3(PT), 0, st, y, e, n, d);
    DWF_HIP(hipGetLastError());
}

void ptc_norms(const float2* u, const float2* r, long n, double* partial, double* stats, hipStream_t st) {
    const int nb = ptc_loss_blocks(n);
    hipLaunchKernelGGL(ptc_norms_partial, dim3(nb), dim3(PT), 0, st, u, r, n, partial);
    hipLaunchKernelGGL(ptc_loss_finalize, dim3(1), dim3(64), 0, st, partial, nb, stats);
    DWF_HIP(hipGetLastError());
}

void ptc_scale_grad(const float2* w, long n, const double* stats, float2* g, hipStream_t st) {
    hipLaunchKernelGGL(ptc_scale_grad, dim3(ptc_loss_blocks(n)), dim3(PT), 0, st, w, n, stats, g);
    DWF_HIP(hipGetLastError());
}

void ptc_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, int step,
              hipStream_t st) {
    const float bc1 = 1.f - std::pow(b1, (float)step), bc2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(ptc_adam_kernel, dim3((n + PT - 1) / PT), dim3(PT), 0, st, w, g, m, v, n, lr, b1, b2, eps, bc1,
                       bc2);
    DWF_HIP(hipGetLastError());
}

void ptc_adjoint(const float2* W, float2* Wt, int A, int B, hipStream_t st) {
    const int n = 11 * A * B * 16;
    hipLaunchKernelGGL(ptc_adjoint_weights, dim3((n + PT - 1) / PT), dim3(PT), 0, st, W, Wt, A, B);
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
