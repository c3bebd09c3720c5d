// Vector kernels of flexible GCR (FP32 storage, FP64 reductions): batched
// inner products against the stored directions, their coefficients, the
// combined update of q and z, and the x / r step.
#include "dwf_internal.h"
#include "fgcr.h"

namespace dwf {

constexpr int FT = 256;

__device__ __forceinline__ void bsum2(double& a, double& b, double (*red)[FT / 64]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0; b = 0;
        for (int k = 0; k < FT / 64; ++k) { a += red[0][k]; b += red[1][k]; }
    }
}

// partial[(i * nb + block) * 2 + {0,1}] = <Q_i, q> over the block's elements, i = blockIdx.y
__global__ __launch_bounds__(FT) void fg_mdot(const float2* Q, long n, const float2* q, double* partial) {
    __shared__ double red[2][FT / 64];
    const float2* Qi = Q + (long)blockIdx.y * n;
    double re = 0, im = 0;
    for (long k = (long)blockIdx.x * FT + threadIdx.x; k < n; k += (long)gridDim.x * FT) {
        const float2 a = Qi[k], b = q[k];
        re += (double)a.x * b.x + (double)a.y * b.y;
        im += (double)a.x * b.y - (double)a.y * b.x;
    }
    bsum2(re, im, red);
    if (threadIdx.x == 0) {
        partial[((long)blockIdx.y * gridDim.x + blockIdx.x) * 2] = re;
        partial[((long)blockIdx.y * gridDim.x + blockIdx.x) * 2 + 1] = im;
    }
}

// coef[i] = <Q_i, q> / |Q_i|^2 (one block per i); qq[i] = |Q_i|^2
__global__ __launch_bounds__(FT) void fg_mcoef(const double* partial, int nb, const double* qq, double2* coef) {
    __shared__ double red[2][FT / 64];
    const int i = blockIdx.x;
    double re = 0, im = 0;
    for (int k = threadIdx.x; k < nb; k += FT) {
        re += partial[((long)i * nb + k) * 2];
        im += partial[((long)i * nb + k) * 2 + 1];
    }
    bsum2(re, im, red);
    if (threadIdx.x == 0) {
        const double d = qq[i];
        coef[i] = d > 0 ? make_double2(re / d, im / d) : make_double2(0.0, 0.0);
    }
}

// q -= sum_i coef_i Q_i ; z -= sum_i coef_i Z_i
__global__ __launch_bounds__(FT) void fg_maxpy(float2* q, float2* z, const float2* Q, const float2* Z, long n, int j,
                                               const double2* coef) {
    for (long k = (long)blockIdx.x * FT + threadIdx.x; k < n; k += (long)gridDim.x * FT) {
        float2 a = q[k], b = z[k];
        for (int i = 0; i < j; ++i) {
            const double2 c = coef[i];
            const float cr = (float)c.x, ci = (float)c.y;
            const float2 qi = Q[(long)i * n + k], zi = Z[(long)i * n + k];
            a.x -= cr * qi.x - ci * qi.y;
            a.y -= cr * qi.y + ci * qi.x;
            b.x -= cr * zi.x - ci * zi.y;
            b.y -= cr * zi.y + ci * zi.x;
        }
        q[k] = a;
        z[k] = b;
    }
}

// partial: |q|^2 and <q, r> (re, im) per block
__global__ __launch_bounds__(FT) void fg_qr(const float2* q, const float2* r, long n, double* partial) {
    __shared__ double red[2][FT / 64];
    __shared__ double red2[2][FT / 64];
    double qq = 0, dummy = 0, re = 0, im = 0;
    for (long k = (long)blockIdx.x * FT + threadIdx.x; k < n; k += (long)gridDim.x * FT) {
        const float2 a = q[k], b = r[k];
        qq += (double)a.x * a.x + (double)a.y * a.y;
        re += (double)a.x * b.x + (double)a.y * b.y;
        im += (double)a.x * b.y - (double)a.y * b.x;
    }
    bsum2(qq, dummy, red);
    bsum2(re, im, red2);
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 3] = qq;
        partial[blockIdx.x * 3 + 1] = re;
        partial[blockIdx.x * 3 + 2] = im;
    }
}

// qq_out = |q|^2, alpha = <q, r> / |q|^2
__global__ __launch_bounds__(FT) void fg_alpha(const double* partial, int nb, double* qq_out, double2* alpha,
                                               double* nanflag) {
    __shared__ double red[2][FT / 64];
    __shared__ double red2[2][FT / 64];
    double qq = 0, dummy = 0, re = 0, im = 0;
    for (int k = threadIdx.x; k < nb; k += FT) {
        qq += partial[k * 3];
        re += partial[k * 3 + 1];
        im += partial[k * 3 + 2];
    }
    bsum2(qq, dummy, red);
    bsum2(re, im, red2);
    if (threadIdx.x == 0) {
        *qq_out = qq;
        const bool ok = qq > 0 && isfinite(qq) && isfinite(re) && isfinite(im);
        *alpha = ok ? make_double2(re / qq, im / qq) : make_double2(0.0, 0.0);
        if (!ok) *nanflag = 1.0;
    }
}

// x += alpha z; r -= alpha q; partial |r|^2
__global__ __launch_bounds__(FT) void fg_update(float2* x, float2* r, const float2* z, const float2* q, long n,
                                                const double2* alpha, double* partial) {
    __shared__ double red[2][FT / 64];
    const float ar = (float)alpha->x, ai = (float)alpha->y;
    double rr = 0, dummy = 0;
    for (long k = (long)blockIdx.x * FT + threadIdx.x; k < n; k += (long)gridDim.x * FT) {
        float2 xv = x[k], rv = r[k];
        const float2 zv = z[k], qv = q[k];
        xv.x += ar * zv.x - ai * zv.y;
        xv.y += ar * zv.y + ai * zv.x;
        rv.x -= ar * qv.x - ai * qv.y;
        rv.y -= ar * qv.y + ai * qv.x;
        x[k] = xv;
        r[k] = rv;
        rr += (double)rv.x * rv.x + (double)rv.y * rv.y;
    }
    bsum2(rr, dummy, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = rr;
}

// ---------------------------------------------------------------------
int fg_blocks(long n) {
    long b = (n + FT - 1) / FT;
    return (int)(b > 1024 ? 1024 : (b < 1 ? 1 : b));
}

void fg_orthogonalize(float2* q, float2* z, const float2* Q, const float2* Z, long n, int j, const double* qq,
                      double* partial, double2* coef, hipStream_t st) {
    if (j <= 0) return;
    const int nb = fg_blocks(n);
    hipLaunchKernelGGL(fg_mdot, dim3(nb, j), dim3(FT), 0, st, Q, n, q, partial);
    hipLaunchKernelGGL(fg_mcoef, dim3(j), dim3(FT), 0, st, partial, nb, qq, coef);
    hipLaunchKernelGGL(fg_maxpy, dim3(nb), dim3(FT), 0, st, q, z, Q, Z, n, j, coef);
    DWF_HIP(hipGetLastError());
}

void fg_step(float2* x, float2* r, const float2* z, const float2* q, long n, double* partial, double* qq_out,
             double2* alpha, double* rr_partial, double* nanflag, hipStream_t st) {
    const int nb = fg_blocks(n);
    hipLaunchKernelGGL(fg_qr, dim3(nb), dim3(FT), 0, st, q, r, n, partial);
    hipLaunchKernelGGL(fg_alpha, dim3(1), dim3(FT), 0, st, partial, nb, qq_out, alpha, nanflag);
    hipLaunchKernelGGL(fg_update, dim3(nb), dim3(FT), 0, st, x, r, z, q, n, alpha, rr_partial);
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
