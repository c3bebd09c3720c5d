// Kernels of the five-dimensional even-odd split (layout and operator in
// eo5d.h).  One thread per (site, s) of the output half field: the 5D
// blocks have no dense fifth-dimension part, so there is nothing for MFMA
// here; the hop is the spin-projected Wilson hop of the fused kernel's
// conventions, with the K and 1 / M_ss scalings folded into per-slice,
// per-chirality factors.
#include <type_traits>

#include "eo5d.h"
#include "precision.h"

namespace dwf {

namespace {

template <class T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };

// Chiral basis: gamma_mu = [[0, B],[B^dag, 0]] with B = -i sigma_1, -i sigma_2,
// -i sigma_3, 1 for mu = x, y, z, t.  (1 + SG gamma_mu) psi = (w, SG B^dag w),
// w = psi_up + SG B psi_lo.  Components: index spin * 3 + colour, re/im pairs.
template <class T>
__device__ __forceinline__ void project(int mu, T sg, const T (&p)[24], T (&w)[12]) {
    // w[h * 6 + a * 2 + reim] for half-spinor row h = 0, 1
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T u0r = p[(0 * 3 + a) * 2], u0i = p[(0 * 3 + a) * 2 + 1];
        const T u1r = p[(1 * 3 + a) * 2], u1i = p[(1 * 3 + a) * 2 + 1];
        const T l0r = p[(2 * 3 + a) * 2], l0i = p[(2 * 3 + a) * 2 + 1];
        const T l1r = p[(3 * 3 + a) * 2], l1i = p[(3 * 3 + a) * 2 + 1];
        T b0r, b0i, b1r, b1i;   // B psi_lo
        if (mu == 0) {          // -i sigma_1: (-i l1, -i l0)
            b0r = l1i; b0i = -l1r; b1r = l0i; b1i = -l0r;
        } else if (mu == 1) {   // -i sigma_2 = [[0,-1],[1,0]]: (-l1, l0)
            b0r = -l1r; b0i = -l1i; b1r = l0r; b1i = l0i;
        } else if (mu == 2) {   // -i sigma_3: (-i l0, i l1)
            b0r = l0i; b0i = -l0r; b1r = -l1i; b1i = l1r;
        } else {                // 1
            b0r = l0r; b0i = l0i; b1r = l1r; b1i = l1i;
        }
        w[0 * 6 + a * 2] = u0r + sg * b0r;
        w[0 * 6 + a * 2 + 1] = u0i + sg * b0i;
        w[1 * 6 + a * 2] = u1r + sg * b1r;
        w[1 * 6 + a * 2 + 1] = u1i + sg * b1i;
    }
}

// acc_up += v, acc_lo += SG B^dag v for v = U w (two half-spinor rows)
template <class T>
__device__ __forceinline__ void reconstruct(int mu, T sg, const T (&v)[12], T (&acc)[24]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T v0r = v[0 * 6 + a * 2], v0i = v[0 * 6 + a * 2 + 1];
        const T v1r = v[1 * 6 + a * 2], v1i = v[1 * 6 + a * 2 + 1];
        acc[(0 * 3 + a) * 2] += v0r;
        acc[(0 * 3 + a) * 2 + 1] += v0i;
        acc[(1 * 3 + a) * 2] += v1r;
        acc[(1 * 3 + a) * 2 + 1] += v1i;
        T c0r, c0i, c1r, c1i;   // B^dag v
        if (mu == 0) {          // i sigma_1: (i v1, i v0)
            c0r = -v1i; c0i = v1r; c1r = -v0i; c1i = v0r;
        } else if (mu == 1) {   // [[0,1],[-1,0]]: (v1, -v0)
            c0r = v1r; c0i = v1i; c1r = -v0r; c1i = -v0i;
        } else if (mu == 2) {   // i sigma_3: (i v0, -i v1)
            c0r = -v0i; c0i = v0r; c1r = v1i; c1i = -v1r;
        } else {
            c0r = v0r; c0i = v0i; c1r = v1r; c1i = v1i;
        }
        acc[(2 * 3 + a) * 2] += sg * c0r;
        acc[(2 * 3 + a) * 2 + 1] += sg * c0i;
        acc[(3 * 3 + a) * 2] += sg * c1r;
        acc[(3 * 3 + a) * 2 + 1] += sg * c1i;
    }
}

}  // namespace

template <class T>
__global__ __launch_bounds__(256) void eo5_kernel(Eo5Params P) {
    using V2 = typename C2<T>::type;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long Vh = P.Vh;
    if (t >= (long)P.Ls * Vh) return;
    const int s = (int)(t / Vh);
    const long i = t - (long)s * Vh;
    const int q = (P.par + s) & 1;   // 4D parity of the output site
    const double* KD = P.coef + EO5_KD;
    const double* MINV = P.coef + EO5_MINV;
    const double* MM = P.coef + EO5_M;
    const V2* in = static_cast<const V2*>(P.in);

    // scalings of the hop's input (slice s) and of its result, per chirality
    T cin[2], cout[2];
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
        const T mi = P.pre ? T(MINV[chi * 16 + s]) : T(1);
        cin[chi] = P.dagger ? mi : T(KD[chi * 16 + s]) * mi;
        cout[chi] = P.dagger ? T(KD[chi * 16 + s]) : T(1);
    }

    T acc[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] = 0;
    const V2* lk = static_cast<const V2*>(P.links) + (long)q * P.lpar;
    constexpr int CB = (int)sizeof(V2);
    for (int d = 0; d < 8; ++d) {
        const int mu = d & 3;
        // forward hop (x + mu) carries (1 - gamma), backward (1 + gamma);
        // the adjoint (gamma_5 H gamma_5) flips both
        T sg = d < 4 ? T(-1) : T(1);
        if (P.dagger) sg = -sg;
        const long j = P.nbr[((long)q * 8 + d) * P.Vhp + i];
        const V2* src = in + (long)s * 12 * Vh + j;
        T p[24];
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const V2 v = src[(long)k * Vh];
            const T c = k < 6 ? cin[0] : cin[1];
            p[2 * k] = c * v.x;
            p[2 * k + 1] = c * v.y;
        }
        T w[12];
        project<T>(mu, sg, p, w);
        T u[18];
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            const V2 v = lk[lidx(d, e, i, P.Vhp, CB)];
            u[2 * e] = v.x;
            u[2 * e + 1] = v.y;
        }
        T v[12];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T re = 0, im = 0;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const T ur = u[(a * 3 + b) * 2], ui = u[(a * 3 + b) * 2 + 1];
                    const T xr = w[h * 6 + b * 2], xi = w[h * 6 + b * 2 + 1];
                    re += ur * xr - ui * xi;
                    im += ur * xi + ui * xr;
                }
                v[h * 6 + a * 2] = re;
                v[h * 6 + a * 2 + 1] = im;
            }
        reconstruct<T>(mu, sg, v, acc);
    }
    // -1/2 H (times K on the output side for the adjoint)
#pragma unroll
    for (int k = 0; k < 24; ++k) acc[k] *= T(-0.5) * (k < 12 ? cout[0] : cout[1]);

    // shift in s at the same site: (M - diag M) per chirality, rows s and
    // columns s -/+ 1 (transposed for the adjoint)
    const int Ls = P.Ls;
    const int qm = (s + Ls - 1) % Ls, qp = (s + 1) % Ls;
    int qs[2], nq = 0;   // distinct neighbouring slices (one for Ls = 2, none for Ls = 1)
    if (qm != s) qs[nq++] = qm;
    if (qp != s && qp != qm) qs[nq++] = qp;
    for (int n = 0; n < nq; ++n) {
        const int sq = qs[n];
        T c[2];
#pragma unroll
        for (int chi = 0; chi < 2; ++chi) {
            const double m = P.dagger ? MM[(chi * 16 + sq) * 16 + s] : MM[(chi * 16 + s) * 16 + sq];
            c[chi] = T(m) * (P.pre ? T(MINV[chi * 16 + sq]) : T(1));
        }
        const V2* src = in + (long)sq * 12 * Vh + i;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const V2 v = src[(long)k * Vh];
            const T cc = k < 6 ? c[0] : c[1];
            acc[2 * k] += cc * v.x;
            acc[2 * k + 1] += cc * v.y;
        }
    }
    const T mo[2] = {T(MINV[0 * 16 + s]), T(MINV[1 * 16 + s])};
    const T sgn = T(P.sgn), a = T(P.a);
    V2* out = static_cast<V2*>(P.out) + (long)s * 12 * Vh + i;
    const V2* loc = P.loc ? static_cast<const V2*>(P.loc) + (long)s * 12 * Vh + i : nullptr;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const T hs = P.post_hop ? (k < 6 ? mo[0] : mo[1]) : T(1);
        T re = sgn * hs * acc[2 * k], im = sgn * hs * acc[2 * k + 1];
        if (loc) {
            const V2 l = loc[(long)k * Vh];
            const T ls = a * (P.post_loc ? (k < 6 ? mo[0] : mo[1]) : T(1));
            re += ls * l.x;
            im += ls * l.y;
        }
        V2 o;
        o.x = re;
        o.y = im;
        out[(long)k * Vh] = o;
    }
}

// element t of a half field of 5D parity par <-> its entry in the canonical 5D field
__device__ __forceinline__ long eo5_full_index(long t, const int* lex, long Vh, long V, int par) {
    const long sk = t / Vh;
    const long i = t - sk * Vh;
    const int s = (int)(sk / 12), k = (int)(sk - (long)s * 12);
    const int q = (par + s) & 1;
    return ((long)s * V + lex[(long)q * Vh + i]) * 12 + k;
}

__global__ __launch_bounds__(256) void eo5_pack_kernel(double2* half, const double2* full, const int* lex,
                                                       long Vh, long V, int Ls, int par) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < (long)Ls * Vh * 12) half[t] = full[eo5_full_index(t, lex, Vh, V, par)];
}

__global__ __launch_bounds__(256) void eo5_unpack_kernel(double2* full, const double2* half, const int* lex,
                                                         long Vh, long V, int Ls, int par) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < (long)Ls * Vh * 12) full[eo5_full_index(t, lex, Vh, V, par)] = half[t];
}

__global__ __launch_bounds__(256) void eo5_f64_to_f32_kernel(float2* dst, const double2* src, long n) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) dst[t] = make_float2((float)src[t].x, (float)src[t].y);
}

__global__ __launch_bounds__(256) void eo5_f32_to_f64_kernel(double2* dst, const float2* src, long n) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) dst[t] = make_double2((double)src[t].x, (double)src[t].y);
}

__global__ __launch_bounds__(256) void eo5_diag_kernel(double2* out, const double2* in, const double* coef, long Vh,
                                                       int Ls) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)Ls * Vh * 12) return;
    const long sk = t / Vh;
    const int s = (int)(sk / 12), k = (int)(sk - (long)s * 12);
    const int chi = k < 6 ? 0 : 1;
    const double m = coef[EO5_M + (chi * 16 + s) * 16 + s];
    out[t] = make_double2(m * in[t].x, m * in[t].y);
}

static unsigned grid_of(long work) { return (unsigned)((work + 255) / 256); }

void launch_eo5(int kind, const Eo5Params& P, hipStream_t st) {
    DWF_REQUIRE(P.Ls >= 1 && P.Ls <= LS_MAX, DWF_EDIMS, "Ls out of range for the 5D even-odd split");
    const long work = (long)P.Ls * P.Vh;
    if (work == 0) return;
    if (kind == ST_F64) hipLaunchKernelGGL(eo5_kernel<double>, dim3(grid_of(work)), dim3(256), 0, st, P);
    else if (kind == ST_F32) hipLaunchKernelGGL(eo5_kernel<float>, dim3(grid_of(work)), dim3(256), 0, st, P);
    else throw Error{DWF_EINVAL, "the 5D even-odd split runs in FP64 or FP32"};
    DWF_HIP(hipGetLastError());
}

void eo5_pack(void* half, const void* full5, const int* lex_of_site, long Vh, long V, int Ls, int par,
              hipStream_t st) {
    const long n = (long)Ls * Vh * 12;
    if (n == 0) return;
    hipLaunchKernelGGL(eo5_pack_kernel, dim3(grid_of(n)), dim3(256), 0, st, static_cast<double2*>(half),
                       static_cast<const double2*>(full5), lex_of_site, Vh, V, Ls, par);
    DWF_HIP(hipGetLastError());
}

void eo5_unpack(void* full5, const void* half, const int* lex_of_site, long Vh, long V, int Ls, int par,
                hipStream_t st) {
    const long n = (long)Ls * Vh * 12;
    if (n == 0) return;
    hipLaunchKernelGGL(eo5_unpack_kernel, dim3(grid_of(n)), dim3(256), 0, st, static_cast<double2*>(full5),
                       static_cast<const double2*>(half), lex_of_site, Vh, V, Ls, par);
    DWF_HIP(hipGetLastError());
}

void eo5_convert(int kd, int ks, void* dst, const void* src, long n, hipStream_t st) {
    if (n == 0) return;
    if (kd == ks) {
        DWF_HIP(hipMemcpyAsync(dst, src, (size_t)n * (kd == ST_F64 ? 16 : 8), hipMemcpyDeviceToDevice, st));
        return;
    }
    if (kd == ST_F32 && ks == ST_F64)
        hipLaunchKernelGGL(eo5_f64_to_f32_kernel, dim3(grid_of(n)), dim3(256), 0, st, static_cast<float2*>(dst),
                           static_cast<const double2*>(src), n);
    else if (kd == ST_F64 && ks == ST_F32)
        hipLaunchKernelGGL(eo5_f32_to_f64_kernel, dim3(grid_of(n)), dim3(256), 0, st, static_cast<double2*>(dst),
                           static_cast<const float2*>(src), n);
    else
        throw Error{DWF_EINVAL, "5D even-odd fields are FP64 or FP32"};
    DWF_HIP(hipGetLastError());
}

void eo5_diag(void* out, const void* in, const double* coef, long Vh, int Ls, hipStream_t st) {
    const long n = (long)Ls * Vh * 12;
    if (n == 0) return;
    hipLaunchKernelGGL(eo5_diag_kernel, dim3(grid_of(n)), dim3(256), 0, st, static_cast<double2*>(out),
                       static_cast<const double2*>(in), coef, Vh, Ls);
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
