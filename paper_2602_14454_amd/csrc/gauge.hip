// Quenched gauge configurations for the plaquette action, the ensembles of
// the paper's study (Sec. 3.1: beta = 6.0 and 5.7 on 16^4 and 32^4):
//   S = beta * sum_P (1 - Re tr U_P / 3),
//   U_P(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
// A link U_mu(x) sees the staple sum
//   A = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//                    + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
// and the action -beta/3 Re tr(U A).  One launch updates the links of one
// direction on the sites of one parity (their staples do not contain each
// other), one thread per link, FP64, in the canonical layout.
//
// Heatbath (Cabibbo-Marinari): U <- R U with R in the SU(2) subgroups on
// rows (0,1), (0,2), (1,2) in turn, drawn from exp(beta/3 Re tr(R W)),
// W = U A.  The 2x2 block r of W enters through Re tr(X r) = k Re tr(X V^dag)
// (X, V in SU(2), k >= 0), so R = Y V with y0 of Y from
// sqrt(1 - y0^2) exp(2 beta k/3 y0): y0 = 1 - delta, delta Gamma(3/2) from
// two logarithms and a cosine, accepted with probability sqrt(1 - delta/2)
// (Kennedy-Pendleton); the rest of Y uniform on the sphere of radius
// sqrt(1 - y0^2).  Over-relaxation: R = V^2 (Re tr(R r) unchanged).
// Random numbers: SplitMix64 of counters, uniform in (0, 1]:
//   key = mix(seed K1 + sweep K2), u(c) = mix(key + (c + 1) golden),
//   c = ((lex * 4 + mu) * 3 + subgroup) * 4096 + draw;
// attempt t uses draws 4t .. 4t+3, the direction draws 4000 and 4001; a link
// without acceptance in 1000 attempts keeps that subgroup unchanged.
#include "dwf_internal.h"
#include "blas.h"
#include "gauge.h"

namespace dwf {

namespace {

constexpr int GT = 256;
// the update kernels: one thread per link of one direction and parity (V/2
// threads, 128 blocks of 256 on 16^4, half the 256 CUs); 64-thread blocks put
// work on every CU
constexpr int GU = 64;
constexpr unsigned long long GOLD = 0x9E3779B97F4A7C15ull;
constexpr unsigned long long GK1 = 0x2545F4914F6CDD1Dull;
constexpr unsigned long long GK2 = 0x632BE59BD9B4E019ull;

__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

__device__ inline double uniform01(unsigned long long key, unsigned long long c) {
    const unsigned long long z = mix64(key + (c + 1ull) * GOLD);
    return ((double)(z >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

struct M3 {
    double2 e[9];
};

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

__device__ inline M3 load_link(const double2* U, long lex, int mu) {
    M3 m;
    const double2* p = U + (lex * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) m.e[k] = p[k];
    return m;
}

__device__ inline M3 dag(const M3& a) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.e[i * 3 + j] = cconj(a.e[j * 3 + i]);
    return r;
}

__device__ inline M3 mul(const M3& a, const M3& b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double2 s = cmul(a.e[i * 3], b.e[j]);
            s = cadd(s, cmul(a.e[i * 3 + 1], b.e[3 + j]));
            s = cadd(s, cmul(a.e[i * 3 + 2], b.e[6 + j]));
            r.e[i * 3 + j] = s;
        }
    return r;
}

struct Geo {
    int L[4];
    __device__ long lex(const int c[4]) const { return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3])); }
    __device__ void coords(long x, int c[4]) const {
        for (int mu = 0; mu < 4; ++mu) {
            c[mu] = (int)(x % L[mu]);
            x /= L[mu];
        }
    }
    __device__ long shift(const int c[4], int mu, int step) const {
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] = (d[mu] + step + L[mu]) % L[mu];
        return lex(d);
    }
};

// lexicographic index of site i of parity p (Lx even: sites 2i and 2i+1 share y, z, t)
__device__ inline long site_of(const Geo& g, long i, int p) {
    const long l0 = 2 * i;
    int c[4];
    g.coords(l0, c);
    return l0 + ((p + c[1] + c[2] + c[3]) & 1);
}

// SU(2) element q0 + i (q1 s1 + q2 s2 + q3 s3) as a 2x2 complex matrix
__device__ inline void su2(const double q[4], double2 X[4]) {
    X[0] = make_double2(q[0], q[3]);
    X[1] = make_double2(q[2], q[1]);
    X[2] = make_double2(-q[2], q[1]);
    X[3] = make_double2(q[0], -q[3]);
}

__device__ inline void mul2(const double2 a[4], const double2 b[4], double2 r[4]) {
    r[0] = cadd(cmul(a[0], b[0]), cmul(a[1], b[2]));
    r[1] = cadd(cmul(a[0], b[1]), cmul(a[1], b[3]));
    r[2] = cadd(cmul(a[2], b[0]), cmul(a[3], b[2]));
    r[3] = cadd(cmul(a[2], b[1]), cmul(a[3], b[3]));
}

// rows i, j of M <- R (rows i, j)
__device__ inline void apply_rows(M3& m, int i, int j, const double2 R[4]) {
#pragma unroll
    for (int col = 0; col < 3; ++col) {
        const double2 a = m.e[i * 3 + col], b = m.e[j * 3 + col];
        m.e[i * 3 + col] = cadd(cmul(R[0], a), cmul(R[1], b));
        m.e[j * 3 + col] = cadd(cmul(R[2], a), cmul(R[3], b));
    }
}

__global__ __launch_bounds__(GU) void gauge_update_kernel(double2* __restrict__ U, Geo g, int mu, int parity,
                                                          double beta, unsigned long long key, int heatbath,
                                                          long Vh) {
    const long i = (long)blockIdx.x * GU + threadIdx.x;
    if (i >= Vh) return;
    const long x = site_of(g, i, parity);
    int c[4];
    g.coords(x, c);
    M3 A;
#pragma unroll
    for (int k = 0; k < 9; ++k) A.e[k] = make_double2(0.0, 0.0);
    const long xpmu = g.shift(c, mu, +1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        const long xpnu = g.shift(c, nu, +1), xmnu = g.shift(c, nu, -1);
        int cm[4] = {c[0], c[1], c[2], c[3]};
        cm[nu] = (cm[nu] - 1 + g.L[nu]) % g.L[nu];
        const long xpmu_mnu = g.shift(cm, mu, +1);
        const M3 up = mul(mul(load_link(U, xpmu, nu), dag(load_link(U, xpnu, mu))), dag(load_link(U, x, nu)));
        const M3 dn = mul(mul(dag(load_link(U, xpmu_mnu, nu)), dag(load_link(U, xmnu, mu))), load_link(U, xmnu, nu));
#pragma unroll
        for (int k = 0; k < 9; ++k) A.e[k] = cadd(A.e[k], up.e[k]);
#pragma unroll
        for (int k = 0; k < 9; ++k) A.e[k] = cadd(A.e[k], dn.e[k]);
    }
    M3 Ul = load_link(U, x, mu);
    M3 W = mul(Ul, A);
    const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sg = 0; sg < 3; ++sg) {
        const int a = sub[sg][0], b = sub[sg][1];
        const double2 r00 = W.e[a * 3 + a], r01 = W.e[a * 3 + b], r10 = W.e[b * 3 + a], r11 = W.e[b * 3 + b];
        double q[4] = {0.5 * (r00.x + r11.x), -0.5 * (r01.y + r10.y), -0.5 * (r01.x - r10.x),
                       -0.5 * (r00.y - r11.y)};
        const double k = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double kn = k > 0.0 ? k : 1.0;
        for (int t = 0; t < 4; ++t) q[t] /= kn;
        double2 V[4], R[4];
        su2(q, V);
        if (heatbath) {
            const double alpha = k > 0.0 ? 2.0 * beta * k / 3.0 : 1e-300;
            const unsigned long long c0 = ((unsigned long long)(x * 4 + mu) * 3ull + (unsigned long long)sg) * 4096ull;
            bool ok = false;
            double y0 = 1.0;
            for (int t = 0; t < 1000 && !ok; ++t) {
                const unsigned long long cb = c0 + 4ull * (unsigned long long)t;
                const double u1 = uniform01(key, cb), u2 = uniform01(key, cb + 1), u3 = uniform01(key, cb + 2),
                             u4 = uniform01(key, cb + 3);
                const double cs = cos(2.0 * M_PI * u2);
                const double delta = -(log(u1) + cs * cs * log(u3)) / alpha;
                if (u4 * u4 <= 1.0 - 0.5 * delta) {
                    y0 = 1.0 - delta;
                    ok = true;
                }
            }
            if (ok) {
                const double cth = 2.0 * uniform01(key, c0 + 4000) - 1.0;
                const double phi = 2.0 * M_PI * uniform01(key, c0 + 4001);
                const double rad = sqrt(fmax(0.0, 1.0 - y0 * y0));
                const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
                const double y[4] = {y0, rad * sth * cos(phi), rad * sth * sin(phi), rad * cth};
                double2 Y[4];
                su2(y, Y);
                mul2(Y, V, R);
            } else {
                R[0] = make_double2(1.0, 0.0);
                R[1] = make_double2(0.0, 0.0);
                R[2] = make_double2(0.0, 0.0);
                R[3] = make_double2(1.0, 0.0);
            }
        } else {
            mul2(V, V, R);
        }
        apply_rows(Ul, a, b, R);
        apply_rows(W, a, b, R);
    }
    double2* p = U + (x * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = Ul.e[k];
}

// rows 0, 1 normalised and orthogonalised, row 2 = conj(row0 x row1)
__global__ __launch_bounds__(GT) void gauge_reunitarize_kernel(double2* __restrict__ U, long nlinks) {
    const long l = (long)blockIdx.x * GT + threadIdx.x;
    if (l >= nlinks) return;
    double2* m = U + l * 9;
    double2 a[3], b[3];
    double na = 0.0;
    for (int k = 0; k < 3; ++k) {
        a[k] = m[k];
        na += a[k].x * a[k].x + a[k].y * a[k].y;
    }
    na = sqrt(na);
    for (int k = 0; k < 3; ++k) a[k] = make_double2(a[k].x / na, a[k].y / na);
    double2 dot = make_double2(0.0, 0.0);
    for (int k = 0; k < 3; ++k) {
        b[k] = m[3 + k];
        dot = cadd(dot, cmul(cconj(a[k]), b[k]));
    }
    double nb = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double2 t = cmul(dot, a[k]);
        b[k] = make_double2(b[k].x - t.x, b[k].y - t.y);
        nb += b[k].x * b[k].x + b[k].y * b[k].y;
    }
    nb = sqrt(nb);
    for (int k = 0; k < 3; ++k) b[k] = make_double2(b[k].x / nb, b[k].y / nb);
    const double2 c0 = cadd(cmul(a[1], b[2]), make_double2(-cmul(a[2], b[1]).x, -cmul(a[2], b[1]).y));
    const double2 c1 = cadd(cmul(a[2], b[0]), make_double2(-cmul(a[0], b[2]).x, -cmul(a[0], b[2]).y));
    const double2 c2 = cadd(cmul(a[0], b[1]), make_double2(-cmul(a[1], b[0]).x, -cmul(a[1], b[0]).y));
    for (int k = 0; k < 3; ++k) {
        m[k] = a[k];
        m[3 + k] = b[k];
    }
    m[6] = cconj(c0);
    m[7] = cconj(c1);
    m[8] = cconj(c2);
}

__global__ __launch_bounds__(GT) void gauge_plaquette_kernel(const double2* __restrict__ U, Geo g, long V,
                                                             double* __restrict__ partial) {
    __shared__ double red[GT / 64];
    const long x = (long)blockIdx.x * GT + threadIdx.x;
    double acc = 0.0;
    if (x < V) {
        int c[4];
        g.coords(x, c);
        for (int mu = 0; mu < 4; ++mu) {
            const long xpmu = g.shift(c, mu, +1);
            for (int nu = mu + 1; nu < 4; ++nu) {
                const long xpnu = g.shift(c, nu, +1);
                const M3 P = mul(mul(mul(load_link(U, x, mu), load_link(U, xpmu, nu)), dag(load_link(U, xpnu, mu))),
                                 dag(load_link(U, x, nu)));
                acc += P.e[0].x + P.e[4].x + P.e[8].x;
            }
        }
    }
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < GT / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

__global__ void gauge_scale_kernel(double* v, double f) { v[0] *= f; }

Geo geo_of(const int dims[4]) {
    Geo g;
    for (int mu = 0; mu < 4; ++mu) g.L[mu] = dims[mu];
    return g;
}

}  // namespace

void gauge_sweep(void* U, const int dims[4], double beta, unsigned long long seed, long long sweep_index,
                 bool heatbath, hipStream_t st) {
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3], Vh = V / 2;
    const Geo g = geo_of(dims);
    const unsigned long long key = mix64(seed * GK1 + (unsigned long long)sweep_index * GK2);
    const unsigned blocks = (unsigned)((Vh + GU - 1) / GU);
    for (int mu = 0; mu < 4; ++mu)
        for (int p = 0; p < 2; ++p) {
            hipLaunchKernelGGL(gauge_update_kernel, dim3(blocks), dim3(GU), 0, st, static_cast<double2*>(U), g, mu, p,
                               beta, key, heatbath ? 1 : 0, Vh);
            DWF_HIP(hipGetLastError());
        }
    const long nl = V * 4;
    hipLaunchKernelGGL(gauge_reunitarize_kernel, dim3((unsigned)((nl + GT - 1) / GT)), dim3(GT), 0, st,
                       static_cast<double2*>(U), nl);
    DWF_HIP(hipGetLastError());
}

int gauge_plaquette_partials(const int dims[4]) {
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    return (int)((V + GT - 1) / GT);
}

void gauge_plaquette(const void* U, const int dims[4], double* partial, double* out_dev, hipStream_t st) {
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const int nb = gauge_plaquette_partials(dims);
    hipLaunchKernelGGL(gauge_plaquette_kernel, dim3(nb), dim3(GT), 0, st, static_cast<const double2*>(U),
                       geo_of(dims), V, partial);
    DWF_HIP(hipGetLastError());
    finalize(partial, nb, 1, out_dev, 0, st);
    hipLaunchKernelGGL(gauge_scale_kernel, dim3(1), dim3(1), 0, st, out_dev, 1.0 / (18.0 * (double)V));
    DWF_HIP(hipGetLastError());
}

}  // namespace dwf
