// Extreme eigenvalues of the CGNR normal operator D^dag D^ (the condition
// number study of the paper, Sec. 3.2.1, which used implicitly restarted
// Lanczos in double precision).  Here: thick-restart Lanczos in FP64, which
// for a Hermitian operator is equivalent to implicit restarting.
//
// The Krylov basis lives in HBM as FP64 internal half fields.  Every new
// vector is orthogonalised against the whole basis twice (classical
// Gram-Schmidt with one re-orthogonalisation), all inner products of a step
// are reduced on the device and read back once.  The projected matrix is real
// symmetric (arrowhead after a restart, tridiagonal otherwise) and is
// diagonalised on the host by cyclic Jacobi rotations.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "blas.h"
#include "dwf_internal.h"
#include "ops.h"
#include "solver.h"

namespace dwf {

// Cyclic Jacobi eigenvalue method for a real symmetric n x n matrix A
// (row-major).  Returns eigenvalues ascending in w and the eigenvectors as
// the columns of Z (row-major, Z[i*n + k] = component i of vector k).
static void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& Z) {
    Z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                const double a = A[(size_t)p * n + q];
                if (p == q) diag += a * a; else off += a * a;
            }
        if (off <= 1e-30 * diag || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double zkp = Z[(size_t)k * n + p], zkq = Z[(size_t)k * n + q];
                    Z[(size_t)k * n + p] = c * zkp - s * zkq;
                    Z[(size_t)k * n + q] = s * zkp + c * zkq;
                }
            }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
    std::vector<double> Zs((size_t)n * n);
    w.resize(n);
    for (int k = 0; k < n; ++k) {
        w[k] = A[(size_t)idx[k] * n + idx[k]];
        for (int i = 0; i < n; ++i) Zs[(size_t)i * n + k] = Z[(size_t)i * n + idx[k]];
    }
    Z.swap(Zs);
}

namespace {
struct Ctx {
    const dwf_op* op;
    hipStream_t st;
    long n;
    std::vector<DevBuf> V;   // basis (m + 1) followed by restart temporaries
    DevBuf w, to, tv, partial, scal;
    double* hs;               // pinned host scalars
    int nparts;
    int matvecs = 0;

    void apply(void* out, const void* in) {
        apply_normal(op, ST_F64, out, in, to.p, tv.p, nullptr, 1, st);
        ++matvecs;
    }
    // complex inner products <V[i], x> for i < cnt, one device read-back
    void dots(int cnt, const void* x, std::vector<double>& re, std::vector<double>& im) {
        double* pp = partial.as<double>();
        double* sc = scal.as<double>();
        for (int i = 0; i < cnt; ++i) {
            dot_partial(ST_F64, V[i].p, x, n, pp + (size_t)i * 2 * nparts, st);
            finalize(pp + (size_t)i * 2 * nparts, nparts, 2, sc + 2 * i, 0, st);
            finalize(pp + (size_t)i * 2 * nparts + 1, nparts, 2, sc + 2 * i + 1, 0, st);
        }
        DWF_HIP(hipMemcpyAsync(hs, sc, sizeof(double) * 2 * cnt, hipMemcpyDeviceToHost, st));
        DWF_HIP(hipStreamSynchronize(st));
        re.resize(cnt);
        im.resize(cnt);
        for (int i = 0; i < cnt; ++i) { re[i] = hs[2 * i]; im[i] = hs[2 * i + 1]; }
    }
    double norm(const void* x) {
        double* pp = partial.as<double>();
        double* sc = scal.as<double>();
        norm2_partial(ST_F64, x, n, pp, st);
        finalize(pp, nparts, 1, sc, 0, st);
        DWF_HIP(hipMemcpyAsync(hs, sc, sizeof(double), hipMemcpyDeviceToHost, st));
        DWF_HIP(hipStreamSynchronize(st));
        return std::sqrt(hs[0]);
    }
};
}  // namespace

// One thick-restart Lanczos run targeting the smallest (largest = false) or
// largest eigenvalue.  Returns the converged Ritz value (or the best one).
static double trlan(Ctx& C, int m, int keep, int max_restarts, double tol, bool largest, bool* conv,
                    unsigned long long seed) {
    const long n = C.n;
    const dwf_lattice* L = C.op->lat;
    std::vector<double> H((size_t)(m + 1) * (m + 1), 0.0);
    auto Hs = [&](int i, int j) -> double& { return H[(size_t)i * (m + 1) + j]; };
    // random start vector, normalised
    random_fill_f64(C.V[0].p, (long)C.op->Ls * 12, L->Vh, L->Vhp, seed, C.st);
    {
        const double nv = C.norm(C.V[0].p);
        axpby(ST_F64, ST_F64, C.V[0].p, C.V[0].p, n, nullptr, 1.0 / nv, nullptr, 0.0, nullptr, C.st);
    }
    int jstart = 0;
    double theta_best = 0.0;
    *conv = false;
    std::vector<double> re, im, re2, im2, w, Z;
    for (int cycle = 0; cycle <= max_restarts; ++cycle) {
        for (int j = jstart; j < m; ++j) {
            C.apply(C.w.p, C.V[j].p);
            C.dots(j + 1, C.w.p, re, im);
            for (int i = 0; i <= j; ++i) caxpy(ST_F64, C.w.p, C.V[i].p, n, -re[i], -im[i], C.st);
            C.dots(j + 1, C.w.p, re2, im2);
            for (int i = 0; i <= j; ++i) caxpy(ST_F64, C.w.p, C.V[i].p, n, -re2[i], -im2[i], C.st);
            for (int i = 0; i <= j; ++i) Hs(i, j) = Hs(j, i) = re[i] + re2[i];
            const double beta = C.norm(C.w.p);
            Hs(j + 1, j) = Hs(j, j + 1) = beta;
            if (!(beta > 0.0) || !std::isfinite(beta)) throw Error{DWF_ENAN, "Lanczos breakdown"};
            axpby(ST_F64, ST_F64, C.V[j + 1].p, C.w.p, n, nullptr, 1.0 / beta, nullptr, 0.0, nullptr, C.st);
        }
        std::vector<double> Hm((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) Hm[(size_t)i * m + j] = Hs(i, j);
        jacobi_eigen(m, Hm, w, Z);
        const double beta_m = Hs(m, m - 1);
        // order of preference: ascending (smallest) or descending (largest)
        std::vector<int> order(m);
        std::iota(order.begin(), order.end(), 0);
        if (largest) std::reverse(order.begin(), order.end());
        const int t = order[0];
        theta_best = w[t];
        const double res = std::fabs(beta_m * Z[(size_t)(m - 1) * m + t]);
        if (res <= tol * std::fabs(theta_best)) {
            *conv = true;
            break;
        }
        if (cycle == max_restarts) break;
        // thick restart: keep the `keep` preferred Ritz vectors and the residual direction
        for (int q = 0; q < keep; ++q) {
            void* dst = C.V[m + 1 + q].p;
            axpby(ST_F64, ST_F64, dst, C.V[0].p, n, nullptr, Z[(size_t)0 * m + order[q]], nullptr, 0.0, nullptr, C.st);
            for (int l = 1; l < m; ++l)
                axpby(ST_F64, ST_F64, dst, C.V[l].p, n, nullptr, Z[(size_t)l * m + order[q]], nullptr, 1.0, nullptr,
                      C.st);
        }
        for (int q = 0; q < keep; ++q) std::swap(C.V[q], C.V[m + 1 + q]);
        std::swap(C.V[keep], C.V[m]);
        std::fill(H.begin(), H.end(), 0.0);
        for (int q = 0; q < keep; ++q) {
            Hs(q, q) = w[order[q]];
            Hs(keep, q) = Hs(q, keep) = beta_m * Z[(size_t)(m - 1) * m + order[q]];
        }
        jstart = keep;
    }
    return theta_best;
}

void lanczos_extremes(const dwf_op* op, int m, int keep, int max_restarts, double tol, double* lmin, double* lmax,
                      int* matvecs, int* converged, hipStream_t st) {
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    DWF_REQUIRE(m >= 4 && keep >= 1 && keep < m - 1, DWF_EINVAL, "need 4 <= basis and 1 <= keep < basis - 1");
    Ctx C;
    C.op = op;
    C.st = st;
    C.n = (long)op->Ls * 12 * L->Vhp;
    const size_t bytes = 16 * (size_t)C.n;
    for (int i = 0; i < m + 1 + keep; ++i) C.V.emplace_back(bytes);
    C.w.alloc(bytes);
    C.to.alloc(bytes);
    C.tv.alloc(bytes);
    C.nparts = blas_grid(C.n);
    C.partial.alloc(sizeof(double) * 2 * (size_t)C.nparts * (m + 1) + 64);
    C.scal.alloc(sizeof(double) * 2 * (m + 2));
    DWF_HIP(hipHostMalloc(reinterpret_cast<void**>(&C.hs), sizeof(double) * 2 * (m + 2), hipHostMallocDefault));
    int conv_lo = 0, conv_hi = 0;
    try {
        bool c1 = false, c2 = false;
        const double hi = trlan(C, m, keep, max_restarts, tol, true, &c1, 0x5eed1234ull);
        const double lo = trlan(C, m, keep, max_restarts, tol, false, &c2, 0x5eed5678ull);
        conv_hi = c1;
        conv_lo = c2;
        if (lmin) *lmin = lo;
        if (lmax) *lmax = hi;
    } catch (...) {
        (void)hipHostFree(C.hs);
        throw;
    }
    (void)hipHostFree(C.hs);
    if (matvecs) *matvecs = C.matvecs;
    if (converged) *converged = conv_lo && conv_hi;
}

}  // namespace dwf
