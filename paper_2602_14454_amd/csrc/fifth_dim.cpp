// Fifth-dimension (s) algebra of the domain-wall operator, host FP64.
//
// The Neff-form operator is the standard one multiplied on the right by a
// 5D-local diagonal: D^(alpha) = D^(1) T with
//   T = diag_s(P_- + a P_+, a, ..., a, P_+ + a P_-),
// which follows from the paper's relation D^(alpha) P = D P A (Sec. 2.3,
// eq. relation_to_alpha=1) since T = P A P^dag.  (The paper's later remark
// writes P A^-1 P^dag; the relation itself fixes P A P^dag, and only the
// locality of T matters for its argument.)
//
// Writing D_+^(s) = b_s D_W + 1, D_-^(s) = c_s D_W - 1 (Sec. 2.2; row s of
// eq. domainwall_general carries the coefficients of that s) and collecting
// the s-structure into the shift M5
//   (M5 psi)_s = P_- psi_{s+1} + P_+ psi_{s-1},  P_+ psi_0 -> -m P_+ psi_Ls,
//                                                P_- psi_{Ls+1} -> -m P_- psi_1,
// gives D^(alpha) = D_W K + N with K = (B + C M5) T and N = (1 - M5) T,
// B = diag(b_s), C = diag(c_s) acting on the row index, all real Ls x Ls per
// chirality (s-independent (b, c): K = (b + c M5) T).  With D_W = (4 - M0) - H/2 (H the hopping term):
//   D = M - (1/2) H K,  M = (4 - M0) K + N   (site-diagonal, D_ee = D_oo = M),
// and the even-odd Schur operator of Sec. 2.3 becomes
//   D^ = 1 - (1/4) M^-1 H_eo Q H_oe K,  Q = K M^-1,
//   D^dag = 1 - (1/4) g5 K^T H_eo Q^T H_oe M^-T g5.
// Chirality chi = 0 is P_+ (spins 0,1), chi = 1 is P_- (spins 2,3).
#include <cmath>
#include <stdexcept>

#include "dwf_internal.h"

namespace dwf {

static std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n) {
    std::vector<double> C(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double a = A[i * n + k];
            if (a == 0.0) continue;
            for (int j = 0; j < n; ++j) C[i * n + j] += a * B[k * n + j];
        }
    return C;
}

static std::vector<double> inverse(std::vector<double> A, int n) {
    std::vector<double> X(n * n, 0.0);
    for (int i = 0; i < n; ++i) X[i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
        if (A[piv * n + col] == 0.0) throw Error{DWF_EINVAL, "singular site-local block M"};
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                std::swap(A[col * n + j], A[piv * n + j]);
                std::swap(X[col * n + j], X[piv * n + j]);
            }
        const double inv = 1.0 / A[col * n + col];
        for (int j = 0; j < n; ++j) { A[col * n + j] *= inv; X[col * n + j] *= inv; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[r * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[col * n + j]; X[r * n + j] -= f * X[col * n + j]; }
        }
    }
    return X;
}

FifthDim build_fifth_dim(int Ls, double M0, double m, const std::vector<double>& b, const std::vector<double>& c,
                         double alpha) {
    DWF_REQUIRE((int)b.size() == Ls && (int)c.size() == Ls, DWF_EINVAL, "b and c need Ls entries");
    FifthDim f;
    f.Ls = Ls;
    const int n = Ls;
    for (int chi = 0; chi < 2; ++chi) {
        std::vector<double> T(n * n, 0.0), M5(n * n, 0.0), I(n * n, 0.0);
        for (int s = 0; s < n; ++s) I[s * n + s] = 1.0;
        for (int s = 0; s < n; ++s) T[s * n + s] = alpha;
        if (chi == 0) {
            T[(n - 1) * n + (n - 1)] = 1.0;              // P_+ part of (P_+ + a P_-) at s = Ls
            for (int s = 1; s < n; ++s) M5[s * n + (s - 1)] += 1.0;
            M5[0 * n + (n - 1)] += -m;
        } else {
            T[0] = 1.0;                                  // P_- part of (P_- + a P_+) at s = 1
            for (int s = 0; s + 1 < n; ++s) M5[s * n + (s + 1)] += 1.0;
            M5[(n - 1) * n + 0] += -m;
        }
        std::vector<double> bcM5(n * n), omM5(n * n);
        for (int r = 0; r < n; ++r)
            for (int q = 0; q < n; ++q) {
                const int i = r * n + q;
                bcM5[i] = b[r] * I[i] + c[r] * M5[i];
                omM5[i] = I[i] - M5[i];
            }
        std::vector<double> K = matmul(bcM5, T, n);
        std::vector<double> N = matmul(omM5, T, n);
        std::vector<double> M(n * n);
        for (int i = 0; i < n * n; ++i) M[i] = (4.0 - M0) * K[i] + N[i];
        std::vector<double> Minv = inverse(M, n);
        f.T[chi] = T;
        f.M5[chi] = M5;
        f.K[chi] = K;
        f.N[chi] = N;
        f.M[chi] = M;
        f.Minv[chi] = Minv;
        f.Q[chi] = matmul(K, Minv, n);
    }
    return f;
}

}  // namespace dwf
