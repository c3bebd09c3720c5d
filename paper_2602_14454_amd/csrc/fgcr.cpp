// Flexible GCR on the CGNR normal equations with the learned preconditioner
// as right preconditioner (the flexible variant allows a preconditioner
// that is not a fixed polynomial of the operator).  Each iteration:
//   z_j = M r,  q_j = D^dag D^ z_j,  orthogonalise q_j (and z_j alongside)
//   against the q_i of the cycle,  alpha = <q_j, r> / |q_j|^2,
//   x += alpha z_j,  r -= alpha q_j.
// The directions are discarded every m iterations (restart); x and r carry on.
#include "fgcr.h"

#include <cmath>
#include <cstring>

#include "blas.h"
#include "ops.h"
#include "ptc_model.h"

namespace dwf {

FgcrWork::FgcrWork(const dwf_op* op, int m_) : m(m_) {
    DWF_REQUIRE(m >= 1 && m <= 64, DWF_EINVAL, "FGCR restart length must be 1..64");
    n = (long)op->Ls * 12 * op->lat->Vhp;
    const size_t fb = (size_t)n * sizeof(float2);
    x.alloc(fb);
    r.alloc(fb);
    t.alloc(fb);
    v.alloc(fb);
    Z.alloc((size_t)m * fb);
    Q.alloc((size_t)m * fb);
    const long nb = fg_blocks(n);
    partial.alloc((size_t)std::max<long>(std::max<long>(nb * 3, (long)m * nb * 2), blas_grid(n)) * sizeof(double) +
                  64);
    // scal: qq [m] | coef [m] double2 | alpha double2 | rr | nanflag
    scal.alloc(((size_t)m + 2 * (size_t)m + 2 + 2 + 2) * sizeof(double));
}

int fgcr(const dwf_op* op, dwf_ptc* M, FgcrWork& W, const void* b32, double tol_rel, int maxiter, int check_every,
         hipStream_t st, double* final_rel, bool* failed) {
    const long n = W.n;
    const int m = W.m;
    *failed = false;
    if (check_every < 1) check_every = 1;
    double* sc = W.scal.as<double>();
    double* qq = sc;
    double2* coef = reinterpret_cast<double2*>(sc + m);
    double2* alpha = reinterpret_cast<double2*>(sc + 3 * m);
    double* rr_slot = sc + 3 * m + 2;
    double* nanflag = sc + 3 * m + 3;
    double* pp = W.partial.as<double>();
    float2* x = W.x.as<float2>();
    float2* r = W.r.as<float2>();
    DWF_HIP(hipMemsetAsync(W.scal.p, 0, W.scal.bytes, st));
    DWF_HIP(hipMemsetAsync(W.x.p, 0, W.x.bytes, st));
    apply_dhat(op, ST_F32, 1, r, b32, W.t.p, W.v.p, 1, st);
    norm2_partial(ST_F32, r, n, pp, st);
    finalize(pp, blas_grid(n), 1, rr_slot, 0, st);
    double h[2];
    DWF_HIP(hipMemcpyAsync(h, rr_slot, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
    const double rr0 = h[0];
    if (!std::isfinite(rr0)) {
        *failed = true;
        return 0;
    }
    if (rr0 == 0.0) {
        if (final_rel) *final_rel = 0.0;
        return 0;
    }
    const double stop = tol_rel * tol_rel * rr0;
    double rr = rr0, rr_cycle = rr0;
    const int nbf = fg_blocks(n);
    int it = 0;
    while (it < maxiter) {
        const int j = it % m;
        float2* zj = W.Z.as<float2>() + (size_t)j * n;
        float2* qj = W.Q.as<float2>() + (size_t)j * n;
        if (M) M->forward(op, r, zj, st);
        else convert(ST_F32, ST_F32, zj, r, n, st);
        apply_normal(op, ST_F32, qj, zj, W.t.p, W.v.p, nullptr, 1, st);
        fg_orthogonalize(qj, zj, W.Q.as<float2>(), W.Z.as<float2>(), n, j, qq, pp, coef, st);
        fg_step(x, r, zj, qj, n, pp, qq + j, alpha, pp + 3 * nbf, nanflag, st);
        finalize(pp + 3 * nbf, nbf, 1, rr_slot, 0, st);
        ++it;
        const bool cycle_end = j == m - 1;
        if (it % check_every == 0 || it == maxiter || cycle_end) {
            DWF_HIP(hipMemcpyAsync(h, rr_slot, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
            DWF_HIP(hipStreamSynchronize(st));
            rr = h[0];
            if (h[1] != 0.0 || !std::isfinite(rr)) {
                *failed = true;
                break;
            }
            if (rr <= stop) break;
            if (cycle_end) {
                if (rr > 0.998 * rr_cycle) {   // |r| fell by less than 0.1% over a cycle
                    *failed = true;
                    break;
                }
                rr_cycle = rr;
            }
        }
    }
    if (final_rel) *final_rel = std::sqrt(rr / rr0);
    return it;
}

}  // namespace dwf
