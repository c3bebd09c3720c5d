// Flexible GCR (fgcr_kernels.hip kernels, fgcr.cpp solver).
#pragma once

#include <hip/hip_runtime.h>

#include "dwf_internal.h"

struct dwf_ptc;

namespace dwf {

int fg_blocks(long n);
// q -= sum_{i<j} c_i Q_i, z -= sum_{i<j} c_i Z_i with c_i = <Q_i, q> / qq[i] (classical Gram-Schmidt)
void fg_orthogonalize(float2* q, float2* z, const float2* Q, const float2* Z, long n, int j, const double* qq,
                      double* partial, double2* coef, hipStream_t st);
// qq_out = |q|^2, alpha = <q, r>/|q|^2, x += alpha z, r -= alpha q, rr_partial per block
void fg_step(float2* x, float2* r, const float2* z, const float2* q, long n, double* partial, double* qq_out,
             double2* alpha, double* rr_partial, double* nanflag, hipStream_t st);

// FGCR(m) on D^dag D^ e = D^dag b (b: FP32 Schur residual), right-preconditioned
// by the network M (nullptr: identity), FP32 vectors, from e = 0.  Stops when
// |r| <= tol_rel |r0| (normal residual) or after maxiter iterations.  Sets
// *failed on NaN or when a full cycle of m iterations reduces |r| by less
// than 0.1%; then x must not be used.  Result in W.x.
struct FgcrWork {
    int m;
    long n;
    DevBuf x, r, Z, Q, t, v, partial, scal;
    FgcrWork(const dwf_op* op, int m);
};
int fgcr(const dwf_op* op, dwf_ptc* M, FgcrWork& W, const void* b32, double tol_rel, int maxiter, int check_every,
         hipStream_t st, double* final_rel, bool* failed);

}  // namespace dwf
