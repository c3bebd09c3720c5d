// CG workspace and solver entry points (solver.cpp).
#pragma once

#include <functional>
#include <string>

#include "dwf_internal.h"

namespace dwf {

// Page-locked host doubles (read-back of device CG scalars).
struct Pinned {
    double* h = nullptr;
    explicit Pinned(size_t n);
    ~Pinned();
    Pinned(const Pinned&) = delete;
    Pinned& operator=(const Pinned&) = delete;
};

// Inner CGNR workspace: x, r in storage kx; p, t (odd), v, w in storage kp;
// device CG scalars and their host read-back buffer.
struct CgWork {
    int kx, kp, nrhs;
    long n;   // complex elements per field (all RHS)
    DevBuf x, r, p, t, v, w, partial, scal;
    Pinned hs;
    // search directions of the last iterations and their alphas: x is formed
    // from them every ring_len iterations and at the end of a solve instead of
    // being read and written by every iteration
    int ring_len = 0;
    DevBuf ring, alphas;
    DevBuf ra, rb;   // temporaries of the right-preconditioned Schur CG (allocated on first use)
    CgWork(const dwf_op* op, int kx, int kp, int nrhs);
};

// Slots of a direction ring whose slots hold slot_bytes each: up to 16, as
// many as fit in 8 GiB, at least 2 (a shorter ring only folds into x more often).
int ring_slots(size_t slot_bytes);

// CG on D^dag D^ e = D^dag b from e = 0; b in storage kp.  Stops when the
// recursive residual |r| <= tol_rel |r0| or after maxiter iterations.
// Result in W.x.  Returns the iteration count.
// on_iter (optional) is called after iteration k with the device pointer of x_k.
using IterHook = std::function<void(int, const void*)>;
// predict_checks: the host convergence check comes at most check_every
// iterations after the previous one, sooner where the decrease of |r|^2 since
// that check, taken as geometric, predicts the target (see next_check_gap in
// solver.cpp); false: every check_every iterations.
int cgnr(const dwf_op* op, CgWork& W, const void* b_kp, double tol_rel, int maxiter, int check_every,
         hipStream_t st, double* final_rel, bool* nan_seen, const IterHook& on_iter = IterHook(),
         bool predict_checks = false);

// defect-correction inner target and step ratio (solver.cpp); DWF_TRACE in
// the environment prints one line per outer step to stderr
// *last (optional): the step asks for what reaching tol needs (the intended
// last step) rather than the standard reduction
double dc_target(double tol, double rel5, int kp, double standard, double f, bool* last = nullptr);
double dc_ratio(double achieved, double requested);
bool trace_on();

int solve(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm, dwf_solve_info* info,
          hipStream_t st);
double true_residual(const dwf_op* op, const void* x5, const void* b5, hipStream_t st);
// *converged (may be NULL): whether the inner m = 1 solve met tol_inner
double residual_4d(const dwf_op* op, const void* x4, const void* b4, double tol_inner, hipStream_t st,
                   bool* converged = nullptr);

// batch.cpp: batched solves and the tile autotuner of the work-list hop
int solve_batch(int n, const dwf_op* const* ops, void* const* x5, const void* const* b5, const int* nrhs,
                const dwf_solve_params* prm, dwf_solve_info* infos, hipStream_t st);
void autotune_batch(int n, const dwf_op* const* ops, const int* nrhs, int kp, int force, int* nrb, int* order,
                    double* ms, hipStream_t st);
bool tune_get(const std::string& key, int* nrb, int* order, double* ms);
void tune_put(const std::string& key, int nrb, int order, double ms);
void tune_forget();

// lanczos.cpp: extreme eigenvalues of D^dag D^ (thick-restart Lanczos, FP64)
void lanczos_extremes(const dwf_op* op, int m, int keep, int max_restarts, double tol, double* lmin, double* lmax,
                      int* matvecs, int* converged, hipStream_t st);

}  // namespace dwf
