/*
 * dwf.h -- C ABI of libdwf, an MI355X (gfx950) solver for the 5D domain-wall
 * fermion system of lattice QCD, standard and Neff (alpha) form.
 *
 * The operations follow the paper's statement of the problem
 * (arXiv 2602.14454):
 *   D_W     Wilson kernel D_W(-M0)                      Sec. 2.1, eq. Wilson_matrix
 *   D       5D operator, standard form                  Sec. 2.2, eq. domainwall_general
 *   D^(a)   Neff form (alpha)                           Sec. 2.3, eq. domainwall_neff
 *   b5, x4  b5 = (-D_-) P^dag (0,..,0,b4), x4 = [P^dag x5]_{s=1}
 *                                                       Sec. 2.3, eq. 5D_linear_equation
 *   D^      even-odd Schur operator 1 - Dee^-1 Deo Doo^-1 Doe
 *                                                       Sec. 2.3, eq. even-odd_linear_equation
 *   solve   CG on D^dag D^ (CGNR), optionally with a low-precision inner
 *           solve inside FP64 defect correction          Sec. 2.3 (CGNR and the
 *                                                       single-precision-preconditioner paragraph)
 *
 * Status codes: every call returns an int.
 *   DWF_OK 0, DWF_NOT_CONVERGED 1 (outputs hold the best iterate),
 *   DWF_EINVAL -1 (bad argument / null pointer), DWF_EDIMS -2 (odd or too
 *   small lattice extent, unsupported Ls), DWF_ENOMEM -3, DWF_EHIP -4 (HIP
 *   runtime error), DWF_ESTATE -5 (object not ready, e.g. no gauge field),
 *   DWF_ENAN -6 (NaN/Inf met in a reduction).
 *   No C++ exception crosses the ABI; dwf_last_error() returns a
 *   thread-local message describing the last failure.
 *
 * Canonical layouts (all buffers are DEVICE pointers owned by the caller,
 * contiguous; the library never frees or keeps them):
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) & 1; eo = lex >> 1
 *   gauge  complex128 U[lex][mu][row][col], mu = 0..3 <-> x,y,z,t; U_mu(x): x -> x+mu
 *   4D     complex128 v[lex][spin][colour]
 *   5D     complex128 v[s][lex][spin][colour], s = 0..Ls-1 (paper s = 1..Ls)
 *   even   complex128 v[s][eo][spin][colour] over parity-0 sites
 *   gamma matrices: chiral basis, gamma_5 = diag(1,1,-1,-1); P+ = spins 0,1.
 *   4D boundary conditions: periodic in x, y, z; antiperiodic in t if asked.
 *   Multi-RHS buffers are nrhs canonical vectors back to back.
 *
 * Streams: every call enqueues on `stream` (a hipStream_t; NULL = default
 * stream).  Calls that return host scalars (solve, residuals, Lanczos)
 * synchronise that stream before returning.
 */
#ifndef DWF_H
#define DWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    DWF_OK = 0, DWF_NOT_CONVERGED = 1,
    DWF_EINVAL = -1, DWF_EDIMS = -2, DWF_ENOMEM = -3, DWF_EHIP = -4,
    DWF_ESTATE = -5, DWF_ENAN = -6
};

typedef enum { DWF_F64 = 0, DWF_F32 = 1, DWF_BF16 = 2 } dwf_prec;
typedef enum { DWF_FULL5D = 0, DWF_EVEN5D = 1 } dwf_space;
typedef enum {
    DWF_ALGO_CGNR = 0,         /* FP64 CGNR (restarted if the 5D residual is not yet met)        */
    DWF_ALGO_DC = 1,           /* FP64 defect correction around restarted low-precision CGNR     */
    DWF_ALGO_FGCR_LEARNED = 2, /* FP64 defect correction around FP32 flexible GCR on D^dag D^,    */
                               /* right-preconditioned by the learned network (ptc_model); on  */
                               /* NaN or stagnation the solve continues with CGNR (fallback)   */
    DWF_ALGO_MIXED = 3         /* low-precision CGNR with FP64 reliable updates (inner_tol: the  */
                               /* residual drop that triggers an update; <= 0: 0.1 FP32, 0.25 BF16) */
} dwf_algo;

typedef struct dwf_lattice dwf_lattice;
typedef struct dwf_op dwf_op;
typedef struct dwf_ptc dwf_ptc;             /* learned preconditioner (network weights, Adam state) */
typedef struct dwf_ptc_pairs dwf_ptc_pairs; /* device-resident training pairs of one operator */

typedef struct {
    double   tol;         /* target true relative residual of the 5D system |b5 - D x5| / |b5| */
    int      maxiter;     /* cap on operator applications of the (inner) CG, counted as iterations */
    int      algo;        /* dwf_algo */
    int      inner_prec;  /* dwf_prec of the inner CG for DWF_ALGO_DC (F32 or BF16) */
    double   inner_tol;   /* relative reduction asked of each inner solve (DC) */
    int      check_every; /* host convergence check period of the CG loop (>= 1); the FP32 inner
                             step of DWF_ALGO_DC meant to reach tol checks sooner where the
                             decrease of the residual since the previous check predicts its
                             target (never later) */
    int      paper_mode;  /* 1: plain CGNR in inner_prec stopping at |r|^2/|D^dag b~|^2 < 1e-14
                             (Sec. 3.2 criterion), no defect correction; iteration counting only.
                             Returns DWF_NOT_CONVERGED (converged = 0) if maxiter stops it first. */
    void*    ptc_model;   /* dwf_ptc* for DWF_ALGO_FGCR_LEARNED (NULL: FGCR without preconditioner) */
    int      restart;     /* FGCR restart length (1..64) */
    int      autotune;    /* batched solves: 0 cached tiles or defaults, 1 tune when not cached,
                             2 always re-tune */
    int      use_graph;   /* batched solves: 1 replay the CG iteration body as a HIP graph */
    int      schur;       /* single solves: 0 the left Schur system (1 - Dee^-1 Deo Doo^-1 Doe) x_e = b~_e
                             (the solver; Sec. 2.3 eq. even-odd_linear_equation); 1 the right form
                             (1 - Deo Doo^-1 Doe Dee^-1) y_e = b'_e, x_e = Dee^-1 y_e (Sec. 2.3
                             eq. another_even-odd_linear_equation), CGNR on its normal equations,
                             composed from unfused kernels (algo CGNR or DC only); the alpha of the
                             Neff form cancels in it, the measurement of that claim; 2 the left form
                             with the sites split by their 5D parity (x+y+z+t+s) mod 2 (Sec. 2.3: the
                             split can be made in 5D or 4D), for c_s = 0 and even Ls only, where D_ee
                             and D_oo are diagonal (algo CGNR or DC, inner_prec F64 or F32;
                             DWF_EINVAL otherwise) */
} dwf_solve_params;

/* Solve report.  `iters` is the total of inner CG iterations over all
 * defect-correction steps (the total inner count; for plain FP64 CGNR it is
 * the CGNR iteration count).  The 4D residual is not a field because
 * dwf_solve receives b5 only: it comes from dwf_residual_4d(x4, b4) after
 * dwf_project_4d. */
typedef struct {
    int    iters;              /* total CG iterations (each = one D^ and one D^dag) */
    int    outer_iters;        /* defect-correction steps */
    int    fallback_used;      /* 1 if a fallback path was taken (stagnation / learned failure) */
    int    converged;
    double true_res5;          /* |b5 - D x5| / |b5| computed in FP64 at the end */
    double seconds;            /* wall time of the solve on the stream, b5 on device -> x5 on device */
    double final_rel_res_even; /* recursive relative residual of the even system at exit */
    int    final_inner_prec;   /* dwf_prec of the last inner solve (after any stagnation step-up) */
} dwf_solve_info;

/* Default solve parameters (FP64 CGNR to 1e-10). */
void dwf_solve_params_default(dwf_solve_params* p);

/* ---- lattice and gauge field -------------------------------------- */

/* Creates geometry (index maps, neighbour tables) for dims[4] = (Lx,Ly,Lz,Lt).
 * Every extent must be even and >= 2 (even-odd split, Sec. 2.3).  Owns its
 * device memory; free with dwf_lattice_destroy. */
int dwf_lattice_create(const int dims[4], int antiperiodic_t, dwf_lattice** out);
void dwf_lattice_destroy(dwf_lattice* lat);

/* Uploads the gauge links U_mu(x) (Sec. 2.1), canonical complex128 layout.
 * on_device = 1: U is a device pointer; 0: host pointer.  The library keeps
 * FP64, FP32 and BF16 copies in its internal layout (links gathered per
 * output parity, backward links stored as U^dag, antiperiodic phase folded). */
int dwf_lattice_set_gauge(dwf_lattice* lat, const void* U, int on_device, void* stream);

/* Lattice geometry queries (for tests), read back from the device tables the
 * kernels use and written to host arrays.  The library keeps each parity's
 * sites in an internal order (spatial bricks swept in t, for cache reuse):
 * lex_of_site [2][V/2] gives the lexicographic index of internal site i of
 * parity p; nbr [2][8][V/2] the lexicographic index of its neighbour in
 * direction d (d = 0..3: x+mu for mu = x,y,z,t; d = 4..7: x-mu). */
int dwf_lattice_maps(const dwf_lattice* lat, int* lex_of_site, int* nbr);

/* ---- operator ------------------------------------------------------- */

/* D^(alpha) with s-independent (b, c) (Sec. 2.2; Sec. 2.3 eq. domainwall_neff).
 * 2 <= Ls <= 16.  The op references lat (lat must outlive it). */
int dwf_op_create(dwf_lattice* lat, int Ls, double M0, double m, double b, double c,
                  double alpha, dwf_op** out);
/* The same with s-dependent coefficients: D_+^(s) = b[s] D_W + 1 and
 * D_-^(s) = c[s] D_W - 1 in row s = 0..Ls-1 (paper s = 1..Ls) of
 * eq. domainwall_general (Sec. 2.2: Shamir (1,0), Borici (1,1), Moebius
 * b - c constant, and Chiu's optimal b_s = c_s = omega_s), Neff form by
 * alpha as above.  b, c: host arrays of Ls finite doubles, copied.  The
 * source -D_- P^dag (0,..,b4) of dwf_source_4d uses c[0] and c[Ls-1]. */
int dwf_op_create_sdep(dwf_lattice* lat, int Ls, double M0, double m, const double* b, const double* c,
                       double alpha, dwf_op** out);
void dwf_op_destroy(dwf_op* op);

/* out = D^(alpha) in (space = FULL5D, 5D canonical) or D^ in (EVEN5D, even
 * canonical); dagger = 1 applies the adjoint.  prec selects the arithmetic
 * (inputs/outputs are complex128 and converted).  in and out must not alias. */
int dwf_apply(const dwf_op* op, int space, int dagger, int prec, void* out, const void* in,
              void* stream);

/* out = D^dag D^ in on even canonical vectors (the CGNR normal operator). */
int dwf_apply_normal(const dwf_op* op, int prec, void* out, const void* in, void* stream);

/* Schur operator of the split by 5D parity (Sec. 2.3: even and odd sites in
 * five instead of four dimensions; eq. even-odd_linear_equation with those
 * blocks): out5 = D^5 in5 = (1 - D_ee^-1 D_eo D_oo^-1 D_oe) in5, or its
 * adjoint for dagger = 1, where "e" are the (s, x) with (x+y+z+t+s) even
 * (s = 0..Ls-1).  in5, out5: canonical 5D complex128 device fields
 * (Ls*V*12); only the 5D-even entries of in5 are read, the 5D-odd entries of
 * out5 are set to zero.  prec DWF_F64 or DWF_F32 (inputs and outputs stay
 * complex128).  Needs c_s = 0 for every s and an even Ls (D_ee, D_oo
 * diagonal; the mass term joins s = Ls-1 to s = 0), else DWF_EINVAL; in5
 * and out5 must not alias.  Synchronous on `stream`. */
int dwf_apply_eo5(const dwf_op* op, int prec, int dagger, void* out5, const void* in5, void* stream);

/* out = D^dag D^ in as dwf_apply_normal, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Allocates nothing: its four half-field
 * temporaries live in a static device array of the library (128 MiB per GPU,
 * held until the process ends); a lattice whose four half fields in
 * precision prec exceed it is rejected with DWF_EDIMS before anything is
 * enqueued (e.g. Ls = 16: up to about 10^4 sites per parity in FP64).  The
 * work is enqueued on `stream` and the call does not synchronise.  Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (several streams or host threads) race and must be serialised by the
 * caller.  The operator's lattice must live on the current device. */
int dwf_apply_normal_noalloc(const dwf_op* op, int prec, void* out, const void* in, void* stream);

/* One CGNR residual update (Sec. 2.3, CG on D^dag D^): with rr = |r|^2,
 * alpha = rr / |D^ p|^2 and r <- r - alpha D^dag D^ p, computed as inside
 * dwf_solve (the update is fused into the last hop of D^dag D^, the norms
 * reduced in FP64).  r and p are even canonical complex128 device vectors;
 * r is updated in place (rounded through the compute type: FP64 for
 * DWF_F64, FP32 otherwise), p is read in precision prec.  alpha and rr_new
 * (= |r|^2 after the update; each may be NULL) are host outputs.
 * Synchronises the stream. */
int dwf_cg_residual_update(const dwf_op* op, int prec, void* r, const void* p, double* alpha, double* rr_new,
                           void* stream);

/* b5 = (-D_-) P^dag (0, ..., 0, b4)  (Sec. 2.3, eq. 5D_linear_equation). */
int dwf_source_4d(const dwf_op* op, void* b5, const void* b4, void* stream);

/* x4 = P_- x5(s=1) + P_+ x5(s=Ls)  (Sec. 2.2 eq. 4d_quark_field). */
int dwf_project_4d(const dwf_op* op, void* x4, const void* x5, void* stream);

/* Solves D^(alpha) x5 = b5 through the even-odd Schur system (x5, b5 5D
 * canonical).  info may be NULL.  Returns DWF_OK or DWF_NOT_CONVERGED.
 * The operator keeps its solve workspace (nine FP64 half-lattice vectors
 * plus the inner-precision CG vectors) from the first solve until
 * dwf_op_destroy, so later solves allocate nothing; solves on one operator
 * from several threads run one at a time.  A solve that returns an error
 * drops the workspace. */
int dwf_solve(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm,
              dwf_solve_info* info, void* stream);

/* Batched solve of n operators (lattices may differ in size, Ls, mass and
 * (b, c, alpha)), nrhs[i] right-hand sides each: x5[i] and b5[i] hold
 * nrhs[i] 5D canonical fields back to back (device).  Each right-hand side
 * ("slot") is solved as by dwf_solve with algo DWF_ALGO_DC (FP64 defect
 * correction around an FP32/BF16-storage CGNR, Sec. 2.3) or DWF_ALGO_CGNR
 * (FP64 inner); the slots share every kernel launch of the inner iteration
 * (the hops of all operators with the same ceil(Ls/4) in one work-list
 * launch, links of a tile reused across right-hand sides), each with its own
 * CG scalars and stopping test, and the iteration body is replayed as a HIP
 * graph (prm->use_graph).  Tiles (right-hand sides per block, block order)
 * come from the autotuner (prm->autotune).  infos: sum(nrhs) entries in slot
 * order (operator-major), or NULL; `seconds` is the time of the whole batch.
 * prm NULL: DC with FP32 inner, tol 1e-10.  Returns DWF_OK when every slot
 * reached tol, else DWF_NOT_CONVERGED. */
int dwf_solve_batch(int n, const dwf_op* const* ops, void* const* x5, const void* const* b5, const int* nrhs,
                    const dwf_solve_params* prm, dwf_solve_info* infos, void* stream);

/* Tile autotuner of the batched solve: times the four hops of D^dag D^ for
 * every (right-hand sides per block, block order) candidate with HIP events
 * and keeps the fastest, keyed by (arch, precision, dims, Ls, nrhs of every
 * operator), in memory and in the text file named by $DWF_TUNE_CACHE
 * (default $HOME/.cache/libdwf_tune.txt; "off": memory only).  force = 1
 * re-times a cached key.  ms (may be NULL): time of the four hops.
 * Cache key: "gfx950|p<prec>" followed by "|<Lx>x<Ly>x<Lz>x<Lt>s<Ls>r<nrhs>"
 * per operator in batch order; entry (nrb = right-hand sides per block
 * 1..64, order = 0 tiles fastest / 1 right-hand-side chunks fastest). */
int dwf_autotune_batch(int n, const dwf_op* const* ops, const int* nrhs, int prec, int force, int* nrb,
                       int* order, double* ms, void* stream);
/* Tune-cache access (host only, no GPU call): put an entry, look one up
 * (DWF_NOT_CONVERGED when absent), and drop the in-memory copy so the next
 * access re-reads the file. */
int dwf_tune_cache_put(const char* key, int nrb, int order, double ms);
int dwf_tune_cache_get(const char* key, int* nrb, int* order, double* ms);
int dwf_tune_cache_reload(void);

/* |b5 - D^(alpha) x5| / |b5| in FP64. */
int dwf_true_residual(const dwf_op* op, const void* x5, const void* b5, double* rel, void* stream);

/* 4D residual |r4| / |b4| of a 4D solution x4 for source b4 (both 4D
 * canonical, device).  With D_eff(m) y = [P^dag D(1)^-1 D(m) P (y,0,..,0)]_{s=1}
 * at alpha = 1, the exact x4 of any alpha satisfies (1-m) x4 + b4 =
 * D_eff^-1 b4 (the 4D solution is alpha independent, Sec. 2.3), so
 * r4 = b4 - D_eff((1-m) x4 + b4).  Costs one D(m) and one m = 1 FP64
 * solve to tol_inner (<= 0: 1e-13).  Returns DWF_NOT_CONVERGED (rel still
 * written) when that inner solve stops short of tol_inner.  Synchronises
 * the stream. */
int dwf_residual_4d(const dwf_op* op, const void* x4, const void* b4, double tol_inner, double* rel,
                    void* stream);

/* Smallest and largest eigenvalue of the CGNR normal operator D^dag D^ (the
 * condition number study of Sec. 3.2.1, measured there with implicitly
 * restarted Lanczos in double precision).  Thick-restart Lanczos in FP64
 * with full re-orthogonalisation: `basis` Krylov vectors (device memory:
 * (basis + 1 + keep) even FP64 fields), restart keeping `keep` Ritz vectors,
 * at most `max_restarts` restarts per end, convergence when the Ritz
 * residual |beta_m y_m| <= tol * |theta|.  matvecs and converged may be NULL.
 * Returns DWF_OK, or DWF_NOT_CONVERGED with the best Ritz values. */
int dwf_lanczos_extremes(const dwf_op* op, int basis, int keep, int max_restarts, double tol,
                         double* lambda_min, double* lambda_max, int* matvecs, int* converged, void* stream);

/* ---- learned preconditioner ----------------------------------------
 * A linear gauge-equivariant parallel-transport convolution network
 * M = PTC_2 o PTC_1 (1 -> hidden -> 1 channels) used as the right
 * preconditioner of flexible GCR on the CGNR normal equations
 * (D^dag D^, Sec. 2.3).  One layer:
 *   out^a(x,s) = sum_b sum_p W_p^{ab} T_p[in^b](x,s)
 * with W_p^{ab} a complex 4x4 spin matrix and the 11 paths p = 0 (identity),
 * 1..4 (T_{+mu} psi(x) = U_mu(x) psi(x+mu), mu = x,y,z,t), 5..8
 * (T_{-mu} psi(x) = U_mu(x-mu)^dag psi(x-mu)), 9 and 10 (psi(s+1), psi(s-1),
 * zero outside the fifth dimension).  The fermion boundary phase is part of
 * the transports.  Layer 1 reads an even field and writes hidden channels on
 * both parities; layer 2 writes the even output.  FP32 weights and
 * activations.  Weights (host, complex64 interleaved): W1 [11][hidden][1][4][4]
 * followed by W2 [11][1][hidden][4][4], 2*11*hidden*16 complex numbers. */

/* New model: W = identity on path 0 / channel 0 of both layers plus seeded
 * complex Gaussian noise of standard deviation init_scale; 1 <= hidden <= 64. */
int dwf_ptc_create(int hidden, unsigned long long seed, double init_scale, dwf_ptc** out);
void dwf_ptc_destroy(dwf_ptc* m);
/* Training loss of the model (used by gradient, train and eval), for pairs
 * (r, e) with r = A e, A = D^dag D^:
 *   kind 0:           |M r - e|^2 / |e|^2                       (error loss)
 *   kind 1 (default): |A (M r - e)|^2 / |r|^2 = |A M r - r|^2 / |r|^2
 *                     (residual left by the right-preconditioned operator;
 *                     costs two more applications of A per step).  The error
 *                     loss weights the low modes a local network cannot
 *                     invert; fitted with it, A M is not positive and FGCR
 *                     stalls. */
int dwf_ptc_set_loss(dwf_ptc* m, int kind);
/* hidden channels, number of complex weights, Adam steps taken (each may be NULL) */
int dwf_ptc_info(const dwf_ptc* m, int* hidden, int* nweights, int* steps);
int dwf_ptc_get_weights(const dwf_ptc* m, void* weights_c64_host);
int dwf_ptc_set_weights(dwf_ptc* m, const void* weights_c64_host);
/* out_e = M in_e on even canonical complex128 device vectors (computed in FP32). */
int dwf_ptc_apply(dwf_ptc* m, const dwf_op* op, void* out_e, const void* in_e, void* stream);
/* Loss |M r - e|^2 / |e|^2 and its gradient dL/dRe W + i dL/dIm W (host,
 * complex64, weight layout; may be NULL) for one pair of even canonical
 * complex128 device vectors. */
int dwf_ptc_gradient(dwf_ptc* m, const dwf_op* op, const void* r_e, const void* e_e, double* loss,
                     void* grad_c64_host, void* stream);
/* Training pairs from the solver itself: CGNR on the Schur system is run
 * from 0 and at each iteration k in snap_iters the pair
 * (r_k = D^dag D^ e_k, e_k = x* - x_k) is kept on the device in FP32.  The
 * system is that of the 5D source b5 (canonical, device; x* by FP64 CGNR
 * to 1e-10) or, with b5 = NULL, one with known solution: x* a seeded
 * uniform random even field and b~ = D^ x* (k = 0 then gives the pair
 * (D^dag D^ x*, x*) of a random error). */
int dwf_ptc_pairs_create(const dwf_op* op, const void* b5, unsigned long long seed, int nsnap,
                         const int* snap_iters, dwf_ptc_pairs** out, void* stream);
/* copies pair k out as even canonical complex128 device vectors */
int dwf_ptc_pairs_get(const dwf_ptc_pairs* p, int k, void* r_e, void* e_e, void* stream);
void dwf_ptc_pairs_destroy(dwf_ptc_pairs* p);
/* `steps` Adam steps (learning rate lr, betas 0.9/0.999, eps 1e-8), each on
 * one pair drawn by a seeded counter hash over all sets; loss_history
 * (host, `steps` doubles, may be NULL) receives the loss of every step.  The
 * sets' operators (and lattices) must still exist. */
int dwf_ptc_train(dwf_ptc* m, int nsets, dwf_ptc_pairs* const* sets, int steps, double lr,
                  unsigned long long seed, double* loss_history, void* stream);
/* mean loss over every pair of the sets */
int dwf_ptc_eval(dwf_ptc* m, int nsets, dwf_ptc_pairs* const* sets, double* mean_loss, void* stream);
/* Checkpoint: "DWFPTC01", hidden, Adam step, weights and Adam moments, FNV-1a
 * checksum; load rejects a file whose checksum or size does not match. */
int dwf_ptc_save(const dwf_ptc* m, const char* path);
int dwf_ptc_load(const char* path, dwf_ptc** out);

/* ---- quenched gauge fields ------------------------------------------
 * The paper's ensembles are quenched configurations of the plaquette gauge
 * action S = beta sum_P (1 - Re tr U_P / 3) at beta = 6.0 and 5.7 (Sec. 3.1).
 * U: canonical complex128 links U[lex][mu][3][3] on the device, periodic in
 * every direction, updated in place; every extent even and >= 2.
 *
 * dwf_gauge_sweeps: nsweeps times (one heatbath sweep, then n_or
 * over-relaxation sweeps) over all links: Cabibbo-Marinari SU(2)-subgroup
 * heatbath with Kennedy-Pendleton's sampler and the microcanonical reflection
 * in the same subgroups, links of one direction and one site parity updated
 * together (mu = 0..3, parity 0 then 1), re-projection onto SU(3) after
 * every sweep.  Random numbers are a pure function of (seed, sweep index
 * sweep0 + k, link, subgroup, draw) (SplitMix64 of counters), so a run is
 * reproducible and can be continued by passing sweep0.  Synchronises. */
int dwf_gauge_sweeps(const int dims[4], void* U, double beta, int nsweeps, int n_or, unsigned long long seed,
                     long long sweep0, void* stream);
/* average Re tr U_P / 3 over all sites and planes (FP64); synchronises */
int dwf_gauge_plaquette(const int dims[4], const void* U, double* plaq, void* stream);

/* ---- measurement helpers ------------------------------------------ */

/* Times `nrep` launches of the fused half-lattice hop kernel of D^ (the
 * first half, out_o = Q H_oe K in_e) in precision prec on internal
 * buffers, with HIP events on the stream the kernel runs on.  Writes the
 * mean kernel time in ms and the algorithmic bytes of one launch. */
int dwf_bench_hop(const dwf_op* op, int prec, int nrep, double* ms_per_launch,
                  double* bytes_per_launch, void* stream);

/* Times `nrep` applications of the learned preconditioner (its three layer
 * kernels on internal FP32 fields of `op`, seeded non-zero input) with HIP
 * events on `stream`; writes the mean time of one application in ms. */
int dwf_ptc_bench_apply(dwf_ptc* m, const dwf_op* op, int nrep, double* ms_per_apply, void* stream);

/* Times `nrep` launches of a plain 16-byte-vector copy of `bytes` bytes
 * (device buffers owned by the library); used to calibrate memory counters. */
int dwf_bench_copy(size_t bytes, int nrep, double* ms_per_launch, void* stream);

const char* dwf_status_string(int status);
const char* dwf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
