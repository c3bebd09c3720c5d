/*
 * FP64 CPU oracle for the domain-wall fermion solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its Python binding) never calls it, and the two share
 * no code: no headers, kernels, helpers, tables or constant generators.
 *
 * Everything here is written straight from the paper's definitions, in
 * double precision, without blocking, fusion or reordering:
 *   - Wilson operator D_W(-M0) with full 4x4 (1 -/+ gamma_mu)      (Sec. 2.1, eq. Wilson_matrix)
 *   - 5D domain-wall operator, standard and Neff (alpha) form, as a
 *     block matrix in the fifth dimension                          (Sec. 2.2 eq. domainwall_general,
 *                                                                   Sec. 2.3 eq. domainwall_neff)
 *   - 5D source b5 = (-D_-) P^dag (0,..,0,b4) and projection
 *     x4 = [P^dag x5]_{s=1}                                        (Sec. 2.3, eq. 5D_linear_equation)
 *   - 4D even-odd Schur complement by restricting the 5D operator
 *     to parity sub-spaces; D_ee, D_oo inverted as dense per-site
 *     blocks                                                       (Sec. 2.3 Even-odd preconditioning,
 *                                                                   eq. even-odd_linear_equation)
 *   - CG on the normal equations D^dag D                           (Sec. 2.3, CGNR paragraph)
 *
 * Conventions (shared with the GPU path only through the ABI description):
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) & 1; eo = lex >> 1 (Lx even)
 *   links  U[(lex*4 + mu)*9 + row*3 + col], mu = 0..3 <-> x,y,z,t, U_mu(x): x -> x+mu
 *   4D     v[(lex*4 + spin)*3 + colour]
 *   5D     v[((s*V + lex)*4 + spin)*3 + colour], s = 0..Ls-1 (paper s = 1..Ls)
 *   even   v[((s*Vh + eo)*4 + spin)*3 + colour] over parity-0 sites
 *   gamma  chiral basis: gamma_k = [[0,-i sigma_k],[i sigma_k,0]], gamma_4 = [[0,1],[1,0]],
 *          gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 (paper Sec. 2.1)
 *   4D boundary: periodic in x,y,z; antiperiodic in t when antiperiodic_t != 0
 *   (a hop across the t boundary picks up -1).
 */
#ifndef DWF_ORACLE_H
#define DWF_ORACLE_H

#include <complex.h>

typedef double _Complex or_cplx;

typedef struct {
    int dims[4];
    int antiperiodic_t;
    int Ls;
    double M0;     /* domain-wall height; D_W = D_W(-M0) */
    double m;      /* quark mass */
    double b, c;   /* D_+ = b D_W + 1, D_- = c D_W - 1 (s-independent) */
    double alpha;  /* Neff parameter, alpha = 1 is the standard form */
    /* s-dependent coefficients (Sec. 2.2: D_+^(i) = b_i D_W + 1 and
     * D_-^(i) = c_i D_W - 1 in row i of the 5D matrix): Ls doubles each, or
     * NULL to use b, c for every row */
    const double* bs;
    const double* cs;
} or_params;

long or_volume(const int dims[4]);
void or_gamma(int mu, or_cplx out[16]);
void or_site_maps(const int dims[4], int* parity, int* eo, int* lex_of_eo_even, int* lex_of_eo_odd);
void or_neighbors(const int dims[4], int* nbr);
void or_wilson(const or_params* p, const or_cplx* U, const or_cplx* in, or_cplx* out,
               int dagger, int parity_mask);
void or_dwf_apply(const or_params* p, const or_cplx* U, const or_cplx* in5, or_cplx* out5,
                  int dagger, int parity_mask);
void or_local_block(const or_params* p, or_cplx* Mloc);
int  or_invert_dense(int n, const or_cplx* A, or_cplx* Ainv);
void or_dhat(const or_params* p, const or_cplx* U, const or_cplx* in_e, or_cplx* out_e, int dagger);
void or_schur_rhs(const or_params* p, const or_cplx* U, const or_cplx* b5, or_cplx* bt_e);
void or_reconstruct(const or_params* p, const or_cplx* U, const or_cplx* x_e,
                    const or_cplx* b5, or_cplx* x5);
int  or_cgnr_even(const or_params* p, const or_cplx* U, const or_cplx* bt_e, or_cplx* x_e,
                  double tol, int maxiter);
int  or_solve(const or_params* p, const or_cplx* U, const or_cplx* b5, or_cplx* x5,
              double tol, int maxiter, double* true_res);
void or_source_4d(const or_params* p, const or_cplx* U, const or_cplx* b4, or_cplx* b5);
void or_project_4d(const or_params* p, const or_cplx* x5, or_cplx* x4);
double or_residual_4d(const or_params* p, const or_cplx* U, const or_cplx* x4,
                      const or_cplx* b4, double tol_inner);
double or_true_residual(const or_params* p, const or_cplx* U, const or_cplx* x5, const or_cplx* b5);
int  or_num_threads(void);
/* OpenMP threads of later calls (CPU-baseline timing only; no arithmetic) */
void or_set_num_threads(int n);

#endif
