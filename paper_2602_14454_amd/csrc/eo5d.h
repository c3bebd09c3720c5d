// Even-odd preconditioning in five dimensions (eo5d.hip, eo5d_solve.cpp).
//
// Sec. 2.3 notes that the sites can be split into even and odd either in
// four dimensions (the solver's split) or in five.  With the 5D parity
// (x + y + z + t + s) mod 2, both the 4D hop (fixed s) and the shift in s
// (fixed x) connect opposite parities, and for c_s = 0 (K = B T diagonal)
// every remaining term is diagonal in (site, s, chirality) provided Ls is
// even (the mass term joins s = Ls-1 and s = 0, of equal parity for odd Ls):
//   D_PP   = diag_s M_ss                       (M = (4 - M0) K + N)
//   D_P,P' = -1/2 H K + (M - diag M)           (P' = 1 - P)
// so that the Schur operator D^5 = 1 - D_ee^-1 D_eo D_oo^-1 D_oe of
// eq. even-odd_linear_equation needs no dense fifth-dimension algebra.
//
// Half fields of 5D parity P: slice s holds the 4D sites of parity
// (P + s) mod 2 in the lattice's internal site order, component-major
// [s][spin * 3 + colour][site] (Vh sites per row, consecutive lanes read
// consecutive sites).  The 4D neighbours of such a site at
// slice s, and the same site at slices s -/+ 1, are then entries of the
// opposite half field at the indices of the 4D tables.
#pragma once

#include <hip/hip_runtime.h>

#include "dwf_internal.h"

namespace dwf {

// Coefficients of one operator on the device (doubles): K_ss and 1 / M_ss
// per chirality (2 x 16 each), then M (2 x 16 x 16), zero padded.
constexpr int EO5_KD = 0, EO5_MINV = 32, EO5_M = 64, EO5_NCOEF = 64 + 2 * 16 * 16;

struct Eo5Params {
    void* out;
    const void* in;
    const void* loc;        // nullptr: no local term
    const void* links;      // the lattice's hop links of this storage kind (both output parities)
    const int* nbr;         // [2][8][Vhp]
    const double* coef;     // EO5_NCOEF doubles
    long Vh, Vhp, lpar;     // lpar: complex link elements of one output parity
    int Ls, par;            // par: 5D parity of the output
    int dagger;             // 0: D_{P,P'}; 1: (D^dag)_{P,P'} = (D_{P',P})^dag
    int pre;                // input scaled by 1 / M_ss of its slice first
    int post_hop, post_loc; // the hop result / the local term scaled by 1 / M_ss of the output slice
    double a, sgn;          // out = a [post_loc] loc + sgn [post_hop] (hop result)
};

// out = a loc + sgn D_{P,P'} in with the scalings of Eo5Params (kind F64 or F32).
void launch_eo5(int kind, const Eo5Params& P, hipStream_t st);
// canonical 5D (FP64, [s][lex][12]) <-> FP64 half field of 5D parity par
void eo5_pack(void* half, const void* full5, const int* lex_of_site, long Vh, long V, int Ls, int par,
              hipStream_t st);
void eo5_unpack(void* full5, const void* half, const int* lex_of_site, long Vh, long V, int Ls, int par,
                hipStream_t st);
// elementwise FP64 <-> FP32 copy of n complex numbers (kinds ST_F64 / ST_F32)
void eo5_convert(int kd, int ks, void* dst, const void* src, long n, hipStream_t st);
// out = M_ss(chirality) in over one FP64 half field (the 5D-diagonal block)
void eo5_diag(void* out, const void* in, const double* coef, long Vh, int Ls, hipStream_t st);

// host side (eo5d_solve.cpp)
// FP64 coefficients of op; throws DWF_EINVAL unless every c_s is 0 and Ls is even
void eo5_coefficients(const dwf_op* op, double* h /* EO5_NCOEF */);
// D^5 (dagger 0) or D^5^dag on even half fields of storage `kind`; tmp_o is an odd half field
void eo5_dhat(const dwf_op* op, int kind, int dagger, void* out_e, const void* in_e, void* tmp_o,
              const double* coef, hipStream_t st);
// x5 = D^-1 b5 through the 5D split (dwf_solve with schur = 2)
int solve_eo5(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm, dwf_solve_info* info,
              hipStream_t st);
// out5 = D^5 in5 (or its adjoint) on the 5D-even entries of canonical 5D fields;
// the 5D-odd entries of out5 are set to zero
void apply_eo5_schur(const dwf_op* op, int kind, int dagger, void* out5, const void* in5, hipStream_t st);

}  // namespace dwf
