// Operator applications on internal half fields (ops.cpp).  All field
// pointers are device buffers of StoreKind `kind` in the internal layout;
// nrhs fields are stored back to back.
#pragma once

#include <complex>

#include "dwf_internal.h"
#include "hop.h"

namespace dwf {

inline size_t complex_bytes_of(int kind) { return kind == ST_F64 ? 16 : kind == ST_F32 ? 8 : 4; }

// Parameters of one fused hop (see hop.h) without launching it.
HopParams hop_params(const dwf_op* op, int kind, int out_parity, const void* in, const void* loc, void* out,
                     int pre_slot, int post_slot, int locmix_slot, double loc_scale, void* out2, int post2_slot,
                     int locmix2_slot, double* partial, int reduce, int Ls_override = 0);
// Generic fused hop; see hop.h.  *_slot < 0 means "not used".
void hop(const dwf_op* op, int kind, int out_parity, const void* in, const void* loc, void* out,
         int pre_slot, int post_slot, int locmix_slot, double loc_scale, void* out2, int post2_slot,
         int locmix2_slot, double* partial, int reduce, int nrhs, hipStream_t st, int Ls_override = 0,
         int bench_tag = 0);
void mix(const dwf_op* op, int kind, const void* in, void* out, int slot, double* partial, int nrhs,
         hipStream_t st);
int hop_partials(const dwf_op* op, int nrhs);
int mix_partials(const dwf_op* op, int nrhs);

void apply_dhat(const dwf_op* op, int kind, int dagger, void* out_e, const void* in_e, void* tmp_o,
                void* tmp_e, int nrhs, hipStream_t st);
void apply_normal(const dwf_op* op, int kind, void* out_e, const void* in_e, void* tmp_o, void* tmp_v,
                  double* qq_partial, int nrhs, hipStream_t st);
// One CGNR step's operator work with the residual update fused into the last
// hop: alpha = rr / |D^ p|^2 (scal[CG_QQ], scal[CG_ALPHA]), then
// r -= alpha D^dag D^ p with partial |r|^2 per hop block in `partial`
// (hop_partials(op, nrhs) of them).  r holds the compute type (FP64 for
// kind FP64, FP32 otherwise); D^dag D^ p itself is not stored.
// alpha_copy (or nullptr) also receives alpha.
void apply_normal_update_r(const dwf_op* op, int kind, void* r, const void* p, void* tmp_o, void* tmp_v,
                           double* partial, double* scal, int nrhs, hipStream_t st, double* alpha_copy = nullptr);
void apply_full(const dwf_op* op, int kind, int dagger, void* out_e, void* out_o, const void* in_e,
                const void* in_o, int nrhs, hipStream_t st);
void schur_rhs(const dwf_op* op, int kind, void* bt_e, const void* b_e, const void* b_o, void* tmp_o,
               int nrhs, hipStream_t st);
void reconstruct_odd(const dwf_op* op, int kind, void* x_o, const void* x_e, const void* b_o, int nrhs,
                     hipStream_t st);
void source_pair(const dwf_op* op, void* out_pair_p, const void* pair_other, const void* pair_p, int parity,
                 hipStream_t st);

// objects.cpp
void build_geometry(dwf_lattice* L);
void upload_gauge(dwf_lattice* L, const std::complex<double>* U);
void setup_op(dwf_op* op);

}  // namespace dwf
