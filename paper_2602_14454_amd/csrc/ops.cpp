// Operator applications composed from the fused hop (hop.hip).
//
// With D = M - (1/2) H K (fifth_dim.cpp) every operator of the solve is a
// short chain of fused hops:
//   D^ x     : t_o = Q H_oe K x;            out = (-1/4 Minv) H_eo t_o + x
//   D^dag x  : v = g5 Minv^T x;  t_o = Q^T H_oe v;  out = (-1/4 g5 K^T) H_eo t_o + x
//   normal   : as D^ then D^dag, with v = g5 Minv^T q produced directly by the
//              second hop (q is never stored; |q|^2 is reduced on the fly) and
//              q = g5 M^T v recovered in the last hop
//   D        : out_p = (-1/2) H K x_{1-p} + M x_p
//   D^dag    : out_p = (-1/2 K^T g5) H g5 x_{1-p} + M^T x_p
//   b~_e     : (1/2 Minv) H_eo (Q b_o) + Minv b_e              (Schur RHS)
//   x_o      : (1/2 Minv) H_oe K x_e + Minv b_o                 (reconstruction)
//   -D_- P^dag (0,..,b4): (c_s/2) H y + (1 - c_s(4 - M0)) y on the pair (P+ b4, P- b4),
//                       s = 1 and s = Ls
#include "ops.h"

#include "blas.h"
#include "hop.h"
#include "precision.h"

namespace dwf {

HopParams hop_params(const dwf_op* op, int kind, int out_parity, const void* in, const void* loc, void* out,
                     int pre_slot, int post_slot, int locmix_slot, double loc_scale, void* out2, int post2_slot,
                     int locmix2_slot, double* partial, int reduce, int Ls_override) {
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    HopParams P{};
    const long Vh = L->Vh, Vhp = L->Vhp;
    const size_t cb = complex_bytes_of(kind);
    P.in = in;
    P.loc = loc;
    P.out = out;
    P.out2 = out2;
    P.links = static_cast<const char*>(L->links[kind].p) + (size_t)out_parity * link_elems_parity(Vhp, (int)cb) * cb;
    P.nbr = L->nbr.as<int>() + (size_t)out_parity * 8 * Vhp;
    P.pre = pre_slot >= 0 ? op->pre(kind, pre_slot) : nullptr;
    P.pre_mode = pre_slot < 0 ? 0 : (pre_slot == PRE_K && op->any_c() ? 2 : 1);
    if (P.pre_mode == 1 && pre_slot == PRE_K) {
        // the kernel factors the upper-chirality diagonal out of the hop sum;
        // a zero entry takes the general pre-mix path instead
        for (int s = 0; s < op->Ls; ++s)
            if (op->fd.K[0][(size_t)s * op->Ls + s] == 0.0) P.pre_mode = 2;
    }
    P.post = op->mat(kind, post_slot);
    P.locmix = (loc && locmix_slot >= 0) ? op->mat(kind, locmix_slot) : nullptr;
    P.post2 = out2 ? op->mat(kind, post2_slot) : nullptr;
    P.locmix2 = (out2 && loc) ? op->mat(kind, locmix2_slot) : nullptr;
    P.partial = partial;
    P.reduce = reduce;
    P.Vh = Vh;
    P.Vhp = Vhp;
    P.Ls = Ls_override > 0 ? Ls_override : op->Ls;
    P.loc_scale = loc_scale;
    P.done = nullptr;
    P.done_stride = 0;
    P.pstride = hop_grid_blocks(Vh);
    // the kernels address one right-hand side with 32-bit byte offsets
    DWF_REQUIRE((double)P.Ls * 12.0 * (double)Vhp * (double)cb < 4294967296.0, DWF_EDIMS,
                "field too large for 32-bit in-kernel offsets");
    return P;
}

void hop(const dwf_op* op, int kind, int out_parity, const void* in, const void* loc, void* out,
         int pre_slot, int post_slot, int locmix_slot, double loc_scale, void* out2, int post2_slot,
         int locmix2_slot, double* partial, int reduce, int nrhs, hipStream_t st, int Ls_override,
         int bench_tag) {
    const HopParams P = hop_params(op, kind, out_parity, in, loc, out, pre_slot, post_slot, locmix_slot, loc_scale,
                                   out2, post2_slot, locmix2_slot, partial, reduce, Ls_override);
    launch_hop(kind, P, nrhs, st, bench_tag);
}

void mix(const dwf_op* op, int kind, const void* in, void* out, int slot, double* partial, int nrhs,
         hipStream_t st) {
    MixParams P{};
    P.in = in;
    P.out = out;
    P.mat = op->mat(kind, slot);
    P.partial = partial;
    P.Vh = op->lat->Vh;
    P.Vhp = op->lat->Vhp;
    P.Ls = op->Ls;
    launch_mix(kind, P, nrhs, st);
}

int hop_partials(const dwf_op* op, int nrhs) { return hop_grid_blocks(op->lat->Vh) * nrhs; }
int mix_partials(const dwf_op* op, int nrhs) { return mix_grid_blocks(op->lat->Vh) * nrhs; }

void apply_dhat(const dwf_op* op, int kind, int dagger, void* out_e, const void* in_e, void* tmp_o,
                void* tmp_e, int nrhs, hipStream_t st) {
    if (!dagger) {
        hop(op, kind, 1, in_e, nullptr, tmp_o, PRE_K, MAT_Q, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
        hop(op, kind, 0, tmp_o, in_e, out_e, -1, MAT_MQMINV, -1, 1.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    } else {
        mix(op, kind, in_e, tmp_e, MAT_G5MIT, nullptr, nrhs, st);
        hop(op, kind, 1, tmp_e, nullptr, tmp_o, -1, MAT_QT, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
        hop(op, kind, 0, tmp_o, in_e, out_e, -1, MAT_MQG5KT, -1, 1.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    }
}

void apply_normal(const dwf_op* op, int kind, void* out_e, const void* in_e, void* tmp_o, void* tmp_v,
                  double* qq_partial, int nrhs, hipStream_t st) {
    // t = Q H_oe K p
    hop(op, kind, 1, in_e, nullptr, tmp_o, PRE_K, MAT_Q, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    // q = (-1/4 Minv) H_eo t + p (not stored, |q|^2 reduced);  v = g5 Minv^T q
    {
        HopParams P = hop_params(op, kind, 0, tmp_o, in_e, nullptr, -1, MAT_MQMINV, -1, 1.0, tmp_v,
                                 DWF_CHAIN2 ? MAT_G5MIT : MAT_G5MIT_MQMINV, MAT_G5MIT, qq_partial, qq_partial ? 1 : 0);
        P.chain2 = DWF_CHAIN2;
        launch_hop(kind, P, nrhs, st);
    }
    // t = Q^T H_oe v
    hop(op, kind, 1, tmp_v, nullptr, tmp_o, -1, MAT_QT, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    // out = (-1/4 g5 K^T) H_eo t + g5 M^T v   (= D^dag q)
    hop(op, kind, 0, tmp_o, tmp_v, out_e, -1, MAT_MQG5KT, MAT_G5MT, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
}

void apply_normal_update_r(const dwf_op* op, int kind, void* r, const void* p, void* tmp_o, void* tmp_v,
                           double* partial, double* scal, int nrhs, hipStream_t st, double* alpha_copy) {
    hop(op, kind, 1, p, nullptr, tmp_o, PRE_K, MAT_Q, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    {
        HopParams P = hop_params(op, kind, 0, tmp_o, p, nullptr, -1, MAT_MQMINV, -1, 1.0, tmp_v,
                                 DWF_CHAIN2 ? MAT_G5MIT : MAT_G5MIT_MQMINV, MAT_G5MIT, partial, 1);
        P.chain2 = DWF_CHAIN2;
        launch_hop(kind, P, nrhs, st);
    }
    finalize(partial, hop_partials(op, nrhs), 1, scal, 1, st, alpha_copy);   // alpha
    hop(op, kind, 1, tmp_v, nullptr, tmp_o, -1, MAT_QT, -1, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    HopParams P = hop_params(op, kind, 0, tmp_o, tmp_v, nullptr, -1, MAT_MQG5KT, MAT_G5MT, 0.0, nullptr, 0, 0,
                             partial, 3);
    P.upd = r;
    P.upd_alpha = scal + CG_ALPHA;
    launch_hop(kind, P, nrhs, st);
}

void apply_full(const dwf_op* op, int kind, int dagger, void* out_e, void* out_o, const void* in_e,
                const void* in_o, int nrhs, hipStream_t st) {
    if (!dagger) {
        hop(op, kind, 0, in_o, in_e, out_e, PRE_K, MAT_MHALFI, MAT_M, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
        hop(op, kind, 1, in_e, in_o, out_o, PRE_K, MAT_MHALFI, MAT_M, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
    } else {
        hop(op, kind, 0, in_o, in_e, out_e, PRE_G5, MAT_MHALFKTG5, MAT_MT, 0.0, nullptr, 0, 0, nullptr, 0, nrhs,
            st);
        hop(op, kind, 1, in_e, in_o, out_o, PRE_G5, MAT_MHALFKTG5, MAT_MT, 0.0, nullptr, 0, 0, nullptr, 0, nrhs,
            st);
    }
}

void schur_rhs(const dwf_op* op, int kind, void* bt_e, const void* b_e, const void* b_o, void* tmp_o,
               int nrhs, hipStream_t st) {
    mix(op, kind, b_o, tmp_o, MAT_Q, nullptr, nrhs, st);
    hop(op, kind, 0, tmp_o, b_e, bt_e, -1, MAT_HALFMINV, MAT_MINV, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
}

void reconstruct_odd(const dwf_op* op, int kind, void* x_o, const void* x_e, const void* b_o, int nrhs,
                     hipStream_t st) {
    hop(op, kind, 1, x_e, b_o, x_o, PRE_K, MAT_HALFMINV, MAT_MINV, 0.0, nullptr, 0, 0, nullptr, 0, nrhs, st);
}

void source_pair(const dwf_op* op, void* out_pair_p, const void* pair_other, const void* pair_p, int parity,
                 hipStream_t st) {
    hop(op, ST_F64, parity, pair_other, pair_p, out_pair_p, -1, MAT_CHALF, MAT_SRCLOC, 0.0, nullptr, 0, 0, nullptr,
        0, 1, st, 2);
}

}  // namespace dwf
