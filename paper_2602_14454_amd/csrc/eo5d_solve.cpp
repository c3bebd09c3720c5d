// Host side of the five-dimensional even-odd split (operator in eo5d.h):
// coefficients, the Schur operator D^5 and its adjoint, and the solve
//   b~_e = D_ee^-1 (b_e - D_eo D_oo^-1 b_o)
//   D^5 x_e = b~_e,  D^5 = 1 - D_ee^-1 D_eo D_oo^-1 D_oe   (CGNR on D^5^dag D^5)
//   x_o = D_oo^-1 (b_o - D_oe x_e)
// (Sec. 2.3, eq. even-odd_linear_equation and the two equations after it,
// with the sites split by their 5D parity).  The CG runs in FP64 or FP32
// inside FP64 defect correction, as the 4D-split solve does.
#include "eo5d.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <utility>

#include "blas.h"
#include "ops.h"
#include "precision.h"
#include "solver.h"

namespace dwf {

void eo5_coefficients(const dwf_op* op, double* h) {
    const int Ls = op->Ls;
    DWF_REQUIRE(!op->any_c(), DWF_EINVAL,
                "the 5D even-odd split needs c_s = 0 (for c != 0, D_- contains D_W and D_ee is not local)");
    DWF_REQUIRE(Ls >= 1 && Ls <= LS_MAX, DWF_EDIMS, "Ls out of range");
    // the mass term joins s = Ls-1 to s = 0; for odd Ls both have the same 5D parity
    DWF_REQUIRE(Ls % 2 == 0, DWF_EINVAL, "the 5D even-odd split needs an even Ls");
    std::memset(h, 0, sizeof(double) * EO5_NCOEF);
    for (int chi = 0; chi < 2; ++chi)
        for (int r = 0; r < Ls; ++r) {
            for (int q = 0; q < Ls; ++q) {
                const double kv = op->fd.K[chi][(size_t)r * Ls + q];
                DWF_REQUIRE(r == q || kv == 0.0, DWF_EINVAL, "the 5D even-odd split needs a diagonal K");
                const double mv = op->fd.M[chi][(size_t)r * Ls + q];
                const bool nb = q == (r + 1) % Ls || q == (r + Ls - 1) % Ls;
                DWF_REQUIRE(r == q || nb || mv == 0.0, DWF_EINVAL, "M couples slices beyond s -/+ 1");
                h[EO5_M + (chi * 16 + r) * 16 + q] = mv;
            }
            const double md = op->fd.M[chi][(size_t)r * Ls + r];
            DWF_REQUIRE(md != 0.0, DWF_EINVAL, "singular 5D-diagonal block");
            h[EO5_KD + chi * 16 + r] = op->fd.K[chi][(size_t)r * Ls + r];
            h[EO5_MINV + chi * 16 + r] = 1.0 / md;
        }
}

namespace {

void piece(const dwf_op* op, int kind, int par, int dagger, int pre, int post_hop, int post_loc, double a,
           double sgn, void* out, const void* in, const void* loc, const double* coef, hipStream_t st) {
    const dwf_lattice* L = op->lat;
    Eo5Params P{};
    P.out = out;
    P.in = in;
    P.loc = loc;
    const int cb = (int)complex_bytes_of(kind);
    P.links = L->links[kind].p;
    P.lpar = link_elems_parity(L->Vhp, cb);
    P.nbr = L->nbr.as<int>();
    P.coef = coef;
    P.Vh = L->Vh;
    P.Vhp = L->Vhp;
    P.Ls = op->Ls;
    P.par = par;
    P.dagger = dagger;
    P.pre = pre;
    P.post_hop = post_hop;
    P.post_loc = post_loc;
    P.a = a;
    P.sgn = sgn;
    launch_eo5(kind, P, st);
}

void read_back(const double* dev, Pinned& host, hipStream_t st) {
    DWF_HIP(hipMemcpyAsync(host.h, dev, CG_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
}

double norm2_of(int kind, const void* v, long n, double* partial, double* scal, Pinned& hs, hipStream_t st) {
    norm2_partial(kind, v, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_TMP, 0, st);
    read_back(scal, hs, st);
    return hs.h[CG_TMP];
}

// CG vectors of one storage kind, n complex numbers each (even half fields;
// `to` is an odd one)
struct Eo5Cg {
    int kp;
    long n;
    DevBuf x, r, p, q, w, to, rin;
    Eo5Cg(int kp_, long n_) : kp(kp_), n(n_) {
        const size_t b = complex_bytes_of(kp) * (size_t)n;
        for (DevBuf* d : {&x, &r, &p, &q, &w, &to, &rin}) d->alloc(b);
    }
};

// CG on D^5^dag D^5 y = D^5^dag b from y = 0 (b in W.rin), until
// |r| <= tol_rel |r0| or maxiter iterations; y in W.x
int cgnr5(const dwf_op* op, Eo5Cg& W, const double* coef, double tol_rel, int maxiter, int check_every,
          double* partial, double* scal, Pinned& hs, hipStream_t st, double* final_rel, bool* nan_seen) {
    const int kp = W.kp;
    const long n = W.n;
    if (check_every < 1) check_every = 1;
    DWF_HIP(hipMemsetAsync(scal, 0, CG_NSLOTS * sizeof(double), st));
    eo5_dhat(op, kp, 1, W.r.p, W.rin.p, W.to.p, coef, st);
    DWF_HIP(hipMemsetAsync(W.x.p, 0, complex_bytes_of(kp) * (size_t)n, st));
    DWF_HIP(hipMemcpyAsync(W.p.p, W.r.p, complex_bytes_of(kp) * (size_t)n, hipMemcpyDeviceToDevice, st));
    norm2_partial(kp, W.r.p, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_RR, 0, st);
    read_back(scal, hs, st);
    const double rr0 = hs.h[CG_RR];
    *nan_seen = !std::isfinite(rr0);
    if (rr0 == 0.0 || *nan_seen) {
        *final_rel = 0.0;
        return 0;
    }
    const double stop = tol_rel * tol_rel * rr0;
    double rr = rr0;
    int k = 0;
    while (k < maxiter) {
        eo5_dhat(op, kp, 0, W.q.p, W.p.p, W.to.p, coef, st);              // q = D^5 p
        norm2_partial(kp, W.q.p, n, partial, st);
        finalize(partial, blas_grid(n), 1, scal, 1, st);                   // alpha = rr / |q|^2
        eo5_dhat(op, kp, 1, W.w.p, W.q.p, W.to.p, coef, st);              // w = D^5^dag q
        cg_update_xr(kp, kp, W.x.p, W.r.p, W.p.p, W.w.p, n, scal + CG_ALPHA, partial, st);
        finalize(partial, blas_grid(n), 1, scal, 2, st);                   // beta, |r|^2
        cg_update_p(kp, kp, W.p.p, W.r.p, n, scal + CG_BETA, st);
        ++k;
        if (k % check_every == 0 || k == maxiter) {
            read_back(scal, hs, st);
            rr = hs.h[CG_RR];
            if (hs.h[CG_NANFLAG] != 0.0 || !std::isfinite(rr)) {
                *nan_seen = true;
                break;
            }
            if (rr <= stop) break;
        }
    }
    *final_rel = std::sqrt(rr / rr0);
    return k;
}

}  // namespace

void eo5_dhat(const dwf_op* op, int kind, int dagger, void* out_e, const void* in_e, void* tmp_o,
              const double* coef, hipStream_t st) {
    if (!dagger) {
        // tmp = D_oo^-1 D_oe in;  out = in - D_ee^-1 D_eo tmp
        piece(op, kind, 1, 0, 0, 1, 0, 0.0, 1.0, tmp_o, in_e, nullptr, coef, st);
        piece(op, kind, 0, 0, 0, 1, 0, 1.0, -1.0, out_e, tmp_o, in_e, coef, st);
    } else {
        // D^5^dag = 1 - (D_oe^dag D_oo^-1)(D_eo^dag D_ee^-1):
        // tmp = (D^dag)_oe D_ee^-1 in;  out = in - (D^dag)_eo D_oo^-1 tmp
        piece(op, kind, 1, 1, 1, 0, 0, 0.0, 1.0, tmp_o, in_e, nullptr, coef, st);
        piece(op, kind, 0, 1, 1, 0, 0, 1.0, -1.0, out_e, tmp_o, in_e, coef, st);
    }
}

void apply_eo5_schur(const dwf_op* op, int kind, int dagger, void* out5, const void* in5, hipStream_t st) {
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    DWF_REQUIRE(kind == ST_F64 || kind == ST_F32, DWF_EINVAL, "the 5D even-odd split runs in FP64 or FP32");
    double hc[EO5_NCOEF];
    eo5_coefficients(op, hc);
    DevBuf coef(sizeof hc);
    DWF_HIP(hipMemcpyAsync(coef.p, hc, sizeof hc, hipMemcpyHostToDevice, st));
    const long n = (long)op->Ls * L->Vh * 12;
    const int* lex = L->lex_of_site_dev.as<int>();
    DevBuf e64(16 * n), ek(complex_bytes_of(kind) * n), ok(complex_bytes_of(kind) * n), tk(complex_bytes_of(kind) * n);
    eo5_pack(e64.p, in5, lex, L->Vh, L->V, op->Ls, 0, st);
    eo5_convert(kind, ST_F64, ek.p, e64.p, n, st);
    eo5_dhat(op, kind, dagger, ok.p, ek.p, tk.p, coef.as<double>(), st);
    eo5_convert(ST_F64, kind, e64.p, ok.p, n, st);
    DWF_HIP(hipMemsetAsync(out5, 0, (size_t)op->Ls * L->V * 12 * 16, st));
    eo5_unpack(out5, e64.p, lex, L->Vh, L->V, op->Ls, 0, st);
    DWF_HIP(hipStreamSynchronize(st));
}

int solve_eo5(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm, dwf_solve_info* info,
              hipStream_t st) {
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    const long Vh = L->Vh, V = L->V;
    const int Ls = op->Ls;
    const long n = (long)Ls * Vh * 12;
    int kp = ST_F64;
    if (prm->algo == DWF_ALGO_DC || prm->paper_mode) kp = prm->inner_prec;
    DWF_REQUIRE(kp == ST_F64 || kp == ST_F32, DWF_EINVAL, "the 5D even-odd split runs its CG in FP64 or FP32");
    double hc[EO5_NCOEF];
    eo5_coefficients(op, hc);

    std::lock_guard<std::mutex> lock(op->solve_mu);
    // workspace (this path is a measurement path: allocated per solve, before the timed region)
    DevBuf coef(sizeof hc), be(16 * n), bo(16 * n), bt(16 * n), xe(16 * n), xo(16 * n), rh(16 * n), te(16 * n),
        to(16 * n), partial((blas_grid(n) + 16) * sizeof(double)), scal(CG_NSLOTS * sizeof(double));
    Pinned hs(CG_NSLOTS);
    std::unique_ptr<Eo5Cg> cg[2];
    auto cg_of = [&](int k) -> Eo5Cg& {
        if (!cg[k]) cg[k].reset(new Eo5Cg(k, n));
        return *cg[k];
    };
    cg_of(kp);
    double* pp = partial.as<double>();
    double* sc = scal.as<double>();
    const double* cf = coef.as<double>();
    DWF_HIP(hipMemcpyAsync(coef.p, hc, sizeof hc, hipMemcpyHostToDevice, st));
    DWF_HIP(hipStreamSynchronize(st));

    hipEvent_t e0, e1;
    DWF_HIP(hipEventCreate(&e0));
    DWF_HIP(hipEventCreate(&e1));
    DWF_HIP(hipEventRecord(e0, st));
    const int* lex = L->lex_of_site_dev.as<int>();
    eo5_pack(be.p, b5, lex, Vh, V, Ls, 0, st);
    eo5_pack(bo.p, b5, lex, Vh, V, Ls, 1, st);
    const double b2 = norm2_of(ST_F64, be.p, n, pp, sc, hs, st) + norm2_of(ST_F64, bo.p, n, pp, sc, hs, st);
    // b~_e = D_ee^-1 b_e - D_ee^-1 D_eo D_oo^-1 b_o
    piece(op, ST_F64, 0, 0, 1, 1, 1, 1.0, -1.0, bt.p, bo.p, be.p, cf, st);

    const double tol = prm->tol > 0 ? prm->tol : 1e-10;
    const int maxiter = prm->maxiter > 0 ? prm->maxiter : 100000;
    double inner_tol = prm->inner_tol;
    if (inner_tol <= 0) inner_tol = kp == ST_F64 ? tol : 1e-5;
    if (prm->paper_mode) inner_tol = 1e-7;   // |r|^2 / |r0|^2 < 1e-14

    int total = 0, outer = 0, fallback = 0;
    bool converged = false, nan_seen = false;
    double rel5 = 1.0, last_inner_rel = 0.0, prev_rel = 1e300, f_ratio = 1.0;
    DWF_HIP(hipMemsetAsync(xe.p, 0, 16 * (size_t)n, st));
    DWF_HIP(hipMemcpyAsync(rh.p, bt.p, 16 * (size_t)n, hipMemcpyDeviceToDevice, st));
    if (b2 == 0.0) {
        converged = true;
        rel5 = 0.0;
    }
    while (!converged && total < maxiter && outer < 100) {
        Eo5Cg& W = cg_of(kp);
        eo5_convert(kp, ST_F64, W.rin.p, rh.p, n, st);
        const bool plain = prm->paper_mode || (kp == ST_F64 && outer == 0);
        const double itol = plain ? inner_tol : dc_target(tol, rel5, kp, inner_tol, f_ratio);
        const int it = cgnr5(op, W, cf, itol, maxiter - total, prm->check_every, pp, sc, hs, st, &last_inner_rel,
                             &nan_seen);
        total += it;
        ++outer;
        if (nan_seen) break;
        eo5_convert(ST_F64, kp, te.p, W.x.p, n, st);
        axpby(ST_F64, ST_F64, xe.p, te.p, n, nullptr, 1.0, nullptr, 1.0, nullptr, st);
        // r^ = b~ - D^5 x_e (FP64); the 5D residual is (D_ee r^, 0) after reconstruction
        eo5_dhat(op, ST_F64, 0, te.p, xe.p, to.p, cf, st);
        axpby(ST_F64, ST_F64, te.p, bt.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
        std::swap(rh, te);
        eo5_diag(te.p, rh.p, cf, Vh, Ls, st);
        const double rel5_old = rel5;
        rel5 = b2 > 0 ? std::sqrt(norm2_of(ST_F64, te.p, n, pp, sc, hs, st) / b2) : 0.0;
        f_ratio = dc_ratio(rel5 / rel5_old, itol);
        if (trace_on())
            std::fprintf(stderr, "dwf trace: eo5 solve step %d prec %d requested %.3e iters %d rel5 %.3e\n", outer,
                         kp, itol, it, rel5);
        if (prm->paper_mode) break;
        if (rel5 <= tol) {
            converged = true;
            break;
        }
        if (rel5 > 0.5 * prev_rel && kp != ST_F64) {
            kp = ST_F64;   // stagnation of the correction: step up to FP64
            fallback = 1;
        }
        prev_rel = rel5;
    }
    // x_o = D_oo^-1 b_o - D_oo^-1 D_oe x_e
    piece(op, ST_F64, 1, 0, 0, 1, 1, 1.0, -1.0, xo.p, xe.p, bo.p, cf, st);
    eo5_unpack(x5, xe.p, lex, Vh, V, Ls, 0, st);
    eo5_unpack(x5, xo.p, lex, Vh, V, Ls, 1, st);
    DWF_HIP(hipEventRecord(e1, st));
    DWF_HIP(hipEventSynchronize(e1));
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
    DWF_HIP(hipEventDestroy(e0));
    DWF_HIP(hipEventDestroy(e1));
    // final FP64 true residual of the 5D system (outside the timed region)
    const double true_res = true_residual(op, x5, b5, st);
    const bool paper_ok = prm->paper_mode && !nan_seen && last_inner_rel <= inner_tol;
    if (info) {
        info->iters = total;
        info->outer_iters = outer;
        info->fallback_used = fallback;
        info->converged = (converged || paper_ok) ? 1 : 0;
        info->true_res5 = true_res;
        info->seconds = ms * 1e-3;
        info->final_rel_res_even = last_inner_rel;
        info->final_inner_prec = kp;
    }
    if (nan_seen) throw Error{DWF_ENAN, "NaN/Inf in a CG reduction"};
    if (prm->paper_mode) return paper_ok ? DWF_OK : DWF_NOT_CONVERGED;
    return (converged || true_res <= tol) ? DWF_OK : DWF_NOT_CONVERGED;
}

}  // namespace dwf
