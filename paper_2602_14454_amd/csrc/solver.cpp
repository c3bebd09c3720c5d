// Solvers for D^(alpha) x5 = b5 through the even-odd Schur system
// (Sec. 2.3): CG on D^dag D^ (CGNR), and FP64 defect correction around a
// CGNR in FP32 or BF16 storage (the paper's single-precision solver used as
// the preconditioner of a double-precision solve, Sec. 2.3).
//
// CG scalars stay on the device (finalize kernels compute alpha and beta from
// the FP64 partial sums); the host reads them back every `check_every`
// iterations to test convergence.
#include "eo5d.h"
#include "solver.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <memory>
#include <utility>

#include "blas.h"
#include "fgcr.h"
#include "ops.h"
#include "ptc_model.h"

namespace dwf {

Pinned::Pinned(size_t n) {
    if (hipHostMalloc(reinterpret_cast<void**>(&h), n * sizeof(double), hipHostMallocDefault) != hipSuccess)
        throw Error{DWF_ENOMEM, "hipHostMalloc failed"};
    std::memset(h, 0, n * sizeof(double));
}
Pinned::~Pinned() {
    if (h) (void)hipHostFree(h);
}

int ring_slots(size_t slot_bytes) {
    const size_t cap = size_t(8) << 30;
    const size_t fit = slot_bytes > 0 ? cap / slot_bytes : 16;
    return (int)std::max<size_t>(2, std::min<size_t>(16, fit));
}

static void read_scalars(const double* dev, Pinned& host, hipStream_t st) {
    DWF_HIP(hipMemcpyAsync(host.h, dev, CG_NSLOTS * sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
}

CgWork::CgWork(const dwf_op* op, int kx_, int kp_, int nrhs_) : kx(kx_), kp(kp_), nrhs(nrhs_), hs(CG_NSLOTS) {
    n = (long)op->Ls * 12 * op->lat->Vhp * nrhs;
    const size_t bx = complex_bytes_of(kx) * n, bp = complex_bytes_of(kp) * n;
    x.alloc(bx);
    r.alloc(bx);
    t.alloc(bp);   // p: on first use by a solve without the direction ring
    v.alloc(bp);
    w.alloc(bp);
    const long np = std::max<long>(hop_partials(op, nrhs), blas_grid(n)) * 2 + 16;
    partial.alloc(np * sizeof(double));
    scal.alloc(CG_NSLOTS * sizeof(double));
}

// Iterations from check k (|r|^2 = rr; the previous check at k0 read rr0)
// until the next host convergence check: `every`, or fewer when the decrease
// since k0, taken as geometric, predicts that |r|^2 reaches `stop` sooner.  It
// only brings a check forward, so a solve never runs more iterations past its
// target than with the fixed period.
static int next_check_gap(int k, double rr, int k0, double rr0, double stop, int every) {
    if (every <= 1 || k <= k0 || !(rr > stop) || !(rr0 > rr)) return every;
    const double per_iter = std::log(rr / rr0) / (double)(k - k0);   // < 0
    const double todo = std::log(stop / rr) / per_iter;                // > 0
    if (!(todo > 0.0)) return every;
    return (int)std::max(1.0, std::min((double)every, std::ceil(todo)));
}

int cgnr(const dwf_op* op, CgWork& W, const void* b_kp, double tol_rel, int maxiter, int check_every,
         hipStream_t st, double* final_rel, bool* nan_seen, const IterHook& on_iter, bool predict_checks) {
    const long n = W.n;
    double* partial = W.partial.as<double>();
    double* scal = W.scal.as<double>();
    Pinned& hs = W.hs;
    if (check_every < 1) check_every = 1;
    DWF_HIP(hipMemsetAsync(W.scal.p, 0, CG_NSLOTS * sizeof(double), st));
    // p lives in a ring of W.ring_len slots unless the caller wants x after
    // every iteration (on_iter)
    const bool ring = !on_iter;
    const long Vhp = op->lat->Vhp;
    const size_t pbytes = complex_bytes_of(W.kp) * (size_t)n;
    if (ring && !W.ring.p) {
        W.ring_len = ring_slots(pbytes);
        W.ring.alloc(pbytes * W.ring_len);
        W.alphas.alloc(sizeof(double) * W.ring_len);
    }
    if (!ring && !W.p.p) W.p.alloc(pbytes);
    auto slot = [&](int i) -> void* { return static_cast<char*>(W.ring.p) + (size_t)i * pbytes; };
    // r = D^dag b, p = r, x = 0
    apply_dhat(op, W.kp, 1, W.w.p, b_kp, W.t.p, W.v.p, W.nrhs, st);
    convert(W.kx, W.kp, W.r.p, W.w.p, n, st, Vhp);
    convert(W.kp, W.kx, ring ? slot(0) : W.p.p, W.r.p, n, st, Vhp);
    DWF_HIP(hipMemsetAsync(W.x.p, 0, complex_bytes_of(W.kx) * n, st));
    norm2_partial(W.kx, W.r.p, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_RR, 0, st);
    read_scalars(scal, hs, st);
    const double rr0 = hs.h[CG_RR];
    *nan_seen = !std::isfinite(rr0);
    if (rr0 == 0.0 || *nan_seen) {
        if (final_rel) *final_rel = 0.0;
        return 0;
    }
    const double stop = tol_rel * tol_rel * rr0;
    int k = 0;
    double rr = rr0;
    int cur = 0, pend = 0;   // ring slot of p_k; slots [0, pend) hold directions not yet in x
    double* alphas = W.alphas.as<double>();
    int next_check = check_every, k_prev = 0;
    double rr_prev = rr0;
    while (k < maxiter) {
        // alpha, then r -= alpha D^dag D^ p inside the last hop (|r|^2 partials)
        void* pk = ring ? slot(cur) : W.p.p;
        apply_normal_update_r(op, W.kp, W.r.p, pk, W.t.p, W.v.p, partial, scal, W.nrhs, st,
                              ring ? alphas + cur : nullptr);
        finalize(partial, hop_partials(op, W.nrhs), 1, scal, 2, st);
        if (ring) {
            // p_{k+1} = r + beta p_k into the next slot; a full ring is folded
            // into x first (x += alpha_i p_i in order, as the per-iteration update)
            ++pend;
            int nxt = cur + 1;
            if (nxt == W.ring_len) {
                cg_accumulate_x(W.kx, W.kp, W.x.p, W.ring.p, alphas, pend, n, st, Vhp);
                pend = 0;
                nxt = 0;
            }
            cg_update_p2(W.kx, W.kp, slot(nxt), pk, W.r.p, n, scal + CG_BETA, st, Vhp);
            cur = nxt;
        } else {
            // the x update rides on the p update, which reads p anyway
            cg_update_px(W.kx, W.kp, W.x.p, W.p.p, W.r.p, n, scal + CG_ALPHA, scal + CG_BETA, st, Vhp);
        }
        ++k;
        if (on_iter) on_iter(k, W.x.p);
        if (k == next_check || k == maxiter) {
            read_scalars(scal, hs, st);
            rr = hs.h[CG_RR];
            if (hs.h[CG_NANFLAG] != 0.0 || !std::isfinite(rr)) {
                *nan_seen = true;
                break;
            }
            if (rr <= stop) break;
            next_check = k + (predict_checks ? next_check_gap(k, rr, k_prev, rr_prev, stop, check_every) : check_every);
            k_prev = k;
            rr_prev = rr;
        }
    }
    if (ring) cg_accumulate_x(W.kx, W.kp, W.x.p, W.ring.p, alphas, pend, n, st, Vhp);
    if (final_rel) *final_rel = std::sqrt(rr / rr0);
    return k;
}

// CG on the normal equations of the right-preconditioned Schur operator
// (Sec. 2.3, eq. another_even-odd_linear_equation)
//   D_R = 1 - D_eo D_oo^-1 D_oe D_ee^-1 = M D^ M^-1   (D_ee = D_oo = M),
// D_R^dag = M^-T D^dag M^T (M real per chirality), composed from the local
// mixes and the D^ hops: D_R^dag D_R y = D_R^dag b from y = 0, same
// stopping rule as cgnr; y in W.x.  The alpha factors of the Neff form cancel
// in D_R (D^(alpha) = D T with T 5D-local), so its iterations do not depend on
// alpha.  This path measures that claim; the fused left form is the solver.
static int cgnr_right(const dwf_op* op, CgWork& W, const void* b_kp, double tol_rel, int maxiter, int check_every,
                      hipStream_t st, double* final_rel, bool* nan_seen) {
    const long n = W.n;
    const long Vhp = op->lat->Vhp;
    double* partial = W.partial.as<double>();
    double* scal = W.scal.as<double>();
    Pinned& hs = W.hs;
    if (check_every < 1) check_every = 1;
    const size_t pbytes = complex_bytes_of(W.kp) * (size_t)n;
    if (!W.p.p) W.p.alloc(pbytes);
    if (!W.ra.p) W.ra.alloc(pbytes);
    if (!W.rb.p) W.rb.alloc(pbytes);
    void *ra = W.ra.p, *rb = W.rb.p;
    auto apply_rdag = [&](void* out, const void* in) {   // out = M^-T D^dag M^T in
        mix(op, W.kp, in, rb, MAT_MT, nullptr, 1, st);
        apply_dhat(op, W.kp, 1, ra, rb, W.t.p, W.v.p, 1, st);
        mix(op, W.kp, ra, out, MAT_MIT, nullptr, 1, st);
    };
    DWF_HIP(hipMemsetAsync(W.scal.p, 0, CG_NSLOTS * sizeof(double), st));
    apply_rdag(W.w.p, b_kp);
    convert(W.kx, W.kp, W.r.p, W.w.p, n, st, Vhp);
    convert(W.kp, W.kx, W.p.p, W.r.p, n, st, Vhp);
    DWF_HIP(hipMemsetAsync(W.x.p, 0, complex_bytes_of(W.kx) * n, st));
    norm2_partial(W.kx, W.r.p, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_RR, 0, st);
    read_scalars(scal, hs, st);
    const double rr0 = hs.h[CG_RR];
    *nan_seen = !std::isfinite(rr0);
    if (rr0 == 0.0 || *nan_seen) {
        if (final_rel) *final_rel = 0.0;
        return 0;
    }
    const double stop = tol_rel * tol_rel * rr0;
    double rr = rr0;
    int k = 0;
    while (k < maxiter) {
        // q = D_R p = M D^ M^-1 p, alpha = rr / |q|^2
        mix(op, W.kp, W.p.p, ra, MAT_MINV, nullptr, 1, st);
        apply_dhat(op, W.kp, 0, rb, ra, W.t.p, W.v.p, 1, st);
        mix(op, W.kp, rb, W.w.p, MAT_M, partial, 1, st);
        finalize(partial, mix_partials(op, 1), 1, scal, 1, st);
        // w = D_R^dag q; x += alpha p, r -= alpha w
        mix(op, W.kp, W.w.p, rb, MAT_MT, nullptr, 1, st);
        apply_dhat(op, W.kp, 1, ra, rb, W.t.p, W.v.p, 1, st);
        mix(op, W.kp, ra, W.w.p, MAT_MIT, nullptr, 1, st);
        cg_update_xr(W.kx, W.kp, W.x.p, W.r.p, W.p.p, W.w.p, n, scal + CG_ALPHA, partial, st, Vhp);
        finalize(partial, blas_grid(n), 1, scal, 2, st);
        cg_update_p(W.kx, W.kp, W.p.p, W.r.p, n, scal + CG_BETA, st, Vhp);
        ++k;
        if (k % check_every == 0 || k == maxiter) {
            read_scalars(scal, hs, st);
            rr = hs.h[CG_RR];
            if (hs.h[CG_NANFLAG] != 0.0 || !std::isfinite(rr)) {
                *nan_seen = true;
                break;
            }
            if (rr <= stop) break;
        }
    }
    if (final_rel) *final_rel = std::sqrt(rr / rr0);
    return k;
}

// |v|^2 of a half field (device reduction, host result)
static double norm2_host(int kind, const void* v, long n, double* partial, double* scal, Pinned& hs,
                         hipStream_t st) {
    norm2_partial(kind, v, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_TMP, 0, st);
    read_scalars(scal, hs, st);
    return hs.h[CG_TMP];
}

// Mixed-precision CGNR with reliable updates (Sleijpen and van der Vorst).
// The CG iteration runs with x_lo, r_lo in FP32 storage and p, w and the hop
// temporaries in the low storage precision (FP32 or BF16).  Whenever the
// low-precision residual has dropped by `delta` since the last update, the
// partial solution is folded into the FP64 solution x_hi, the FP64 Schur
// residual r^ = b~ - D^ x_hi and the normal residual D^dag r^ are recomputed,
// and the CG continues with that residual and its old search direction.  The
// Krylov space is kept (unlike a restart), so the iteration count stays close
// to the FP64 one while all operator applications but the updates are cheap.
// Each update also gives the exact 5D residual |M r^| / |b5| (odd rows
// vanish after reconstruction), which is the stopping test.
static int cgnr_reliable(const dwf_op* op, CgWork& W, void* xe, const void* bt, void* rh, void* te, void* to,
                         void* tmp_e, double b2, double tol, double delta, int maxiter, int check_every,
                         double* pp, double* sc, Pinned& hs, hipStream_t st, int* nupdates, double* rel5_out,
                         bool* nan_seen) {
    const long n = W.n;
    double* partial = W.partial.as<double>();
    double* scal = W.scal.as<double>();
    if (check_every < 1) check_every = 1;
    *nupdates = 0;
    *nan_seen = false;
    if (!W.p.p) W.p.alloc(complex_bytes_of(W.kp) * (size_t)n);
    DWF_HIP(hipMemsetAsync(W.scal.p, 0, CG_NSLOTS * sizeof(double), st));
    // r^ = b~ (x_hi = 0), r = D^dag r^
    convert(ST_F64, ST_F64, rh, bt, n, st);
    apply_dhat(op, ST_F64, 1, te, rh, to, tmp_e, 1, st);
    convert(W.kx, ST_F64, W.r.p, te, n, st, op->lat->Vhp);
    convert(W.kp, W.kx, W.p.p, W.r.p, n, st, op->lat->Vhp);
    DWF_HIP(hipMemsetAsync(W.x.p, 0, complex_bytes_of(W.kx) * n, st));
    norm2_partial(W.kx, W.r.p, n, partial, st);
    finalize(partial, blas_grid(n), 1, scal + CG_RR, 0, st);
    read_scalars(scal, hs, st);
    const double rr0 = hs.h[CG_RR];
    if (!std::isfinite(rr0)) { *nan_seen = true; return 0; }
    if (rr0 == 0.0) { *rel5_out = 0.0; return 0; }
    double rmax2 = rr0;
    double target = tol * tol * rr0;
    double rel5 = 1.0;
    int k = 0;
    while (k < maxiter) {
        apply_normal(op, W.kp, W.w.p, W.p.p, W.t.p, W.v.p, partial, W.nrhs, st);
        finalize(partial, hop_partials(op, W.nrhs), 1, scal, 1, st);
        cg_update_xr(W.kx, W.kp, W.x.p, W.r.p, W.p.p, W.w.p, n, scal + CG_ALPHA, partial, st, op->lat->Vhp);
        finalize(partial, blas_grid(n), 1, scal, 2, st);
        ++k;
        if (k % check_every == 0 || k == maxiter) {
            read_scalars(scal, hs, st);
            const double rr = hs.h[CG_RR];
            if (hs.h[CG_NANFLAG] != 0.0 || !std::isfinite(rr)) { *nan_seen = true; break; }
            if (rr < delta * delta * rmax2 || rr < target || k == maxiter) {
                // reliable update: fold x_lo into x_hi and recompute the residual in FP64
                axpby(ST_F64, W.kx, xe, W.x.p, n, nullptr, 1.0, nullptr, 1.0, nullptr, st, op->lat->Vhp);
                DWF_HIP(hipMemsetAsync(W.x.p, 0, complex_bytes_of(W.kx) * n, st));
                apply_dhat(op, ST_F64, 0, te, xe, to, tmp_e, 1, st);
                convert(ST_F64, ST_F64, rh, bt, n, st);
                axpby(ST_F64, ST_F64, rh, te, n, nullptr, -1.0, nullptr, 1.0, nullptr, st);
                mix(op, ST_F64, rh, te, MAT_M, nullptr, 1, st);
                rel5 = std::sqrt(norm2_host(ST_F64, te, n, pp, sc, hs, st) / b2);
                ++*nupdates;
                if (rel5 <= tol || k == maxiter) break;
                apply_dhat(op, ST_F64, 1, te, rh, to, tmp_e, 1, st);
                convert(W.kx, ST_F64, W.r.p, te, n, st, op->lat->Vhp);
                norm2_partial(W.kx, W.r.p, n, partial, st);
                finalize(partial, blas_grid(n), 1, scal, 3, st);
                read_scalars(scal, hs, st);
                const double rr_true = hs.h[CG_RR];
                if (rr < target) {
                    // the recursive residual met the normal-equation target but the
                    // 5D residual did not: tighten the target by the observed gap
                    const double f = tol / rel5;
                    target = rr_true * f * f * 0.25;
                }
                rmax2 = rr_true;
            } else {
                rmax2 = std::max(rmax2, rr);
            }
        }
        cg_update_p(W.kx, W.kp, W.p.p, W.r.p, n, scal + CG_BETA, st, op->lat->Vhp);
    }
    if (*nan_seen) return k;
    *rel5_out = rel5;
    return k;
}

bool trace_on() {
    static const bool on = std::getenv("DWF_TRACE") != nullptr;
    return on;
}

// Inner target of one defect-correction step.  The CG stops on its normal
// residual |D^dag r^|, but the outer test is on the 5D residual |M r^|; their
// reductions differ by a factor f measured on the previous step of the same
// solve.  The step that can reach tol asks for the normal-residual reduction
// that brings the 5D residual to tol/2; a step that cannot (the reduction
// would be below what the inner precision resolves) takes the precision's
// standard reduction.  FP64 restarts of plain CGNR use the same rule.
double dc_target(double tol, double rel5, int kp, double standard, double f, bool* last) {
    const double floor = kp == ST_F64 ? 1e-15 : (kp == ST_F32 ? 1e-6 : 1e-2);
    const double need = 0.5 * tol / std::max(rel5, 1e-300);
    const double want = need >= floor ? need : standard;
    if (last) *last = need >= floor;
    return std::min(0.5, std::max(1e-13, want / f));
}

double dc_ratio(double achieved, double requested) {
    if (!(achieved > 0.0) || !(requested > 0.0)) return 1.0;
    return std::min(1e4, std::max(1e-2, achieved / requested));
}

namespace {
// Workspace of dwf_solve, kept by the operator between solves: allocation and
// release of ~10 full-size vectors per solve cost milliseconds of host time.
// Every buffer keeps one layout (rh and te, both FP64 half fields, trade
// roles between outer steps), so its zero padding (never written by a
// kernel) stays valid; a solve that ends in an error drops the workspace.
struct SolveWs {
    long n = 0;
    DevBuf be, bo, bt, xe, xo, rh, te, to, rin, partial, scal;
    Pinned hs{CG_NSLOTS};
    std::unique_ptr<CgWork> cg[3];   // by inner storage kind
};

SolveWs& solve_ws(const dwf_op* op, long n) {
    auto ws = std::static_pointer_cast<SolveWs>(op->solve_ws);
    if (!ws || ws->n != n) {
        op->solve_ws.reset();   // release the old workspace first
        ws = std::make_shared<SolveWs>();
        const size_t b64 = 16 * (size_t)n;
        for (DevBuf* b : {&ws->be, &ws->bo, &ws->bt, &ws->xe, &ws->xo, &ws->rh, &ws->te, &ws->to, &ws->rin})
            b->alloc(b64);
        ws->partial.alloc((std::max<long>(hop_partials(op, 1), blas_grid(n)) * 2 + 16) * sizeof(double));
        ws->scal.alloc(CG_NSLOTS * sizeof(double));
        ws->n = n;
        op->solve_ws = ws;
    }
    return *ws;
}

CgWork& solve_cg(SolveWs& ws, const dwf_op* op, int kp) {
    if (!ws.cg[kp]) ws.cg[kp].reset(new CgWork(op, kp == ST_F64 ? ST_F64 : ST_F32, kp, 1));
    return *ws.cg[kp];
}

struct DropOnError {
    const dwf_op* op;
    bool ok = false;
    ~DropOnError() {
        if (!ok) op->solve_ws.reset();
    }
};
}  // namespace

int solve(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm, dwf_solve_info* info,
          hipStream_t st) {
    if (prm->schur == 2) return solve_eo5(op, x5, b5, prm, info, st);   // the 5D split (eo5d_solve.cpp)
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    const long Vh = L->Vh, Vhp = L->Vhp, V = L->V;
    const int Ls = op->Ls;
    const long n = (long)Ls * 12 * Vhp;
    const size_t b64 = 16 * n;

    int kp = ST_F64;
    if (prm->algo == DWF_ALGO_DC || prm->algo == DWF_ALGO_MIXED || prm->paper_mode) kp = prm->inner_prec;
    if (prm->algo == DWF_ALGO_FGCR_LEARNED) kp = ST_F32;   // FGCR and the network run in FP32
    DWF_REQUIRE(kp == ST_F64 || kp == ST_F32 || kp == ST_BF16, DWF_EINVAL, "bad inner precision");

    // all workspace exists before the timed region starts
    std::lock_guard<std::mutex> lock(op->solve_mu);
    DropOnError guard{op};
    SolveWs& ws = solve_ws(op, n);
    DevBuf &be = ws.be, &bo = ws.bo, &bt = ws.bt, &xe = ws.xe, &xo = ws.xo, &rh = ws.rh, &te = ws.te, &to = ws.to;
    DevBuf& rin = ws.rin;
    Pinned& hs = ws.hs;
    double* pp = ws.partial.as<double>();
    double* sc = ws.scal.as<double>();
    DevBuf& scal = ws.scal;
    CgWork* W = &solve_cg(ws, op, kp);

    hipEvent_t e0, e1;
    DWF_HIP(hipEventCreate(&e0));
    DWF_HIP(hipEventCreate(&e1));
    DWF_HIP(hipEventRecord(e0, st));
    DWF_HIP(hipMemsetAsync(scal.p, 0, CG_NSLOTS * sizeof(double), st));

    const int* lex = L->lex_of_site_dev.as<int>();
    pack_full(ST_F64, be.p, b5, lex, Vh, Vhp, V, Ls, st);
    pack_full(ST_F64, bo.p, b5, lex + Vh, Vh, Vhp, V, Ls, st);
    const double b2 = norm2_host(ST_F64, be.p, n, pp, sc, hs, st) + norm2_host(ST_F64, bo.p, n, pp, sc, hs, st);
    schur_rhs(op, ST_F64, bt.p, be.p, bo.p, to.p, 1, st);

    const double tol = prm->tol > 0 ? prm->tol : 1e-10;
    const int maxiter = prm->maxiter > 0 ? prm->maxiter : 100000;
    double inner_tol = prm->inner_tol;
    if (inner_tol <= 0) inner_tol = kp == ST_F64 ? tol : (kp == ST_F32 ? 1e-5 : 3e-2);
    if (prm->paper_mode) inner_tol = 1e-7;   // |r|^2 / |r0|^2 < 1e-14

    int total = 0, outer = 0, fallback = 0;
    bool converged = false, nan_seen = false;
    double rel5 = 1.0, last_inner_rel = 0.0;
    DWF_HIP(hipMemsetAsync(xe.p, 0, b64, st));
    convert(ST_F64, ST_F64, rh.p, bt.p, n, st);
    if (b2 == 0.0) {
        converged = true;
        rel5 = 0.0;
    }
    double prev_rel = 1e300;
    double f_ratio = 1.0;
    if (prm->algo == DWF_ALGO_MIXED && !converged) {
        const double delta = prm->inner_tol > 0 ? prm->inner_tol : (kp == ST_BF16 ? 0.25 : 0.1);
        int nup = 0;
        double r5 = 1.0;
        total = cgnr_reliable(op, *W, xe.p, bt.p, rh.p, te.p, to.p, xo.p, b2, tol, delta, maxiter,
                              prm->check_every, pp, sc, hs, st, &nup, &r5, &nan_seen);
        outer = nup;
        rel5 = r5;
        converged = !nan_seen && r5 <= tol;
    }
    const bool right_schur = prm->schur == 1;
    // flexible GCR with the learned preconditioner as the inner solver (FP32);
    // on failure (NaN, stagnation) the solve falls back to CGNR
    bool use_fgcr = prm->algo == DWF_ALGO_FGCR_LEARNED;
    std::unique_ptr<FgcrWork> FW;
    if (use_fgcr) FW.reset(new FgcrWork(op, prm->restart > 0 ? prm->restart : 16));
    while (prm->algo != DWF_ALGO_MIXED && !converged && total < maxiter && outer < 100) {
        const int kx = kp == ST_F64 ? ST_F64 : ST_F32;
        if (W->kp != kp) W = &solve_cg(ws, op, kp);
        convert(kp, ST_F64, rin.p, rh.p, n, st, Vhp);
        // FP64: the first step is the textbook CGNR stop; restarts are calibrated
        const bool plain = prm->paper_mode || (kp == ST_F64 && outer == 0);
        bool last_step = false;
        const double itol = plain ? inner_tol : dc_target(tol, rel5, kp, inner_tol, f_ratio, &last_step);
        int it = 0;
        const void* xin = nullptr;
        if (use_fgcr) {
            bool failed = false;
            it = fgcr(op, static_cast<dwf_ptc*>(prm->ptc_model), *FW, rin.p, itol, maxiter - total, prm->check_every,
                      st, &last_inner_rel, &failed);
            total += it;
            if (failed) {
                // the learned step is discarded; CGNR takes over from the current x
                use_fgcr = false;
                fallback = 1;
                if (trace_on()) std::fprintf(stderr, "dwf trace: FGCR failed after %d iterations, CGNR fallback\n", it);
                continue;
            }
            xin = FW->x.p;
        } else if (right_schur) {
            // the right system for the current residual: D_R y = M r^, then x_e += M^-1 y
            mix(op, ST_F64, rh.p, te.p, MAT_M, nullptr, 1, st);
            convert(kp, ST_F64, rin.p, te.p, n, st, Vhp);
            it = cgnr_right(op, *W, rin.p, itol, maxiter - total, prm->check_every, st, &last_inner_rel, &nan_seen);
            total += it;
            convert(ST_F64, kx, te.p, W->x.p, n, st, Vhp);
            mix(op, ST_F64, te.p, to.p, MAT_MINV, nullptr, 1, st);
            xin = to.p;
        } else {
            // The FP32 step meant to reach tol checks where its target is
            // predicted (iterations past it are waste); earlier steps keep the
            // fixed period, whose overshoot is progress that a later step
            // would otherwise have to make after a restart (predicted checks
            // in every FP32 step took one 16^3x32 point source 200 -> 220
            // iterations; in every CG loop, FP64 CGNR 360 -> 406 and DC-BF16
            // 416 -> 429 on 24^3x48).
            const bool predict = kp == ST_F32 && !prm->paper_mode && last_step;
            it = cgnr(op, *W, rin.p, itol, maxiter - total, prm->check_every, st, &last_inner_rel, &nan_seen,
                      IterHook(), predict);
            total += it;
            xin = W->x.p;
        }
        ++outer;
        if (nan_seen) break;
        axpby(ST_F64, right_schur ? ST_F64 : kx, xe.p, xin, n, nullptr, 1.0, nullptr, 1.0, nullptr, st, Vhp);
        // r^ = b~ - D^ xe (FP64), formed where D^ xe was written; the buffers
        // then trade names so that rh holds r^.  r5_e = -M r^ with |M r^|^2
        // reduced by the mix itself; r5_o = 0 exactly after reconstruction.
        apply_dhat(op, ST_F64, 0, te.p, xe.p, to.p, nullptr, 1, st);
        axpby(ST_F64, ST_F64, te.p, bt.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
        std::swap(rh, te);
        mix(op, ST_F64, rh.p, te.p, MAT_M, pp, 1, st);
        finalize(pp, mix_partials(op, 1), 1, sc + CG_TMP, 0, st);
        read_scalars(sc, hs, st);
        const double rel5_old = rel5;
        rel5 = std::sqrt(hs.h[CG_TMP] / b2);
        f_ratio = dc_ratio(rel5 / rel5_old, itol);
        if (trace_on())
            std::fprintf(stderr, "dwf trace: solve step %d prec %d requested %.3e iters %d rel5 %.3e\n", outer, kp,
                         itol, it, rel5);
        if (prm->paper_mode) break;
        if (rel5 <= tol) {
            converged = true;
            break;
        }
        if (rel5 > 0.5 * prev_rel && (use_fgcr || kp != ST_F64)) {
            // stagnation of the correction: leave FGCR for CGNR, else step up one precision
            if (use_fgcr) use_fgcr = false;
            else kp = kp == ST_BF16 ? ST_F32 : ST_F64;
            fallback = 1;
        }
        prev_rel = rel5;
    }
    reconstruct_odd(op, ST_F64, xo.p, xe.p, bo.p, 1, st);
    unpack_full(ST_F64, x5, xe.p, lex, Vh, Vhp, V, Ls, st);
    unpack_full(ST_F64, x5, xo.p, lex + Vh, Vh, Vhp, V, Ls, st);
    DWF_HIP(hipEventRecord(e1, st));
    // final FP64 true residual of the 5D system (outside the timed region)
    apply_full(op, ST_F64, 0, te.p, to.p, xe.p, xo.p, 1, st);
    axpby(ST_F64, ST_F64, te.p, be.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
    axpby(ST_F64, ST_F64, to.p, bo.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
    const double r2 = norm2_host(ST_F64, te.p, n, pp, sc, hs, st) + norm2_host(ST_F64, to.p, n, pp, sc, hs, st);
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
    DWF_HIP(hipEventDestroy(e0));
    DWF_HIP(hipEventDestroy(e1));
    const double true_res = b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
    // paper mode: converged only when the CG met its own stopping test
    // (|r|^2 / |r0|^2 < 1e-14), not when it ran out of iterations
    const bool paper_ok = prm->paper_mode && !nan_seen && last_inner_rel <= inner_tol;
    if (info) {
        info->iters = total;
        info->outer_iters = outer;
        info->fallback_used = fallback;
        info->converged = (converged || paper_ok) ? 1 : 0;
        info->true_res5 = true_res;
        info->seconds = ms * 1e-3;
        info->final_rel_res_even = last_inner_rel;
        info->final_inner_prec = use_fgcr ? ST_F32 : kp;
    }
    if (nan_seen) throw Error{DWF_ENAN, "NaN/Inf in a CG reduction"};
    guard.ok = true;
    if (prm->paper_mode) return paper_ok ? DWF_OK : DWF_NOT_CONVERGED;
    return (converged || true_res <= tol) ? DWF_OK : DWF_NOT_CONVERGED;
}

double true_residual(const dwf_op* op, const void* x5, const void* b5, hipStream_t st) {
    const dwf_lattice* L = op->lat;
    const long Vh = L->Vh, Vhp = L->Vhp, V = L->V;
    const int Ls = op->Ls;
    const long n = (long)Ls * 12 * Vhp;
    DevBuf xe(16 * n), xo(16 * n), be(16 * n), bo(16 * n), te(16 * n), to(16 * n);
    DevBuf partial((blas_grid(n) + 16) * sizeof(double)), scal(CG_NSLOTS * sizeof(double));
    Pinned hs(CG_NSLOTS);
    const int* lex = L->lex_of_site_dev.as<int>();
    pack_full(ST_F64, xe.p, x5, lex, Vh, Vhp, V, Ls, st);
    pack_full(ST_F64, xo.p, x5, lex + Vh, Vh, Vhp, V, Ls, st);
    pack_full(ST_F64, be.p, b5, lex, Vh, Vhp, V, Ls, st);
    pack_full(ST_F64, bo.p, b5, lex + Vh, Vh, Vhp, V, Ls, st);
    apply_full(op, ST_F64, 0, te.p, to.p, xe.p, xo.p, 1, st);
    double* pp = partial.as<double>();
    double* sc = scal.as<double>();
    const double b2 = norm2_host(ST_F64, be.p, n, pp, sc, hs, st) + norm2_host(ST_F64, bo.p, n, pp, sc, hs, st);
    axpby(ST_F64, ST_F64, te.p, be.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
    axpby(ST_F64, ST_F64, to.p, bo.p, n, nullptr, 1.0, nullptr, -1.0, nullptr, st);
    const double r2 = norm2_host(ST_F64, te.p, n, pp, sc, hs, st) + norm2_host(ST_F64, to.p, n, pp, sc, hs, st);
    return b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
}

// 4D residual of a projected solution (Sec. 2.3: the 4D solution is the
// same for every alpha).  With D_eff(m) y = [P^dag D(1)^-1 D(m) P (y,0,..,0)]_{s=1}
// (alpha = 1; the Pauli-Villars ratio of the domain-wall literature) the
// map G: b4 -> x4 satisfies (1 - m) G + 1 = D_eff^-1, hence
//   r4 = b4 - D_eff((1 - m) x4 + b4)
// vanishes for the exact x4.  Cost: one D(m) application and one well
// conditioned m = 1 solve (FP64 CGNR to tol_inner).
double residual_4d(const dwf_op* op, const void* x4, const void* b4, double tol_inner, hipStream_t st,
                   bool* converged) {
    dwf_lattice* L = op->lat;
    const long V = L->V, Vh = L->Vh, Vhp = L->Vhp;
    const int Ls = op->Ls;
    const long n4 = V * 12, n = (long)Ls * 12 * Vhp;
    dwf_op om, o1;
    om.lat = o1.lat = L;
    om.Ls = o1.Ls = Ls;
    om.M0 = o1.M0 = op->M0;
    om.b = o1.b = op->b;
    om.c = o1.c = op->c;   // b_s, c_s
    om.alpha = o1.alpha = 1.0;
    om.m = op->m;
    o1.m = 1.0;
    setup_op(&om);
    setup_op(&o1);
    DevBuf y(16 * n4), e5(16 * n4 * Ls), z5(16 * n4 * Ls), v5(16 * n4 * Ls), ie(16 * n), io(16 * n), oe(16 * n),
        oo(16 * n), partial((blas_grid(n4 * Ls) + 16) * sizeof(double)), scal(CG_NSLOTS * sizeof(double));
    Pinned hs(CG_NSLOTS);
    const int* lex = L->lex_of_site_dev.as<int>();
    convert(ST_F64, ST_F64, y.p, b4, n4, st);
    axpby(ST_F64, ST_F64, y.p, x4, n4, nullptr, 1.0 - op->m, nullptr, 1.0, nullptr, st);
    embed_4d(e5.p, y.p, V, Ls, st);
    pack_full(ST_F64, ie.p, e5.p, lex, Vh, Vhp, V, Ls, st);
    pack_full(ST_F64, io.p, e5.p, lex + Vh, Vh, Vhp, V, Ls, st);
    apply_full(&om, ST_F64, 0, oe.p, oo.p, ie.p, io.p, 1, st);
    unpack_full(ST_F64, z5.p, oe.p, lex, Vh, Vhp, V, Ls, st);
    unpack_full(ST_F64, z5.p, oo.p, lex + Vh, Vh, Vhp, V, Ls, st);
    dwf_solve_params prm;
    std::memset(&prm, 0, sizeof prm);
    prm.tol = tol_inner;
    prm.maxiter = 100000;
    prm.algo = DWF_ALGO_CGNR;
    prm.inner_prec = DWF_F64;
    prm.check_every = 4;
    if (converged) *converged = solve(&o1, v5.p, z5.p, &prm, nullptr, st) == DWF_OK;
    else solve(&o1, v5.p, z5.p, &prm, nullptr, st);
    project_4d(y.p, v5.p, V, Ls, st);
    axpby(ST_F64, ST_F64, y.p, b4, n4, nullptr, 1.0, nullptr, -1.0, nullptr, st);   // y = b4 - D_eff(...)
    double* pp = partial.as<double>();
    double* sc = scal.as<double>();
    const double r2 = norm2_host(ST_F64, y.p, n4, pp, sc, hs, st);
    const double b2 = norm2_host(ST_F64, b4, n4, pp, sc, hs, st);
    return b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
}

}  // namespace dwf
