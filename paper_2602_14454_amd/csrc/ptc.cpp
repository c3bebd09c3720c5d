// Learned preconditioner: model object, forward, training step, training
// pairs and checkpoint files.  The network (ptc_kernels.hip) is linear:
//   M r = PTC_2(PTC_1(r)),  PTC_1: 1 -> H channels (even input, hidden on
//   both parities),  PTC_2: H -> 1 channel (even output).
// Training minimises |M r - e|^2 / |e|^2 over pairs (r_k = A e_k, e_k =
// x* - x_k) taken from CGNR runs on D^dag D^, with Adam; forward, backward
// and the update all run in the kernels of ptc_kernels.hip.
#include "ptc_model.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <vector>

#include "blas.h"
#include "ops.h"
#include "precision.h"
#include "ptc.h"
#include "solver.h"

using namespace dwf;

namespace dwf {

static const float2* links32(const dwf_op* op, int parity) {
    const dwf_lattice* L = op->lat;
    return static_cast<const float2*>(L->links[ST_F32].p) + (size_t)parity * link_elems_parity(L->Vhp, 8);
}
static const int* nbr_of(const dwf_op* op, int parity) {
    return op->lat->nbr.as<int>() + (size_t)parity * 8 * op->lat->Vhp;
}

static PtcLayerParams layer_params(const dwf_op* op, int parity, const float2* in_loc, const float2* in_hop,
                                   float2* out, const float2* W, int A, int B) {
    PtcLayerParams P{};
    P.in_loc = in_loc;
    P.in_hop = in_hop;
    P.out = out;
    P.W = W;
    P.links = links32(op, parity);
    P.nbr = nbr_of(op, parity);
    P.Vh = op->lat->Vh;
    P.Vhp = op->lat->Vhp;
    P.Ls = op->Ls;
    P.A = A;
    P.B = B;
    P.accumulate = 0;
    return P;
}

long ptc_field_elems(const dwf_op* op) { return (long)op->Ls * 12 * op->lat->Vhp; }

}  // namespace dwf

// ---------------------------------------------------------------------
dwf_ptc::dwf_ptc(int hidden) : H(hidden) {
    nw = 2L * 11 * H * 16;
    W.alloc(nw * sizeof(float2));
    G.alloc(nw * sizeof(float2));
    Wt.alloc((size_t)11 * H * 16 * sizeof(float2));
    m.alloc(2 * nw * sizeof(float));
    v.alloc(2 * nw * sizeof(float));
    stats.alloc(8 * sizeof(double));
    // weight-gradient rows (path, b, first a)
    std::vector<int> r2, r1e, r1o;
    for (int q = 0; q < 11; ++q)
        for (int b = 0; b < H; ++b) r2.insert(r2.end(), {q, b, 0});
    const int ac = ptc_wgrad_ac(H);
    for (int q : {0, 9, 10})
        for (int a = 0; a < H; a += ac) r1e.insert(r1e.end(), {q, 0, a});
    for (int q = 1; q <= 8; ++q)
        for (int a = 0; a < H; a += ac) r1o.insert(r1o.end(), {q, 0, a});
    n2 = (int)r2.size() / 3;
    n1e = (int)r1e.size() / 3;
    n1o = (int)r1o.size() / 3;
    rows.alloc((r2.size() + r1e.size() + r1o.size()) * sizeof(int));
    int* rp = rows.as<int>();
    DWF_HIP(hipMemcpy(rp, r2.data(), r2.size() * sizeof(int), hipMemcpyHostToDevice));
    DWF_HIP(hipMemcpy(rp + r2.size(), r1e.data(), r1e.size() * sizeof(int), hipMemcpyHostToDevice));
    DWF_HIP(hipMemcpy(rp + r2.size() + r1e.size(), r1o.data(), r1o.size() * sizeof(int), hipMemcpyHostToDevice));
}

const float2* dwf_ptc::W1() const { return W.as<float2>(); }
const float2* dwf_ptc::W2() const { return W.as<float2>() + 11L * H * 16; }

void dwf_ptc::reserve(const dwf_op* op) {
    const long n = ptc_field_elems(op);
    if (n > cap_n) {
        he.alloc((size_t)H * n * sizeof(float2));
        ho.alloc((size_t)H * n * sizeof(float2));
        ghe.alloc((size_t)H * n * sizeof(float2));
        gho.alloc((size_t)H * n * sizeof(float2));
        y.alloc(n * sizeof(float2));
        g.alloc(n * sizeof(float2));
        lpartial.alloc(2 * (size_t)ptc_loss_blocks(n) * sizeof(double));
        d.alloc(n * sizeof(float2));
        u.alloc(n * sizeof(float2));
        w.alloc(n * sizeof(float2));
        to.alloc(n * sizeof(float2));
        tv.alloc(n * sizeof(float2));
        cap_n = n;
    }
    PtcLayerParams P = layer_params(op, 0, nullptr, nullptr, nullptr, nullptr, 1, H);
    const size_t need = (size_t)std::max(n2, std::max(n1e, n1o)) * ptc_wgrad_blocks(P) * 64 * sizeof(float);
    if (need > wpart.bytes) wpart.alloc(need);
}

void dwf_ptc::forward(const dwf_op* op, const float2* r, float2* out, hipStream_t st) {
    reserve(op);
    ptc_layer(layer_params(op, 0, r, nullptr, he.as<float2>(), W1(), H, 1), st);
    ptc_layer(layer_params(op, 1, nullptr, r, ho.as<float2>(), W1(), H, 1), st);
    ptc_layer(layer_params(op, 0, he.as<float2>(), ho.as<float2>(), out, W2(), 1, H), st);
}

// Loss of one pair and its gradient with respect to the output y = M r:
//   kind 0:  L = |y - e|^2 / |e|^2,          dL/dy = 2 (y - e) / |e|^2
//   kind 1:  L = |A (y - e)|^2 / |r|^2,      dL/dy = 2 A^2 (y - e) / |r|^2
// (A = D^dag D^ Hermitian; with r = A e the second is |A M r - r|^2 / |r|^2,
// the residual left by the right-preconditioned operator).
void dwf_ptc::loss(const dwf_op* op, const float2* r, const float2* e, bool value_only, hipStream_t st) {
    reserve(op);
    const long n = ptc_field_elems(op);
    forward(op, r, y.as<float2>(), st);
    if (loss_kind == 0) {
        ptc_loss(y.as<float2>(), e, n, lpartial.as<double>(), stats.as<double>(), value_only ? nullptr : g.as<float2>(),
                 st);
        return;
    }
    ptc_sub(y.as<float2>(), e, n, d.as<float2>(), st);
    apply_normal(op, ST_F32, u.p, d.p, to.p, tv.p, nullptr, 1, st);
    ptc_norms(u.as<float2>(), r, n, lpartial.as<double>(), stats.as<double>(), st);
    if (value_only) return;
    apply_normal(op, ST_F32, w.p, u.p, to.p, tv.p, nullptr, 1, st);
    ptc_scale_grad(w.as<float2>(), n, stats.as<double>(), g.as<float2>(), st);
}

void dwf_ptc::gradient(const dwf_op* op, const float2* r, const float2* e, hipStream_t st) {
    loss(op, r, e, false, st);
    DWF_HIP(hipMemsetAsync(G.p, 0, nw * sizeof(float2), st));
    float2* G1 = G.as<float2>();
    float2* G2 = G.as<float2>() + 11L * H * 16;
    const int* rp = rows.as<int>();
    float* wp = wpart.as<float>();
    // layer 2: dL/dW2 from (he, ho) and g
    ptc_wgrad(layer_params(op, 0, he.as<float2>(), ho.as<float2>(), nullptr, W2(), 1, H), g.as<float2>(), rp, n2, wp,
              G2, st);
    // hidden gradients through the adjoint layer
    ptc_adjoint(W2(), Wt.as<float2>(), 1, H, st);
    ptc_layer(layer_params(op, 0, g.as<float2>(), nullptr, ghe.as<float2>(), Wt.as<float2>(), H, 1), st);
    ptc_layer(layer_params(op, 1, nullptr, g.as<float2>(), gho.as<float2>(), Wt.as<float2>(), H, 1), st);
    // layer 1: even outputs (paths 0, +-s), odd outputs (link paths)
    ptc_wgrad(layer_params(op, 0, r, nullptr, nullptr, W1(), H, 1), ghe.as<float2>(), rp + 3 * n2, n1e, wp, G1, st);
    ptc_wgrad(layer_params(op, 1, nullptr, r, nullptr, W1(), H, 1), gho.as<float2>(), rp + 3 * (n2 + n1e), n1o, wp,
              G1, st);
}

void dwf_ptc::train_step(const dwf_op* op, const float2* r, const float2* e, double lr, hipStream_t st) {
    gradient(op, r, e, st);
    ++step;
    ptc_adam(W.as<float>(), G.as<float>(), m.as<float>(), v.as<float>(), (int)(2 * nw), (float)lr, 0.9f, 0.999f,
             1e-8f, step, st);
}

// ---------------------------------------------------------------------
namespace dwf {

static uint64_t splitmix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

dwf_ptc* ptc_create(int hidden, unsigned long long seed, double scale) {
    DWF_REQUIRE(hidden >= 1 && hidden <= 64, DWF_EINVAL, "hidden channels must be 1..64");
    std::unique_ptr<dwf_ptc> M(new dwf_ptc(hidden));
    // identity on path 0 / channel 0 plus seeded Gaussian noise of width scale
    std::vector<float> w(2 * M->nw);
    for (long k = 0; k < 2 * M->nw; k += 2) {
        const uint64_t z1 = splitmix(seed * 0x100000001B3ull + (uint64_t)k);
        const uint64_t z2 = splitmix(z1 ^ 0xD1B54A32D192ED03ull);
        const double u1 = ((z1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
        const double u2 = (z2 >> 11) * (1.0 / 9007199254740992.0);
        const double rad = std::sqrt(-2.0 * std::log(u1)) * scale / std::sqrt(2.0);
        w[k] = (float)(rad * std::cos(6.283185307179586 * u2));
        w[k + 1] = (float)(rad * std::sin(6.283185307179586 * u2));
    }
    const long half = 11L * hidden * 16;   // complex weights per layer
    for (int i = 0; i < 4; ++i) {
        w[2 * (i * 4 + i)] += 1.0f;              // W1[0][0][0] = I + noise
        w[2 * (half + i * 4 + i)] += 1.0f;       // W2[0][0][0] = I + noise
    }
    DWF_HIP(hipMemcpy(M->W.p, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice));
    return M.release();
}

dwf_ptc_pairs* ptc_pairs_create(const dwf_op* op, const void* b5, unsigned long long seed, int nsnap,
                                const int* snaps, hipStream_t st) {
    DWF_REQUIRE(op && nsnap >= 1 && nsnap <= 256 && snaps, DWF_EINVAL, "bad pair request");
    const dwf_lattice* L = op->lat;
    DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
    for (int i = 0; i < nsnap; ++i) DWF_REQUIRE(snaps[i] >= 0, DWF_EINVAL, "snapshot iterations must be >= 0");
    const long n = ptc_field_elems(op);
    const size_t b64 = 16 * (size_t)n;
    DevBuf be(b64), bo(b64), bt(b64), to(b64), xs(b64), tmp(b64);
    const int* lex = L->lex_of_site_dev.as<int>();
    bool nan_seen = false;
    double fr = 0;
    if (b5) {
        // the Schur system of the 5D source; x* to 1e-10 (FP64 CGNR)
        pack_full(ST_F64, be.p, b5, lex, L->Vh, L->Vhp, L->V, op->Ls, st);
        pack_full(ST_F64, bo.p, b5, lex + L->Vh, L->Vh, L->Vhp, L->V, op->Ls, st);
        schur_rhs(op, ST_F64, bt.p, be.p, bo.p, to.p, 1, st);
        CgWork W(op, ST_F64, ST_F64, 1);
        cgnr(op, W, bt.p, 1e-10, 100000, 8, st, &fr, &nan_seen, nullptr);
        DWF_REQUIRE(!nan_seen, DWF_ENAN, "NaN while solving for training pairs");
        convert(ST_F64, ST_F64, xs.p, W.x.p, n, st);
    } else {
        // a system with known solution: x* = seeded random field, b~ = D^ x*
        random_fill_f64(xs.p, (long)op->Ls * 12, L->Vh, L->Vhp, seed, st);
        apply_dhat(op, ST_F64, 0, bt.p, xs.p, to.p, nullptr, 1, st);
    }
    std::unique_ptr<dwf_ptc_pairs> P(new dwf_ptc_pairs);
    P->op = op;
    P->n = n;
    P->count = nsnap;
    P->r.alloc((size_t)nsnap * n * sizeof(float2));
    P->e.alloc((size_t)nsnap * n * sizeof(float2));
    // replay CGNR and keep e_k = x* - x_k at the requested iterations, r_k = A e_k
    int maxk = 0;
    for (int i = 0; i < nsnap; ++i) maxk = std::max(maxk, snaps[i]);
    CgWork W2(op, ST_F64, ST_F64, 1);
    DevBuf t1(8 * (size_t)n), t2(8 * (size_t)n);
    auto take = [&](int k, const void* xk) {
        for (int i = 0; i < nsnap; ++i) {
            if (snaps[i] != k) continue;
            float2* e = P->e.as<float2>() + (size_t)i * n;
            float2* r = P->r.as<float2>() + (size_t)i * n;
            convert(ST_F64, ST_F64, tmp.p, xs.p, n, st);
            axpby(ST_F64, ST_F64, tmp.p, xk, n, nullptr, -1.0, nullptr, 1.0, nullptr, st);
            convert(ST_F32, ST_F64, e, tmp.p, n, st, L->Vhp);
            apply_normal(op, ST_F32, r, e, t1.p, t2.p, nullptr, 1, st);
        }
    };
    {
        // iteration 0: x_0 = 0
        DevBuf zero(b64);
        take(0, zero.p);
    }
    if (maxk > 0) cgnr(op, W2, bt.p, 0.0, maxk, maxk, st, &fr, &nan_seen, take);
    DWF_HIP(hipStreamSynchronize(st));
    return P.release();
}

void ptc_train(dwf_ptc* M, int nsets, dwf_ptc_pairs* const* sets, int steps, double lr, unsigned long long seed,
               double* hist, hipStream_t st) {
    DWF_REQUIRE(M && nsets >= 1 && sets && steps >= 0 && lr > 0, DWF_EINVAL, "bad training request");
    for (int i = 0; i < nsets; ++i) DWF_REQUIRE(sets[i] && sets[i]->count >= 1, DWF_EINVAL, "empty pair set");
    DevBuf dh((size_t)std::max(steps, 1) * sizeof(double));
    for (int k = 0; k < steps; ++k) {
        const uint64_t z = splitmix(seed ^ splitmix((uint64_t)k + 1));
        const dwf_ptc_pairs* S = sets[z % (uint64_t)nsets];
        const int j = (int)((z >> 32) % (uint64_t)S->count);
        M->train_step(S->op, S->r.as<float2>() + (size_t)j * S->n, S->e.as<float2>() + (size_t)j * S->n, lr, st);
        DWF_HIP(hipMemcpyAsync(dh.as<double>() + k, M->stats.p, sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    if (hist && steps > 0)
        DWF_HIP(hipMemcpyAsync(hist, dh.p, (size_t)steps * sizeof(double), hipMemcpyDeviceToHost, st));
    DWF_HIP(hipStreamSynchronize(st));
}

double ptc_eval(dwf_ptc* M, int nsets, dwf_ptc_pairs* const* sets, hipStream_t st) {
    double sum = 0;
    int cnt = 0;
    double h = 0;
    for (int i = 0; i < nsets; ++i) {
        const dwf_ptc_pairs* S = sets[i];
        M->reserve(S->op);
        for (int j = 0; j < S->count; ++j) {
            M->loss(S->op, S->r.as<float2>() + (size_t)j * S->n, S->e.as<float2>() + (size_t)j * S->n, true, st);
            DWF_HIP(hipMemcpyAsync(&h, M->stats.p, sizeof(double), hipMemcpyDeviceToHost, st));
            DWF_HIP(hipStreamSynchronize(st));
            sum += h;
            ++cnt;
        }
    }
    return cnt ? sum / cnt : 0.0;
}

// checkpoint: "DWFPTC01", int32 H, int32 step, int64 nw, W (2 nw float),
// m, v (2 nw float each), uint64 FNV-1a of everything before it
static uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}

void ptc_save(const dwf_ptc* M, const char* path) {
    DWF_REQUIRE(M && path, DWF_EINVAL, "null argument");
    std::vector<unsigned char> buf(8 + 4 + 4 + 8);
    std::memcpy(buf.data(), "DWFPTC01", 8);
    const int32_t H = M->H, step = M->step;
    const int64_t nw = M->nw;
    std::memcpy(buf.data() + 8, &H, 4);
    std::memcpy(buf.data() + 12, &step, 4);
    std::memcpy(buf.data() + 16, &nw, 8);
    const size_t fb = 2 * (size_t)nw * sizeof(float);
    const size_t off = buf.size();
    buf.resize(off + 3 * fb);
    DWF_HIP(hipMemcpy(buf.data() + off, M->W.p, fb, hipMemcpyDeviceToHost));
    DWF_HIP(hipMemcpy(buf.data() + off + fb, M->m.p, fb, hipMemcpyDeviceToHost));
    DWF_HIP(hipMemcpy(buf.data() + off + 2 * fb, M->v.p, fb, hipMemcpyDeviceToHost));
    const uint64_t h = fnv1a(buf.data(), buf.size());
    FILE* f = std::fopen(path, "wb");
    DWF_REQUIRE(f, DWF_EINVAL, std::string("cannot open ") + path);
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size() && std::fwrite(&h, 8, 1, f) == 1;
    std::fclose(f);
    DWF_REQUIRE(ok, DWF_EINVAL, std::string("write failed: ") + path);
}

dwf_ptc* ptc_load(const char* path) {
    DWF_REQUIRE(path, DWF_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    DWF_REQUIRE(f, DWF_EINVAL, std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char tmp[65536];
    size_t got;
    while ((got = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    std::fclose(f);
    DWF_REQUIRE(buf.size() >= 32 && std::memcmp(buf.data(), "DWFPTC01", 8) == 0, DWF_EINVAL, "not a PTC checkpoint");
    int32_t H, step;
    int64_t nw;
    std::memcpy(&H, buf.data() + 8, 4);
    std::memcpy(&step, buf.data() + 12, 4);
    std::memcpy(&nw, buf.data() + 16, 8);
    DWF_REQUIRE(H >= 1 && H <= 64 && nw == 2L * 11 * H * 16, DWF_EINVAL, "corrupt PTC checkpoint header");
    const size_t fb = 2 * (size_t)nw * sizeof(float);
    DWF_REQUIRE(buf.size() == 24 + 3 * fb + 8, DWF_EINVAL, "PTC checkpoint has the wrong size");
    uint64_t h;
    std::memcpy(&h, buf.data() + 24 + 3 * fb, 8);
    DWF_REQUIRE(h == fnv1a(buf.data(), 24 + 3 * fb), DWF_EINVAL, "PTC checkpoint checksum mismatch");
    std::unique_ptr<dwf_ptc> M(new dwf_ptc(H));
    M->step = step;
    DWF_HIP(hipMemcpy(M->W.p, buf.data() + 24, fb, hipMemcpyHostToDevice));
    DWF_HIP(hipMemcpy(M->m.p, buf.data() + 24 + fb, fb, hipMemcpyHostToDevice));
    DWF_HIP(hipMemcpy(M->v.p, buf.data() + 24 + 2 * fb, fb, hipMemcpyHostToDevice));
    return M.release();
}

}  // namespace dwf
