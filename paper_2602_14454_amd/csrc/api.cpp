// extern "C" entry points of libdwf (declared in include/dwf.h).  Every call
// catches internal errors and turns them into status codes; the message is
// kept per thread for dwf_last_error().
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <string>
#include <new>
#include <vector>
#include <algorithm>

#include "blas.h"
#include "gauge.h"
#include "dwf_internal.h"
#include "hop.h"
#include "ops.h"
#include "eo5d.h"
#include "solver.h"
#include "ptc_model.h"

namespace dwf {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace dwf

using namespace dwf;

template <class F>
static int guarded(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return DWF_ENOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return DWF_EINVAL;
    }
}

static hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

extern "C" {

const char* dwf_status_string(int status) {
    switch (status) {
        case DWF_OK: return "ok";
        case DWF_NOT_CONVERGED: return "not converged";
        case DWF_EINVAL: return "invalid argument";
        case DWF_EDIMS: return "unsupported dimensions";
        case DWF_ENOMEM: return "out of memory";
        case DWF_EHIP: return "HIP runtime error";
        case DWF_ESTATE: return "object not ready";
        case DWF_ENAN: return "NaN or Inf in a reduction";
        default: return "unknown status";
    }
}

const char* dwf_last_error(void) { return g_last_error.c_str(); }

void dwf_solve_params_default(dwf_solve_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->tol = 1e-10;
    p->maxiter = 100000;
    p->algo = DWF_ALGO_CGNR;
    p->inner_prec = DWF_F32;
    p->inner_tol = 0.0;
    p->check_every = 1;
    p->paper_mode = 0;
    p->ptc_model = nullptr;
    p->restart = 16;
    p->autotune = 1;
    p->use_graph = 1;
}

int dwf_lattice_create(const int dims[4], int antiperiodic_t, dwf_lattice** out) {
    return guarded([&] {
        DWF_REQUIRE(dims && out, DWF_EINVAL, "null argument");
        for (int mu = 0; mu < 4; ++mu)
            DWF_REQUIRE(dims[mu] >= 2 && dims[mu] % 2 == 0, DWF_EDIMS, "every lattice extent must be even and >= 2");
        std::unique_ptr<dwf_lattice> L(new dwf_lattice());
        for (int mu = 0; mu < 4; ++mu) L->dims[mu] = dims[mu];
        L->antiperiodic_t = antiperiodic_t ? 1 : 0;
        L->V = (long)dims[0] * dims[1] * dims[2] * dims[3];
        DWF_REQUIRE(L->V < (1L << 30), DWF_EDIMS, "lattice volume too large for int32 site indices");
        L->Vh = L->V / 2;
        L->Vhp = L->Vh;
        build_geometry(L.get());
        *out = L.release();
        return DWF_OK;
    });
}

void dwf_lattice_destroy(dwf_lattice* lat) { delete lat; }

int dwf_lattice_set_gauge(dwf_lattice* lat, const void* U, int on_device, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(lat && U, DWF_EINVAL, "null argument");
        const size_t n = (size_t)lat->V * 4 * 9;
        std::vector<std::complex<double>> h(n);
        if (on_device) {
            DWF_HIP(hipMemcpyAsync(h.data(), U, n * 16, hipMemcpyDeviceToHost, S(stream)));
            DWF_HIP(hipStreamSynchronize(S(stream)));
        } else {
            std::memcpy(h.data(), U, n * 16);
        }
        upload_gauge(lat, h.data());
        return DWF_OK;
    });
}

int dwf_lattice_maps(const dwf_lattice* lat, int* lex_of_site, int* nbr) {
    return guarded([&] {
        DWF_REQUIRE(lat, DWF_EINVAL, "null lattice");
        // read back the device tables, so that what the kernels use is what is returned
        std::vector<int> lx(2 * lat->Vh), nb(2 * 8 * lat->Vhp);
        DWF_HIP(hipMemcpy(lx.data(), lat->lex_of_site_dev.p, lat->lex_of_site_dev.bytes, hipMemcpyDeviceToHost));
        DWF_HIP(hipMemcpy(nb.data(), lat->nbr.p, lat->nbr.bytes, hipMemcpyDeviceToHost));
        if (lex_of_site) std::memcpy(lex_of_site, lx.data(), sizeof(int) * lx.size());
        if (nbr)
            for (int p = 0; p < 2; ++p)
                for (int d = 0; d < 8; ++d)
                    for (long i = 0; i < lat->Vh; ++i)
                        nbr[(p * 8 + d) * lat->Vh + i] = lx[(1 - p) * lat->Vh + nb[(p * 8 + d) * lat->Vhp + i]];
        return DWF_OK;
    });
}

int dwf_op_create_sdep(dwf_lattice* lat, int Ls, double M0, double m, const double* b, const double* c,
                       double alpha, dwf_op** out) {
    return guarded([&] {
        DWF_REQUIRE(lat && out && b && c, DWF_EINVAL, "null argument");
        DWF_REQUIRE(Ls >= 2 && Ls <= LS_MAX, DWF_EDIMS, "Ls must be in [2, 16]");
        for (int s = 0; s < Ls; ++s)
            DWF_REQUIRE(std::isfinite(b[s]) && std::isfinite(c[s]), DWF_EINVAL, "non-finite b_s or c_s");
        DWF_REQUIRE(std::isfinite(M0) && std::isfinite(m) && std::isfinite(alpha), DWF_EINVAL, "non-finite parameter");
        std::unique_ptr<dwf_op> op(new dwf_op());
        op->lat = lat;
        op->Ls = Ls;
        op->M0 = M0;
        op->m = m;
        op->b.assign(b, b + Ls);
        op->c.assign(c, c + Ls);
        op->alpha = alpha;
        setup_op(op.get());
        *out = op.release();
        return DWF_OK;
    });
}

int dwf_op_create(dwf_lattice* lat, int Ls, double M0, double m, double b, double c, double alpha, dwf_op** out) {
    if (Ls < 2 || Ls > LS_MAX) {
        set_error("Ls must be in [2, 16]");
        return DWF_EDIMS;
    }
    const std::vector<double> bs(Ls, b), cs(Ls, c);
    return dwf_op_create_sdep(lat, Ls, M0, m, bs.data(), cs.data(), alpha, out);
}

void dwf_op_destroy(dwf_op* op) { delete op; }

static int kind_of(int prec) {
    DWF_REQUIRE(prec == DWF_F64 || prec == DWF_F32 || prec == DWF_BF16, DWF_EINVAL, "bad precision");
    return prec;
}

int dwf_apply(const dwf_op* op, int space, int dagger, int prec, void* out, const void* in, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && out && in, DWF_EINVAL, "null argument");
        DWF_REQUIRE(out != in, DWF_EINVAL, "in and out must not alias");
        const int k = kind_of(prec);
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = L->Vh, Vhp = L->Vhp, V = L->V, n = (long)op->Ls * 12 * Vhp;
        const size_t bytes = complex_bytes_of(k) * n;
        hipStream_t st = S(stream);
        const int* lex = L->lex_of_site_dev.as<int>();
        if (space == DWF_FULL5D) {
            DevBuf ie(bytes), io(bytes), oe(bytes), oo(bytes);
            pack_full(k, ie.p, in, lex, Vh, Vhp, V, op->Ls, st);
            pack_full(k, io.p, in, lex + Vh, Vh, Vhp, V, op->Ls, st);
            apply_full(op, k, dagger, oe.p, oo.p, ie.p, io.p, 1, st);
            unpack_full(k, out, oe.p, lex, Vh, Vhp, V, op->Ls, st);
            unpack_full(k, out, oo.p, lex + Vh, Vh, Vhp, V, op->Ls, st);
            DWF_HIP(hipStreamSynchronize(st));
        } else if (space == DWF_EVEN5D) {
            DevBuf ie(bytes), oe(bytes), to(bytes), te(bytes);
            pack_half(k, ie.p, in, lex, Vh, Vhp, op->Ls, st);
            apply_dhat(op, k, dagger, oe.p, ie.p, to.p, te.p, 1, st);
            unpack_half(k, out, oe.p, lex, Vh, Vhp, op->Ls, st);
            DWF_HIP(hipStreamSynchronize(st));
        } else {
            throw Error{DWF_EINVAL, "bad space"};
        }
        return DWF_OK;
    });
}

int dwf_apply_normal(const dwf_op* op, int prec, void* out, const void* in, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && out && in, DWF_EINVAL, "null argument");
        DWF_REQUIRE(out != in, DWF_EINVAL, "in and out must not alias");
        const int k = kind_of(prec);
        DWF_REQUIRE(op->lat->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = op->lat->Vh, Vhp = op->lat->Vhp, n = (long)op->Ls * 12 * Vhp;
        const size_t bytes = complex_bytes_of(k) * n;
        hipStream_t st = S(stream);
        DevBuf ie(bytes), oe(bytes), to(bytes), tv(bytes);
        const int* lex = op->lat->lex_of_site_dev.as<int>();
        pack_half(k, ie.p, in, lex, Vh, Vhp, op->Ls, st);
        apply_normal(op, k, oe.p, ie.p, to.p, tv.p, nullptr, 1, st);
        unpack_half(k, out, oe.p, lex, Vh, Vhp, op->Ls, st);
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

}  // extern "C"

// Device scratch of dwf_apply_normal_noalloc, for callers that cannot
// allocate: the four half fields of the normal operator (packed input,
// output, two hop temporaries) live in this file-scope array, one copy per
// GPU, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and used from then on.
static constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

void* noalloc_scratch() {
    int dev = 0;
    DWF_HIP(hipGetDevice(&dev));
    DWF_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, DWF_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            throw Error{DWF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

int dwf_apply_normal_noalloc(const dwf_op* op, int prec, void* out, const void* in, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && out && in, DWF_EINVAL, "null argument");
        DWF_REQUIRE(out != in, DWF_EINVAL, "in and out must not alias");
        const int k = kind_of(prec);
        DWF_REQUIRE(op->lat->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = op->lat->Vh, Vhp = op->lat->Vhp, n = (long)op->Ls * 12 * Vhp;
        const size_t slot = (complex_bytes_of(k) * (size_t)n + 255) & ~(size_t)255;
        if (4 * slot > NOALLOC_SCRATCH_BYTES)
            throw Error{DWF_EDIMS, "dwf_apply_normal_noalloc: four half fields of " + std::to_string(slot) +
                                       " bytes exceed its " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                                       " MiB scratch; use dwf_apply_normal"};
        char* base = static_cast<char*>(noalloc_scratch());
        void *ie = base, *oe = base + slot, *to = base + 2 * slot, *tv = base + 3 * slot;
        hipStream_t st = S(stream);
        const int* lex = op->lat->lex_of_site_dev.as<int>();
        pack_half(k, ie, in, lex, Vh, Vhp, op->Ls, st);
        apply_normal(op, k, oe, ie, to, tv, nullptr, 1, st);
        unpack_half(k, out, oe, lex, Vh, Vhp, op->Ls, st);
        return DWF_OK;
    });
}

int dwf_cg_residual_update(const dwf_op* op, int prec, void* r, const void* p, double* alpha, double* rr_new,
                           void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && r && p, DWF_EINVAL, "null argument");
        DWF_REQUIRE(r != p, DWF_EINVAL, "r and p must not alias");
        const int k = kind_of(prec);
        const int kx = k == ST_F64 ? ST_F64 : ST_F32;   // r in the compute type
        DWF_REQUIRE(op->lat->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = op->lat->Vh, Vhp = op->lat->Vhp, n = (long)op->Ls * 12 * Vhp;
        hipStream_t st = S(stream);
        DevBuf rb(complex_bytes_of(kx) * n), pb(complex_bytes_of(k) * n), to(complex_bytes_of(k) * n),
            tv(complex_bytes_of(k) * n);
        DevBuf partial((std::max<long>(hop_partials(op, 1), blas_grid(n)) + 16) * sizeof(double)),
            scal(CG_NSLOTS * sizeof(double));
        const int* lex = op->lat->lex_of_site_dev.as<int>();
        pack_half(kx, rb.p, r, lex, Vh, Vhp, op->Ls, st);
        pack_half(k, pb.p, p, lex, Vh, Vhp, op->Ls, st);
        double* pp = partial.as<double>();
        double* sc = scal.as<double>();
        norm2_partial(kx, rb.p, n, pp, st);
        finalize(pp, blas_grid(n), 1, sc + CG_RR, 0, st);
        apply_normal_update_r(op, k, rb.p, pb.p, to.p, tv.p, pp, sc, 1, st);
        finalize(pp, hop_partials(op, 1), 1, sc + CG_TMP, 0, st);
        unpack_half(kx, r, rb.p, lex, Vh, Vhp, op->Ls, st);
        double h[CG_NSLOTS];
        DWF_HIP(hipMemcpyAsync(h, sc, sizeof h, hipMemcpyDeviceToHost, st));
        DWF_HIP(hipStreamSynchronize(st));
        if (alpha) *alpha = h[CG_ALPHA];
        if (rr_new) *rr_new = h[CG_TMP];
        return DWF_OK;
    });
}

int dwf_source_4d(const dwf_op* op, void* b5, const void* b4, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && b5 && b4, DWF_EINVAL, "null argument");
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = L->Vh, Vhp = L->Vhp, V = L->V;
        const int Ls = op->Ls;
        hipStream_t st = S(stream);
        const int* lex = L->lex_of_site_dev.as<int>();
        const size_t pair_bytes = 16 * (size_t)2 * 12 * Vhp;
        DevBuf pe(pair_bytes), po(pair_bytes), oe(pair_bytes), oo(pair_bytes);
        pack_chiral_pair_f64(pe.p, b4, lex, Vh, Vhp, st);
        pack_chiral_pair_f64(po.p, b4, lex + Vh, Vh, Vhp, st);
        source_pair(op, oe.p, po.p, pe.p, 0, st);
        source_pair(op, oo.p, pe.p, po.p, 1, st);
        // b5 = 0 except s = 0 (slice 0 of the pair) and s = Ls-1 (slice 1)
        DWF_HIP(hipMemsetAsync(b5, 0, (size_t)16 * Ls * V * 12, st));
        const size_t slice = (size_t)16 * 12 * Vhp;
        DevBuf fe((size_t)16 * Ls * 12 * Vhp), fo((size_t)16 * Ls * 12 * Vhp);
        DWF_HIP(hipMemsetAsync(fe.p, 0, fe.bytes, st));
        DWF_HIP(hipMemsetAsync(fo.p, 0, fo.bytes, st));
        DWF_HIP(hipMemcpyAsync(fe.p, oe.p, slice, hipMemcpyDeviceToDevice, st));
        DWF_HIP(hipMemcpyAsync(fo.p, oo.p, slice, hipMemcpyDeviceToDevice, st));
        DWF_HIP(hipMemcpyAsync(fe.as<char>() + slice * (Ls - 1), oe.as<char>() + slice, slice,
                               hipMemcpyDeviceToDevice, st));
        DWF_HIP(hipMemcpyAsync(fo.as<char>() + slice * (Ls - 1), oo.as<char>() + slice, slice,
                               hipMemcpyDeviceToDevice, st));
        unpack_full(ST_F64, b5, fe.p, lex, Vh, Vhp, V, Ls, st);
        unpack_full(ST_F64, b5, fo.p, lex + Vh, Vh, Vhp, V, Ls, st);
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

int dwf_project_4d(const dwf_op* op, void* x4, const void* x5, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && x4 && x5, DWF_EINVAL, "null argument");
        project_4d(x4, x5, op->lat->V, op->Ls, S(stream));
        DWF_HIP(hipStreamSynchronize(S(stream)));
        return DWF_OK;
    });
}

int dwf_solve(const dwf_op* op, void* x5, const void* b5, const dwf_solve_params* prm, dwf_solve_info* info,
              void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && x5 && b5, DWF_EINVAL, "null argument");
        dwf_solve_params def;
        dwf_solve_params_default(&def);
        const dwf_solve_params* p = prm ? prm : &def;
        DWF_REQUIRE(p->algo == DWF_ALGO_CGNR || p->algo == DWF_ALGO_DC || p->algo == DWF_ALGO_MIXED ||
                        p->algo == DWF_ALGO_FGCR_LEARNED,
                    DWF_EINVAL, "unsupported algorithm");
        DWF_REQUIRE(!(p->algo == DWF_ALGO_FGCR_LEARNED && p->paper_mode), DWF_EINVAL,
                    "paper_mode applies to CGNR only");
        DWF_REQUIRE(p->schur == 0 ||
                        ((p->schur == 1 || p->schur == 2) && (p->algo == DWF_ALGO_CGNR || p->algo == DWF_ALGO_DC)),
                    DWF_EINVAL,
                    "schur: 0 (left) for every algorithm, 1 (right) and 2 (5D split) with CGNR or DC only");
        return solve(op, x5, b5, p, info, S(stream));
    });
}

int dwf_apply_eo5(const dwf_op* op, int prec, int dagger, void* out5, const void* in5, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && out5 && in5, DWF_EINVAL, "null argument");
        DWF_REQUIRE(out5 != in5, DWF_EINVAL, "in and out must not alias");
        DWF_REQUIRE(dagger == 0 || dagger == 1, DWF_EINVAL, "dagger: 0 or 1");
        DWF_REQUIRE(prec == DWF_F64 || prec == DWF_F32, DWF_EINVAL, "the 5D even-odd split runs in FP64 or FP32");
        apply_eo5_schur(op, kind_of(prec), dagger, out5, in5, S(stream));
        return DWF_OK;
    });
}

int dwf_true_residual(const dwf_op* op, const void* x5, const void* b5, double* rel, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && x5 && b5 && rel, DWF_EINVAL, "null argument");
        *rel = true_residual(op, x5, b5, S(stream));
        return DWF_OK;
    });
}

int dwf_bench_hop(const dwf_op* op, int prec, int nrep, double* ms_per_launch, double* bytes_per_launch,
                  void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && nrep > 0, DWF_EINVAL, "bad argument");
        const int k = kind_of(prec);
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        const long Vh = L->Vh, n = (long)op->Ls * 12 * L->Vhp;
        const size_t cb = complex_bytes_of(k);
        hipStream_t st = S(stream);
        // seeded non-zero inputs; launches rotate over enough (in, out) sets
        // that the sets together exceed the 256 MB Infinity Cache, so every
        // launch reads its fields from HBM
        const size_t fb = cb * (size_t)n;
        const int nsets = (int)std::min<size_t>(8, std::max<size_t>(1, ((size_t)768 << 20) / (2 * fb) + 1));
        std::vector<DevBuf> ins(nsets), outs(nsets);
        {
            DevBuf tmp(16 * (size_t)n);
            for (int i = 0; i < nsets; ++i) {
                ins[i].alloc(fb);
                outs[i].alloc(fb);
                random_fill_f64(tmp.p, (long)op->Ls * 12, Vh, L->Vhp, 0x5eedULL + (unsigned long long)i, st);
                convert(k, ST_F64, ins[i].p, tmp.p, n, st, L->Vhp);
            }
            DWF_HIP(hipStreamSynchronize(st));
        }
        auto launch = [&](int i) {
            hop(op, k, 1, ins[i % nsets].p, nullptr, outs[i % nsets].p, PRE_K, MAT_Q, -1, 0.0, nullptr, 0, 0,
                nullptr, 0, 1, st, 0, 1);
        };
        for (int i = 0; i < nsets; ++i) launch(i);   // warm up
        hipEvent_t e0, e1;
        DWF_HIP(hipEventCreate(&e0));
        DWF_HIP(hipEventCreate(&e1));
        DWF_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < nrep; ++i) launch(i);
        DWF_HIP(hipEventRecord(e1, st));
        DWF_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
        DWF_HIP(hipEventDestroy(e0));
        DWF_HIP(hipEventDestroy(e1));
        if (ms_per_launch) *ms_per_launch = ms / nrep;
        // read every input spinor once, write every output once, read every link once
        const double w = (double)cb / 2.0;   // bytes per real
        if (bytes_per_launch) *bytes_per_launch = w * (double)Vh * (48.0 * op->Ls + 144.0);
        return DWF_OK;
    });
}

int dwf_solve_batch(int n, const dwf_op* const* ops, void* const* x5, const void* const* b5, const int* nrhs,
                    const dwf_solve_params* prm, dwf_solve_info* infos, void* stream) {
    return guarded([&] {
        dwf_solve_params def;
        dwf_solve_params_default(&def);
        def.algo = DWF_ALGO_DC;
        def.check_every = 8;
        DWF_REQUIRE(!prm || prm->schur == 0, DWF_EINVAL, "batched solves use the left Schur system (schur = 0)");
        return solve_batch(n, ops, x5, b5, nrhs, prm ? prm : &def, infos, S(stream));
    });
}

int dwf_autotune_batch(int n, const dwf_op* const* ops, const int* nrhs, int prec, int force, int* nrb, int* order,
                       double* ms, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(nrb && order, DWF_EINVAL, "null argument");
        double t = 0;
        autotune_batch(n, ops, nrhs, prec, force, nrb, order, &t, S(stream));
        if (ms) *ms = t;
        return DWF_OK;
    });
}

int dwf_tune_cache_put(const char* key, int nrb, int order, double ms) {
    return guarded([&] {
        DWF_REQUIRE(key && nrb >= 1 && nrb <= 64 && (order == 0 || order == 1), DWF_EINVAL, "bad tune entry");
        tune_put(key, nrb, order, ms);
        return DWF_OK;
    });
}

int dwf_tune_cache_get(const char* key, int* nrb, int* order, double* ms) {
    return guarded([&] {
        DWF_REQUIRE(key && nrb && order, DWF_EINVAL, "null argument");
        return tune_get(key, nrb, order, ms) ? DWF_OK : DWF_NOT_CONVERGED;
    });
}

int dwf_tune_cache_reload(void) {
    return guarded([&] {
        tune_forget();
        return DWF_OK;
    });
}

int dwf_lanczos_extremes(const dwf_op* op, int basis, int keep, int max_restarts, double tol, double* lambda_min,
                         double* lambda_max, int* matvecs, int* converged, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && lambda_min && lambda_max, DWF_EINVAL, "null argument");
        lanczos_extremes(op, basis, keep, max_restarts, tol, lambda_min, lambda_max, matvecs, converged, S(stream));
        return (converged && !*converged) ? DWF_NOT_CONVERGED : DWF_OK;
    });
}

// ---- learned preconditioner ------------------------------------------
int dwf_ptc_create(int hidden, unsigned long long seed, double init_scale, dwf_ptc** out) {
    return guarded([&] {
        DWF_REQUIRE(out, DWF_EINVAL, "null argument");
        DWF_REQUIRE(init_scale >= 0.0 && init_scale < 10.0, DWF_EINVAL, "init_scale out of range");
        *out = ptc_create(hidden, seed, init_scale);
        return DWF_OK;
    });
}

void dwf_ptc_destroy(dwf_ptc* m) { delete m; }

int dwf_ptc_set_loss(dwf_ptc* m, int kind) {
    return guarded([&] {
        DWF_REQUIRE(m && (kind == 0 || kind == 1), DWF_EINVAL, "loss kind must be 0 or 1");
        m->loss_kind = kind;
        return DWF_OK;
    });
}

int dwf_ptc_info(const dwf_ptc* m, int* hidden, int* nweights, int* steps) {
    return guarded([&] {
        DWF_REQUIRE(m, DWF_EINVAL, "null model");
        if (hidden) *hidden = m->H;
        if (nweights) *nweights = (int)m->nw;
        if (steps) *steps = m->step;
        return DWF_OK;
    });
}

int dwf_ptc_get_weights(const dwf_ptc* m, void* w) {
    return guarded([&] {
        DWF_REQUIRE(m && w, DWF_EINVAL, "null argument");
        DWF_HIP(hipMemcpy(w, m->W.p, m->nw * 8, hipMemcpyDeviceToHost));
        return DWF_OK;
    });
}

int dwf_ptc_set_weights(dwf_ptc* m, const void* w) {
    return guarded([&] {
        DWF_REQUIRE(m && w, DWF_EINVAL, "null argument");
        DWF_HIP(hipMemcpy(m->W.p, w, m->nw * 8, hipMemcpyHostToDevice));
        return DWF_OK;
    });
}

int dwf_ptc_apply(dwf_ptc* m, const dwf_op* op, void* out_e, const void* in_e, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(m && op && out_e && in_e, DWF_EINVAL, "null argument");
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        hipStream_t st = S(stream);
        const long n = ptc_field_elems(op);
        DevBuf a(8 * (size_t)n), b(8 * (size_t)n);
        const int* lex = L->lex_of_site_dev.as<int>();
        pack_half(ST_F32, a.p, in_e, lex, L->Vh, L->Vhp, op->Ls, st);
        m->forward(op, a.as<float2>(), b.as<float2>(), st);
        unpack_half(ST_F32, out_e, b.p, lex, L->Vh, L->Vhp, op->Ls, st);
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

int dwf_ptc_bench_apply(dwf_ptc* m, const dwf_op* op, int nrep, double* ms_per_apply, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(m && op && nrep > 0 && ms_per_apply, DWF_EINVAL, "bad argument");
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        hipStream_t st = S(stream);
        const long n = ptc_field_elems(op);
        DevBuf a(8 * (size_t)n), b(8 * (size_t)n), t(16 * (size_t)n);
        random_fill_f64(t.p, (long)op->Ls * 12, L->Vh, L->Vhp, 0x7ee5ULL, st);
        convert(ST_F32, ST_F64, a.p, t.p, n, st, L->Vhp);
        m->forward(op, a.as<float2>(), b.as<float2>(), st);   // warm-up (workspace)
        hipEvent_t e0, e1;
        DWF_HIP(hipEventCreate(&e0));
        DWF_HIP(hipEventCreate(&e1));
        DWF_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < nrep; ++i) m->forward(op, a.as<float2>(), b.as<float2>(), st);
        DWF_HIP(hipEventRecord(e1, st));
        DWF_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
        DWF_HIP(hipEventDestroy(e0));
        DWF_HIP(hipEventDestroy(e1));
        *ms_per_apply = ms / nrep;
        return DWF_OK;
    });
}

int dwf_ptc_gradient(dwf_ptc* m, const dwf_op* op, const void* r_e, const void* e_e, double* loss, void* grad,
                     void* stream) {
    return guarded([&] {
        DWF_REQUIRE(m && op && r_e && e_e, DWF_EINVAL, "null argument");
        const dwf_lattice* L = op->lat;
        DWF_REQUIRE(L->has_gauge, DWF_ESTATE, "gauge field not set");
        hipStream_t st = S(stream);
        const long n = ptc_field_elems(op);
        DevBuf r(8 * (size_t)n), e(8 * (size_t)n);
        const int* lex = L->lex_of_site_dev.as<int>();
        pack_half(ST_F32, r.p, r_e, lex, L->Vh, L->Vhp, op->Ls, st);
        pack_half(ST_F32, e.p, e_e, lex, L->Vh, L->Vhp, op->Ls, st);
        m->gradient(op, r.as<float2>(), e.as<float2>(), st);
        double h = 0;
        DWF_HIP(hipMemcpyAsync(&h, m->stats.p, sizeof(double), hipMemcpyDeviceToHost, st));
        if (grad) DWF_HIP(hipMemcpyAsync(grad, m->G.p, m->nw * 8, hipMemcpyDeviceToHost, st));
        DWF_HIP(hipStreamSynchronize(st));
        if (loss) *loss = h;
        return DWF_OK;
    });
}

int dwf_ptc_pairs_create(const dwf_op* op, const void* b5, unsigned long long seed, int nsnap,
                         const int* snap_iters, dwf_ptc_pairs** out, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(out, DWF_EINVAL, "null argument");
        *out = ptc_pairs_create(op, b5, seed, nsnap, snap_iters, S(stream));
        return DWF_OK;
    });
}

int dwf_ptc_pairs_get(const dwf_ptc_pairs* p, int k, void* r_e, void* e_e, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(p && r_e && e_e && k >= 0 && k < p->count, DWF_EINVAL, "bad pair index");
        const dwf_lattice* L = p->op->lat;
        hipStream_t st = S(stream);
        const int* lex = L->lex_of_site_dev.as<int>();
        unpack_half(ST_F32, r_e, p->r.as<float2>() + (size_t)k * p->n, lex, L->Vh, L->Vhp, p->op->Ls, st);
        unpack_half(ST_F32, e_e, p->e.as<float2>() + (size_t)k * p->n, lex, L->Vh, L->Vhp, p->op->Ls, st);
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

void dwf_ptc_pairs_destroy(dwf_ptc_pairs* p) { delete p; }

int dwf_ptc_train(dwf_ptc* m, int nsets, dwf_ptc_pairs* const* sets, int steps, double lr, unsigned long long seed,
                  double* loss_history, void* stream) {
    return guarded([&] {
        ptc_train(m, nsets, sets, steps, lr, seed, loss_history, S(stream));
        return DWF_OK;
    });
}

int dwf_ptc_eval(dwf_ptc* m, int nsets, dwf_ptc_pairs* const* sets, double* mean_loss, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(m && nsets >= 1 && sets && mean_loss, DWF_EINVAL, "null argument");
        for (int i = 0; i < nsets; ++i) DWF_REQUIRE(sets[i], DWF_EINVAL, "null pair set");
        *mean_loss = ptc_eval(m, nsets, sets, S(stream));
        return DWF_OK;
    });
}

int dwf_ptc_save(const dwf_ptc* m, const char* path) {
    return guarded([&] {
        ptc_save(m, path);
        return DWF_OK;
    });
}

int dwf_ptc_load(const char* path, dwf_ptc** out) {
    return guarded([&] {
        DWF_REQUIRE(out, DWF_EINVAL, "null argument");
        *out = ptc_load(path);
        return DWF_OK;
    });
}

int dwf_gauge_sweeps(const int dims[4], void* U, double beta, int nsweeps, int n_or, unsigned long long seed,
                     long long sweep0, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(dims && U, DWF_EINVAL, "null argument");
        for (int mu = 0; mu < 4; ++mu)
            DWF_REQUIRE(dims[mu] >= 2 && dims[mu] % 2 == 0, DWF_EDIMS, "every lattice extent must be even and >= 2");
        DWF_REQUIRE(nsweeps >= 0 && n_or >= 0 && beta > 0.0 && std::isfinite(beta), DWF_EINVAL,
                    "nsweeps, n_or >= 0 and beta > 0 required");
        const double V = (double)dims[0] * dims[1] * dims[2] * dims[3];
        DWF_REQUIRE(V * 4.0 * 3.0 * 4096.0 < 1.8e19, DWF_EDIMS, "lattice too large for the random-number counters");
        hipStream_t st = S(stream);
        for (int k = 0; k < nsweeps; ++k) {
            gauge_sweep(U, dims, beta, seed, sweep0 + k, true, st);
            for (int o = 0; o < n_or; ++o) gauge_sweep(U, dims, beta, seed, sweep0 + k, false, st);
        }
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

int dwf_gauge_plaquette(const int dims[4], const void* U, double* plaq, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(dims && U && plaq, DWF_EINVAL, "null argument");
        for (int mu = 0; mu < 4; ++mu) DWF_REQUIRE(dims[mu] >= 1, DWF_EDIMS, "bad lattice extent");
        hipStream_t st = S(stream);
        DevBuf partial((size_t)(gauge_plaquette_partials(dims) + 1) * sizeof(double));
        double* out = partial.as<double>() + gauge_plaquette_partials(dims);
        gauge_plaquette(U, dims, partial.as<double>(), out, st);
        DWF_HIP(hipMemcpyAsync(plaq, out, sizeof(double), hipMemcpyDeviceToHost, st));
        DWF_HIP(hipStreamSynchronize(st));
        return DWF_OK;
    });
}

int dwf_bench_copy(size_t bytes, int nrep, double* ms_per_launch, void* stream) {
    return guarded([&] {
        DWF_REQUIRE(bytes >= 16 && nrep > 0, DWF_EINVAL, "bad argument");
        bytes &= ~(size_t)15;
        hipStream_t st = S(stream);
        DevBuf a(bytes), b(bytes);
        DWF_HIP(hipMemsetAsync(a.p, 0, bytes, st));
        launch_copy(b.p, a.p, bytes, st);
        hipEvent_t e0, e1;
        DWF_HIP(hipEventCreate(&e0));
        DWF_HIP(hipEventCreate(&e1));
        DWF_HIP(hipEventRecord(e0, st));
        for (int i = 0; i < nrep; ++i) launch_copy(b.p, a.p, bytes, st);
        DWF_HIP(hipEventRecord(e1, st));
        DWF_HIP(hipEventSynchronize(e1));
        float ms = 0;
        DWF_HIP(hipEventElapsedTime(&ms, e0, e1));
        DWF_HIP(hipEventDestroy(e0));
        DWF_HIP(hipEventDestroy(e1));
        if (ms_per_launch) *ms_per_launch = ms / nrep;
        return DWF_OK;
    });
}

int dwf_residual_4d(const dwf_op* op, const void* x4, const void* b4, double tol_inner, double* rel,
                    void* stream) {
    return guarded([&] {
        DWF_REQUIRE(op && x4 && b4 && rel, DWF_EINVAL, "null argument");
        DWF_REQUIRE(op->lat->has_gauge, DWF_ESTATE, "gauge field not set");
        bool ok = false;
        *rel = residual_4d(op, x4, b4, tol_inner > 0 ? tol_inner : 1e-13, S(stream), &ok);
        if (!ok) set_error("the inner m = 1 solve of the 4D residual did not reach tol_inner");
        return ok ? DWF_OK : DWF_NOT_CONVERGED;
    });
}

}  // extern "C"
