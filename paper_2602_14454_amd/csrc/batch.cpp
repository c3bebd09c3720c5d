// Batched solves: several right-hand sides of one operator (the 12
// spin-colour point sources of a propagator) and several independent
// lattices of different size, Ls and mass, solved together.
//
// Method per slot (slot = one right-hand side of one operator): the same
// FP64 defect correction as the single solve (Sec. 2.3: the low-precision
// solver used as the preconditioner of a double-precision solve) around a
// CGNR on D^dag D^ in FP32 or BF16 storage.
//
// Batching: every kernel of the inner CG iteration covers all slots in one
// launch.  The four fused hops of D^dag D^ run as work-list launches (one per
// class of ceil(Ls/4)), the CG vector updates and reductions as slot-table
// launches, and each slot carries its own alpha, beta, stopping threshold,
// iteration count and done flag on the device; like the single solve, a slot
// tests its residual at multiples of the check period.  A slot that has
// converged is skipped by every kernel.  The iteration body (k iterations) is
// captured once into a HIP graph and replayed; the host reads the done
// flags after each replay.  Within a replay the search directions go to a
// ring of batch vectors (at most 16, and at most 8 GiB) and x is formed from
// them at the end of the ring and of the replay, so x is not read or written
// in every iteration.  The FP64 outer steps use the per-operator kernels with
// all right-hand sides of an operator in one launch; each operator takes its
// outer step as soon as all its right-hand sides are done, while the others
// keep iterating.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "slot_blas.h"
#include "blas.h"
#include "dwf_internal.h"
#include "hop.h"
#include "ops.h"
#include "solver.h"

namespace dwf {

// ---------------------------------------------------------------------
// tile autotuner cache: key -> (nrb, order, ms), kept in memory and in a
// text file (one "key nrb order ms" line per entry)
// ---------------------------------------------------------------------
namespace {
struct TuneEntry {
    int nrb, order;
    double ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string cache_path() {
    const char* p = std::getenv("DWF_TUNE_CACHE");
    if (p) return std::string(p) == "off" ? std::string() : std::string(p);
    const char* h = std::getenv("HOME");
    return h ? std::string(h) + "/.cache/libdwf_tune.txt" : std::string();
}

void load_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        TuneEntry e{};
        if (is >> key >> e.nrb >> e.order >> e.ms && e.nrb >= 1 && e.nrb <= 64 && (e.order == 0 || e.order == 1))
            g_tune[key] = e;
    }
}
}  // namespace

bool tune_get(const std::string& key, int* nrb, int* order, double* ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *nrb = it->second.nrb;
    *order = it->second.order;
    if (ms) *ms = it->second.ms;
    return true;
}

void tune_put(const std::string& key, int nrb, int order, double ms) {
    DWF_REQUIRE(!key.empty() && key.find_first_of(" \t\n") == std::string::npos, DWF_EINVAL, "bad tune key");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    g_tune[key] = TuneEntry{nrb, order, ms};
    const std::string path = cache_path();
    if (path.empty()) return;
    const std::string tmp = path + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return;   // an unwritable cache only loses persistence
        for (auto& kv : g_tune) f << kv.first << ' ' << kv.second.nrb << ' ' << kv.second.order << ' ' << kv.second.ms << '\n';
    }
    std::rename(tmp.c_str(), path.c_str());
}

void tune_forget() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_tune_loaded = false;
}

// ---------------------------------------------------------------------
namespace {

struct Item {
    const dwf_op* op;
    int nrhs, slot0;
    long off;   // complex-element offset of the item's first right-hand side
    long n1;    // complex elements of one right-hand side
};

struct HopClass {
    int KK;
    std::vector<int> items;   // indices into Batch::items
    int pm[4] = {-1, -1, -1, -1};   // per stage: the items' common pre-mix mode, -1 if mixed
    int ek[4] = {-1, -1, -1, -1};   // per stage: the items' common epilogue kind, -1 if mixed
};

struct Stream {
    hipStream_t s = nullptr;
    Stream() { DWF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
    ~Stream() { if (s) (void)hipStreamDestroy(s); }
};

struct Event {
    hipEvent_t e = nullptr;
    Event() { DWF_HIP(hipEventCreate(&e)); }
    ~Event() { if (e) (void)hipEventDestroy(e); }
};

struct GraphExec {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~GraphExec() { reset(); }
    void reset() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
        x = nullptr;
        g = nullptr;
    }
};

struct PinnedD {
    double* h = nullptr;
    explicit PinnedD(size_t n) {
        if (hipHostMalloc(reinterpret_cast<void**>(&h), std::max<size_t>(n, 1) * sizeof(double),
                          hipHostMallocDefault) != hipSuccess)
            throw Error{DWF_ENOMEM, "hipHostMalloc failed"};
        std::memset(h, 0, std::max<size_t>(n, 1) * sizeof(double));
    }
    ~PinnedD() { if (h) (void)hipHostFree(h); }
};

std::string tune_key(const std::vector<Item>& items, int kp) {
    std::ostringstream k;
    k << "gfx950|p" << kp;
    for (const Item& it : items) {
        const dwf_lattice* L = it.op->lat;
        k << '|' << L->dims[0] << 'x' << L->dims[1] << 'x' << L->dims[2] << 'x' << L->dims[3] << 's' << it.op->Ls
          << 'r' << it.nrhs;
    }
    return k.str();
}

// The four hops of D^dag D^ (ops.cpp apply_normal) as work-list launches.
// The first two read the search direction, which lives in one of `ring`
// batch vectors: they have one table per ring slot.
struct NormalHops {
    std::vector<HopClass> classes;
    DevBuf items_dev, meta_dev;
    std::vector<int> blocks;   // per class
    int nrb = 1, order = 0, kind = ST_F32, ring = 1;
    size_t per_stage = 0;      // HopParams per stage
    size_t meta_per_class = 0;
    bool stage_loc[4] = {false, false, false, false};   // stage carries a local term

    // table of stage sidx with the direction in ring slot q
    size_t table(int sidx, int q) const { return sidx < 2 ? (size_t)(2 * q + sidx) : (size_t)(2 * ring + sidx - 2); }

    // fields: in/out buffers of storage `kind` (ring slot q of the direction at
    // p_ring + q * ring_bytes); partial/pstride/done for the reductions
    void build(const std::vector<Item>& items, int kind_, int nrb_, int order_, void* p_ring, size_t ring_bytes,
               int ring_, void* t, void* v, void* r, double* partial, long pstride, const double* scal) {
        kind = kind_;
        nrb = nrb_;
        order = order_;
        ring = ring_;
        classes.clear();
        for (int i = 0; i < (int)items.size(); ++i) {
            const int KK = (items[i].op->Ls + 3) / 4;
            auto c = std::find_if(classes.begin(), classes.end(), [&](const HopClass& h) { return h.KK == KK; });
            if (c == classes.end()) classes.push_back(HopClass{KK, {i}});
            else c->items.push_back(i);
        }
        const size_t cb = complex_bytes_of(kind);
        std::vector<HopParams> hp;
        std::vector<int> meta;
        blocks.clear();
        per_stage = items.size();
        meta_per_class = 0;
        for (auto& c : classes) meta_per_class = std::max(meta_per_class, 2 * c.items.size() + 1);
        hp.resize((2 * (size_t)ring + 2) * per_stage);
        meta.assign(classes.size() * meta_per_class, 0);
        int pos = 0;
        for (size_t ci = 0; ci < classes.size(); ++ci) {
            HopClass& c = classes[ci];
            int* m = meta.data() + ci * meta_per_class;
            int acc = 0;
            for (size_t q = 0; q < c.items.size(); ++q) {
                const Item& it = items[c.items[q]];
                m[q] = acc;
                m[c.items.size() + 1 + q] = it.nrhs;
                acc += hop_grid_blocks(it.op->lat->Vh) * ((it.nrhs + nrb - 1) / nrb);
                auto at = [&](void* b) { return static_cast<char*>(b) + (size_t)it.off * cb; };
                const dwf_op* op = it.op;
                double* part = partial + (long)it.slot0 * pstride;
                const double* done = scal + (long)it.slot0 * CG_NSLOTS + CG_DONE;
                HopParams s1 = hop_params(op, kind, 1, at(p_ring), nullptr, at(t), PRE_K, MAT_Q, -1, 0.0, nullptr, 0,
                                          0, nullptr, 0);
                HopParams s2 = hop_params(op, kind, 0, at(t), at(p_ring), nullptr, -1, MAT_MQMINV, -1, 1.0, at(v),
                                          DWF_CHAIN2 ? MAT_G5MIT : MAT_G5MIT_MQMINV, MAT_G5MIT, part, 1);
                s2.chain2 = DWF_CHAIN2;   // v = g5 Minv^T q from q itself
                HopParams s3 = hop_params(op, kind, 1, at(v), nullptr, at(t), -1, MAT_QT, -1, 0.0, nullptr, 0, 0,
                                          nullptr, 0);
                // stage 4 applies r -= alpha D^dag D^ p per slot and reduces |r|^2
                HopParams s4 = hop_params(op, kind, 0, at(t), at(v), nullptr, -1, MAT_MQG5KT, MAT_G5MT, 0.0, nullptr, 0,
                                          0, part, 3);
                s4.upd = static_cast<char*>(r) + (size_t)it.off * complex_bytes_of(kind == ST_F64 ? ST_F64 : ST_F32);
                s4.upd_alpha = scal + (long)it.slot0 * CG_NSLOTS + CG_ALPHA;
                s4.upd_stride = CG_NSLOTS;
                for (HopParams* P : {&s1, &s2, &s3, &s4}) {
                    P->done = done;
                    P->done_stride = CG_NSLOTS;
                    P->pstride = pstride;
                }
                stage_loc[0] = s1.loc != nullptr;
                stage_loc[1] = s2.loc != nullptr;
                stage_loc[2] = s3.loc != nullptr;
                stage_loc[3] = s4.loc != nullptr;
                const HopParams* sp[4] = {&s1, &s2, &s3, &s4};
                for (int k = 0; k < 4; ++k) {
                    int& pm = c.pm[k];
                    pm = q == 0 ? sp[k]->pre_mode : (pm == sp[k]->pre_mode ? pm : -1);
                    const int e = hop_epilogue_kind(*sp[k]);
                    c.ek[k] = q == 0 ? e : (c.ek[k] == e ? e : -1);
                }
                for (int q = 0; q < ring; ++q) {
                    const size_t shift = (size_t)q * ring_bytes;
                    HopParams a = s1, b = s2;
                    a.in = static_cast<const char*>(s1.in) + shift;
                    b.loc = static_cast<const char*>(s2.loc) + shift;
                    hp[table(0, q) * per_stage + pos] = a;
                    hp[table(1, q) * per_stage + pos] = b;
                }
                hp[table(2, 0) * per_stage + pos] = s3;
                hp[table(3, 0) * per_stage + pos] = s4;
                ++pos;
            }
            m[c.items.size()] = acc;
            blocks.push_back(acc);
        }
        items_dev.alloc(hp.size() * sizeof(HopParams));
        meta_dev.alloc(meta.size() * sizeof(int));
        DWF_HIP(hipMemcpy(items_dev.p, hp.data(), hp.size() * sizeof(HopParams), hipMemcpyHostToDevice));
        DWF_HIP(hipMemcpy(meta_dev.p, meta.data(), meta.size() * sizeof(int), hipMemcpyHostToDevice));
    }

    void stage(int sidx, int q, hipStream_t st) const {
        size_t first = 0;
        for (size_t ci = 0; ci < classes.size(); ++ci) {
            const HopParams* it = items_dev.as<HopParams>() + table(sidx, q) * per_stage + first;
            const int* m = meta_dev.as<int>() + ci * meta_per_class;
            launch_hop_batch(kind, classes[ci].KK, it, m, (int)classes[ci].items.size(), blocks[ci], nrb, order,
                             stage_loc[sidx], classes[ci].pm[sidx], classes[ci].ek[sidx], st);
            first += classes[ci].items.size();
        }
    }
};

// all device state of one batched solve
struct Batch {
    std::vector<Item> items;
    std::vector<SlotDesc> slots;
    long N = 0;          // complex elements of one batch vector
    long pstride = 0;    // partials per slot
    int vblocks = 0;     // vector-kernel blocks of a slot-table launch
    int nslots = 0;
    DevBuf slots_dev, partial, scal, inner_tol2;
};

void make_batch(Batch& B, int n, const dwf_op* const* ops, const int* nrhs) {
    int slot = 0;
    long off = 0;
    long pst = 1;
    for (int i = 0; i < n; ++i) {
        const dwf_op* op = ops[i];
        DWF_REQUIRE(op, DWF_EINVAL, "null operator in batch");
        DWF_REQUIRE(op->lat->has_gauge, DWF_ESTATE, "gauge field not set");
        DWF_REQUIRE(nrhs[i] >= 1 && nrhs[i] <= 4096, DWF_EINVAL, "nrhs out of range");
        Item it;
        it.op = op;
        it.nrhs = nrhs[i];
        it.slot0 = slot;
        it.off = off;
        it.n1 = (long)op->Ls * 12 * op->lat->Vhp;
        for (int r = 0; r < it.nrhs; ++r) {
            SlotDesc d{};
            d.off = off + r * it.n1;
            d.n = it.n1;
            d.nb = slot_blocks(it.n1);
            d.block0 = B.vblocks;
            d.nhop = hop_grid_blocks(op->lat->Vh);
            d.Vhp = op->lat->Vhp;
            B.vblocks += d.nb;
            pst = std::max<long>(pst, std::max(d.nb, d.nhop));
            B.slots.push_back(d);
        }
        slot += it.nrhs;
        off += it.n1 * it.nrhs;
        B.items.push_back(it);
    }
    B.N = off;
    B.nslots = slot;
    B.pstride = pst;
    B.slots_dev.alloc(B.slots.size() * sizeof(SlotDesc));
    DWF_HIP(hipMemcpy(B.slots_dev.p, B.slots.data(), B.slots.size() * sizeof(SlotDesc), hipMemcpyHostToDevice));
    B.partial.alloc((size_t)B.pstride * B.nslots * sizeof(double));
    B.scal.alloc((size_t)B.nslots * CG_NSLOTS * sizeof(double));
    B.inner_tol2.alloc((size_t)B.nslots * sizeof(double));
}

// Inner CG state.  The search directions of a check period go to a ring of
// `ring` batch vectors with their alphas (one per slot and ring slot); x is
// formed from them when the ring fills and at the end of the period, in the
// order of the iterations, so it matches x += alpha p per iteration bit for bit.
struct Inner {
    int kx, kp, ring;
    size_t bp;   // bytes of one ring slot (one batch vector of storage kp)
    DevBuf x, r, p, t, v, alph;
    NormalHops hops;
    GraphExec graph;
    int graph_k = 0;
    Inner(const Batch& B, int kx_, int kp_, int ring_) : kx(kx_), kp(kp_), ring(ring_) {
        const size_t bx = complex_bytes_of(kx) * B.N;
        bp = complex_bytes_of(kp) * B.N;
        x.alloc(bx);
        r.alloc(bx);
        p.alloc(bp * ring);
        t.alloc(bp);
        v.alloc(bp);
        alph.alloc(sizeof(double) * B.nslots * ring);
    }
    void* pslot(int q) const { return static_cast<char*>(p.p) + (size_t)q * bp; }
    void build_hops(const Batch& B, int nrb, int order) {
        hops.build(B.items, kp, nrb, order, p.p, bp, ring, t.p, v.p, r.p, B.partial.as<double>(), B.pstride,
                   B.scal.as<double>());
    }
};

// ring length for a check period of k iterations and ring slots of bp bytes
int ring_length(int k, size_t bp) { return std::min(k, ring_slots(bp)); }

// iteration q (0-based) of a check period of k iterations, over every slot
void iteration(const Batch& B, Inner& I, int q, int k, hipStream_t st) {
    const SlotDesc* sd = B.slots_dev.as<SlotDesc>();
    double* pp = B.partial.as<double>();
    double* sc = B.scal.as<double>();
    const int pos = q % I.ring;
    I.hops.stage(0, pos, st);
    I.hops.stage(1, pos, st);
    bfinalize(pp, B.pstride, sd, B.nslots, sc, 1, 1, nullptr, st, I.alph.as<double>() + pos, I.ring);
    I.hops.stage(2, pos, st);
    I.hops.stage(3, pos, st);   // r -= alpha D^dag D^ p, |r|^2 partials per hop tile
    bfinalize(pp, B.pstride, sd, B.nslots, sc, 2, 1, nullptr, st, nullptr, 0, k);
    // the next direction starts a new ring when this one fills it or the period ends:
    // x takes the ring's directions first
    const int next = q + 1 == k ? 0 : (pos + 1) % I.ring;
    if (next == 0)
        bcg_accx(I.kx, I.kp, I.x.p, I.p.p, B.N, I.alph.as<double>(), I.ring, pos + 1, sd, B.nslots, B.vblocks, st);
    bcg_p2(I.kx, I.kp, I.pslot(next), I.pslot(pos), I.r.p, sd, B.nslots, B.vblocks, sc, st);
}

void capture(const Batch& B, Inner& I, int k, hipStream_t cs) {
    I.graph.reset();
    DWF_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
        for (int q = 0; q < k; ++q) iteration(B, I, q, k, cs);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    DWF_HIP(hipStreamEndCapture(cs, &I.graph.g));
    DWF_HIP(hipGraphInstantiate(&I.graph.x, I.graph.g, nullptr, nullptr, 0));
    I.graph_k = k;
}

// times the four hops of D^dag D^ for one (nrb, order)
double time_hops(const Batch& B, Inner& I, int nrb, int order, hipStream_t st) {
    I.build_hops(B, nrb, order);
    Event e0, e1;
    for (int s = 0; s < 4; ++s) I.hops.stage(s, 0, st);
    DWF_HIP(hipEventRecord(e0.e, st));
    const int reps = 5;
    for (int q = 0; q < reps; ++q)
        for (int s = 0; s < 4; ++s) I.hops.stage(s, 0, st);
    DWF_HIP(hipEventRecord(e1.e, st));
    DWF_HIP(hipEventSynchronize(e1.e));
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    return ms / reps;
}

// candidate RHS-per-block values for the largest nrhs of the batch
std::vector<int> nrb_candidates(const Batch& B) {
    int mx = 1;
    for (const Item& it : B.items) mx = std::max(mx, it.nrhs);
    std::vector<int> c;
    for (int v : {1, 2, 3, 4, 6, 8, 12, 16})
        if (v <= mx) c.push_back(v);
    return c;
}

void choose_tiles(const Batch& B, Inner& I, int autotune, hipStream_t st, int* nrb, int* order, double* best_ms) {
    const std::string key = tune_key(B.items, I.kp);
    *nrb = 1;
    *order = 0;
    *best_ms = 0.0;
    if (autotune < 2 && tune_get(key, nrb, order, best_ms)) return;
    if (autotune == 0) return;
    // the done flags must read "active" while timing
    DWF_HIP(hipMemsetAsync(B.scal.p, 0, (size_t)B.nslots * CG_NSLOTS * sizeof(double), st));
    double best = 1e300;
    for (int nb : nrb_candidates(B))
        for (int od = 0; od < 2; ++od) {
            if (nb == 1 && od == 1) {
                int mx = 1;
                for (const Item& it : B.items) mx = std::max(mx, it.nrhs);
                if (mx == 1) continue;   // same schedule as order 0
            }
            const double ms = time_hops(B, I, nb, od, st);
            if (trace_on())
                std::fprintf(stderr, "dwf trace: tune %s nrb %d order %d four hops %.4f ms\n", key.c_str(), nb, od, ms);
            if (ms < best) {
                best = ms;
                *nrb = nb;
                *order = od;
            }
        }
    *best_ms = best;
    tune_put(key, *nrb, *order, best);
}

}  // namespace

// public: explicit tuning (returns the choice and the time of the four hops)
void autotune_batch(int n, const dwf_op* const* ops, const int* nrhs, int kp, int force, int* nrb, int* order,
                    double* ms, hipStream_t st) {
    DWF_REQUIRE(n >= 1 && ops && nrhs, DWF_EINVAL, "empty batch");
    DWF_REQUIRE(kp == ST_F64 || kp == ST_F32 || kp == ST_BF16, DWF_EINVAL, "bad precision");
    Batch B;
    make_batch(B, n, ops, nrhs);
    Inner I(B, kp == ST_F64 ? ST_F64 : ST_F32, kp, 1);
    choose_tiles(B, I, force ? 2 : 1, st, nrb, order, ms);
    DWF_HIP(hipStreamSynchronize(st));
}

int solve_batch(int n, const dwf_op* const* ops, void* const* x5, const void* const* b5, const int* nrhs,
                const dwf_solve_params* prm, dwf_solve_info* infos, hipStream_t user_st) {
    DWF_REQUIRE(n >= 1 && ops && x5 && b5 && nrhs && prm, DWF_EINVAL, "null argument");
    DWF_REQUIRE(prm->algo == DWF_ALGO_CGNR || prm->algo == DWF_ALGO_DC, DWF_EINVAL,
                "batched solves support DWF_ALGO_CGNR and DWF_ALGO_DC");
    DWF_REQUIRE(!prm->paper_mode, DWF_EINVAL, "paper_mode is not available for batched solves");
    for (int i = 0; i < n; ++i) DWF_REQUIRE(x5[i] && b5[i], DWF_EINVAL, "null field pointer");
    Batch B;
    make_batch(B, n, ops, nrhs);
    const long N = B.N;
    const size_t b64 = 16 * (size_t)N;
    DevBuf be(b64), bo(b64), bt(b64), xe(b64), xo(b64), rh(b64), te(b64), to(b64), tmp(b64);
    int kp = prm->algo == DWF_ALGO_DC ? prm->inner_prec : ST_F64;
    DWF_REQUIRE(kp == ST_F64 || kp == ST_F32 || kp == ST_BF16, DWF_EINVAL, "bad inner precision");
    const double tol = prm->tol > 0 ? prm->tol : 1e-10;
    const int maxiter = prm->maxiter > 0 ? prm->maxiter : 100000;
    const int check_every = std::max(1, prm->check_every);
    auto inner_tol_of = [&](int k) {
        if (prm->inner_tol > 0 && k == kp) return prm->inner_tol;
        return k == ST_F64 ? tol : (k == ST_F32 ? 1e-5 : 3e-2);
    };
    const int ring = ring_length(check_every, complex_bytes_of(kp) * (size_t)B.N);
    std::unique_ptr<Inner> I(new Inner(B, kp == ST_F64 ? ST_F64 : ST_F32, kp, ring));
    const int ns = B.nslots;
    PinnedD hs((size_t)ns * CG_NSLOTS);
    std::vector<int> odone(ns, 0);
    std::vector<double> req(ns, 0.0), fr(ns, 1.0);
    PinnedD itol2_h(ns);

    Stream cs;
    Event ev_in, e0, e1;
    // tile choice (may time kernels) before the timed region
    int nrb = 1, order = 0;
    double tms = 0;
    const int autotune = prm->autotune;
    choose_tiles(B, *I, autotune, cs.s, &nrb, &order, &tms);
    I->build_hops(B, nrb, order);

    const SlotDesc* sd = B.slots_dev.as<SlotDesc>();
    double* pp = B.partial.as<double>();
    double* sc = B.scal.as<double>();
    auto read_scal = [&]() {
        DWF_HIP(hipMemcpyAsync(hs.h, sc, sizeof(double) * ns * CG_NSLOTS, hipMemcpyDeviceToHost, cs.s));
        DWF_HIP(hipStreamSynchronize(cs.s));
    };
    auto slot_norms = [&](int kind, const void* f, std::vector<double>& out) {
        bnorm2(kind, f, sd, ns, B.vblocks, pp, B.pstride, sc, cs.s);
        bfinalize(pp, B.pstride, sd, ns, sc, 4, 0, nullptr, cs.s);
        read_scal();
        out.resize(ns);
        for (int v = 0; v < ns; ++v) out[v] = hs.h[(size_t)v * CG_NSLOTS + CG_TMP];
    };
    auto at = [](void* base, long off) { return static_cast<char*>(base) + 16 * (size_t)off; };

    DWF_HIP(hipEventRecord(ev_in.e, user_st));
    DWF_HIP(hipStreamWaitEvent(cs.s, ev_in.e, 0));
    DWF_HIP(hipEventRecord(e0.e, cs.s));
    DWF_HIP(hipMemsetAsync(B.scal.p, 0, (size_t)ns * CG_NSLOTS * sizeof(double), cs.s));
    for (const Item& it : B.items) {
        const dwf_lattice* L = it.op->lat;
        const int* lex = L->lex_of_site_dev.as<int>();
        const long sl = (long)it.op->Ls * it.nrhs;
        const void* src = b5[&it - B.items.data()];
        pack_full(ST_F64, at(be.p, it.off), src, lex, L->Vh, L->Vhp, L->V, sl, cs.s);
        pack_full(ST_F64, at(bo.p, it.off), src, lex + L->Vh, L->Vh, L->Vhp, L->V, sl, cs.s);
        schur_rhs(it.op, ST_F64, at(bt.p, it.off), at(be.p, it.off), at(bo.p, it.off), at(to.p, it.off), it.nrhs,
                  cs.s);
    }
    std::vector<double> b2e, b2o, b2(ns), rel5(ns, 1.0), prev(ns, 1e300), t2;
    slot_norms(ST_F64, be.p, b2e);
    slot_norms(ST_F64, bo.p, b2o);
    for (int v = 0; v < ns; ++v) {
        b2[v] = b2e[v] + b2o[v];
        if (b2[v] == 0.0) { odone[v] = 1; rel5[v] = 0.0; }
    }
    DWF_HIP(hipMemsetAsync(xe.p, 0, b64, cs.s));
    convert(ST_F64, ST_F64, rh.p, bt.p, N, cs.s);

    std::vector<int> iters(ns, 0), outer(ns, 0);
    std::vector<double> inner_rel(ns, 0.0);
    int fallback = 0;
    bool nan_seen = false;
    // Items run their defect-correction steps independently: after each
    // replay, an item whose slots are all done takes its FP64 outer step at
    // once and restarts its inner solve, while the others keep iterating.
    // Item state: 0 idle (inner start due), 1 inner solve running, 2 finished.
    const int nitems = (int)B.items.size();
    std::vector<int> state(nitems, 0), finished0;
    for (int i = 0; i < nitems; ++i) {
        bool all = true;
        for (int v = B.items[i].slot0; v < B.items[i].slot0 + B.items[i].nrhs; ++v) all = all && odone[v] != 0;
        if (all) {
            state[i] = 2;
            finished0.push_back(i);
        }
    }
    // te is reduced per slot after every outer step, also where no item
    // has written it yet: it starts at zero
    DWF_HIP(hipMemsetAsync(te.p, 0, b64, cs.s));
    auto xat = [&](const Item& it) { return static_cast<char*>(I->x.p) + complex_bytes_of(I->kx) * it.off; };
    auto rat = [&](const Item& it) { return static_cast<char*>(I->r.p) + complex_bytes_of(I->kx) * it.off; };
    // inner starts of the items in `start` (r = D^dag r^ in FP64, then stored
    // in kx; p = r; x = 0) and retirement of the items in `retire`; every
    // other slot keeps its state (target 0 to the mode-0 finalize)
    auto restart = [&](const std::vector<int>& start, const std::vector<int>& retire) {
        for (int v = 0; v < ns; ++v) itol2_h.h[v] = 0.0;
        const double itol = inner_tol_of(I->kp);
        for (int i : start) {
            const Item& it = B.items[i];
            apply_dhat(it.op, ST_F64, 1, at(te.p, it.off), at(rh.p, it.off), at(to.p, it.off), at(tmp.p, it.off),
                       it.nrhs, cs.s);
            convert(I->kx, ST_F64, rat(it), at(te.p, it.off), it.n1 * it.nrhs, cs.s, it.op->lat->Vhp);
            convert(I->kp, I->kx, static_cast<char*>(I->pslot(0)) + complex_bytes_of(I->kp) * it.off, rat(it),
                    it.n1 * it.nrhs, cs.s, it.op->lat->Vhp);
            DWF_HIP(hipMemsetAsync(xat(it), 0, complex_bytes_of(I->kx) * it.n1 * it.nrhs, cs.s));
            for (int v = it.slot0; v < it.slot0 + it.nrhs; ++v) {
                const bool plain = I->kp == ST_F64 && outer[v] == 0;
                req[v] = plain ? itol : dc_target(tol, rel5[v], I->kp, itol, fr[v]);
                itol2_h.h[v] = odone[v] ? -1.0 : req[v] * req[v];
            }
            state[i] = 1;
        }
        for (int i : retire)
            for (int v = B.items[i].slot0; v < B.items[i].slot0 + B.items[i].nrhs; ++v) itol2_h.h[v] = -1.0;
        DWF_HIP(hipMemcpyAsync(B.inner_tol2.p, itol2_h.h, sizeof(double) * ns, hipMemcpyHostToDevice, cs.s));
        bnorm2(I->kx, I->r.p, sd, ns, B.vblocks, pp, B.pstride, sc, cs.s);
        bfinalize(pp, B.pstride, sd, ns, sc, 0, 0, B.inner_tol2.as<double>(), cs.s);
    };
    auto idle_items = [&]() {
        std::vector<int> v;
        for (int i = 0; i < nitems; ++i) if (state[i] == 0) v.push_back(i);
        return v;
    };
    const bool use_graph = prm->use_graph != 0;
    restart(idle_items(), finished0);
    bool want_fallback = false;
    for (;;) {
        if (std::none_of(state.begin(), state.end(), [](int q) { return q == 1; })) break;
        if (use_graph && I->graph_k != check_every) capture(B, *I, check_every, cs.s);
        if (use_graph) DWF_HIP(hipGraphLaunch(I->graph.x, cs.s));
        else
            for (int q = 0; q < check_every; ++q) iteration(B, *I, q, check_every, cs.s);
        read_scal();
        std::vector<int> ready;
        for (int i = 0; i < nitems; ++i) {
            if (state[i] != 1) continue;
            bool all = true, over = false;
            for (int v = B.items[i].slot0; v < B.items[i].slot0 + B.items[i].nrhs; ++v) {
                const double* s = hs.h + (size_t)v * CG_NSLOTS;
                if (s[CG_NANFLAG] != 0.0) nan_seen = true;
                if (s[CG_DONE] == 0.0) all = false;
                if (!odone[v] && iters[v] + (int)s[CG_ITERS] >= maxiter) over = true;
            }
            // x is whole after every replay, so an item over its iteration
            // budget takes its outer step too
            if (all || over) ready.push_back(i);
        }
        if (nan_seen) break;
        if (ready.empty()) continue;
        for (int i : ready) {
            const Item& it = B.items[i];
            for (int v = it.slot0; v < it.slot0 + it.nrhs; ++v) {
                const double* s = hs.h + (size_t)v * CG_NSLOTS;
                if (odone[v]) continue;
                iters[v] += (int)s[CG_ITERS];
                outer[v] += 1;
                inner_rel[v] = s[CG_RR0] > 0 ? std::sqrt(s[CG_RR] / s[CG_RR0]) : 0.0;
            }
            // x^ += x; r^ = b~ - D^ x^; 5D residual |M r^| / |b5|
            axpby(ST_F64, I->kx, at(xe.p, it.off), xat(it), it.n1 * it.nrhs, nullptr, 1.0, nullptr, 1.0, nullptr,
                  cs.s, it.op->lat->Vhp);
            apply_dhat(it.op, ST_F64, 0, at(te.p, it.off), at(xe.p, it.off), at(to.p, it.off), nullptr, it.nrhs,
                       cs.s);
            convert(ST_F64, ST_F64, at(rh.p, it.off), at(bt.p, it.off), it.n1 * it.nrhs, cs.s);
            axpby(ST_F64, ST_F64, at(rh.p, it.off), at(te.p, it.off), it.n1 * it.nrhs, nullptr, -1.0, nullptr, 1.0,
                  nullptr, cs.s);
            mix(it.op, ST_F64, at(rh.p, it.off), at(te.p, it.off), MAT_M, nullptr, it.nrhs, cs.s);
        }
        slot_norms(ST_F64, te.p, t2);   // all slots; only the ready items' are used
        std::vector<int> retire;
        for (int i : ready) {
            const Item& it = B.items[i];
            bool all_done = true, spent = false;
            for (int v = it.slot0; v < it.slot0 + it.nrhs; ++v) {
                if (odone[v]) continue;
                const double old5 = rel5[v];
                rel5[v] = std::sqrt(t2[v] / b2[v]);
                fr[v] = dc_ratio(rel5[v] / old5, req[v]);
                if (trace_on())
                    std::fprintf(stderr,
                                 "dwf trace: batch step %d slot %d prec %d requested %.3e iters %d rel5 %.3e\n",
                                 outer[v], v, I->kp, req[v], iters[v], rel5[v]);
                if (rel5[v] <= tol) odone[v] = 1;
                else if (rel5[v] > 0.5 * prev[v] && I->kp != ST_F64) want_fallback = true;
                prev[v] = rel5[v];
                if (!odone[v]) all_done = false;
                if (iters[v] >= maxiter || outer[v] >= 100) spent = true;
            }
            state[i] = (all_done || spent) ? 2 : 0;
            if (state[i] == 2) retire.push_back(i);
        }
        std::vector<int> start;
        if (!want_fallback) {
            start = idle_items();
        } else if (std::none_of(state.begin(), state.end(), [](int q) { return q == 1; })) {
            // step the inner storage up one precision once no item is running
            const int nk = I->kp == ST_BF16 ? ST_F32 : ST_F64;
            I.reset(new Inner(B, nk == ST_F64 ? ST_F64 : ST_F32, nk, ring));
            I->build_hops(B, nrb, order);
            fallback = 1;
            want_fallback = false;
            start = idle_items();
        }
        if (!start.empty() || !retire.empty()) restart(start, retire);
    }
    for (const Item& it : B.items) {
        const dwf_lattice* L = it.op->lat;
        const int* lex = L->lex_of_site_dev.as<int>();
        const long sl = (long)it.op->Ls * it.nrhs;
        void* dst = x5[&it - B.items.data()];
        reconstruct_odd(it.op, ST_F64, at(xo.p, it.off), at(xe.p, it.off), at(bo.p, it.off), it.nrhs, cs.s);
        unpack_full(ST_F64, dst, at(xe.p, it.off), lex, L->Vh, L->Vhp, L->V, sl, cs.s);
        unpack_full(ST_F64, dst, at(xo.p, it.off), lex + L->Vh, L->Vh, L->Vhp, L->V, sl, cs.s);
    }
    DWF_HIP(hipEventRecord(e1.e, cs.s));
    // FP64 true 5D residual per slot (outside the timed region)
    for (const Item& it : B.items)
        apply_full(it.op, ST_F64, 0, at(te.p, it.off), at(to.p, it.off), at(xe.p, it.off), at(xo.p, it.off), it.nrhs,
                   cs.s);
    axpby(ST_F64, ST_F64, te.p, be.p, N, nullptr, 1.0, nullptr, -1.0, nullptr, cs.s);
    axpby(ST_F64, ST_F64, to.p, bo.p, N, nullptr, 1.0, nullptr, -1.0, nullptr, cs.s);
    std::vector<double> r2e, r2o;
    slot_norms(ST_F64, te.p, r2e);
    slot_norms(ST_F64, to.p, r2o);
    float ms = 0;
    DWF_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
    // the caller's stream continues after the batch
    DWF_HIP(hipEventRecord(ev_in.e, cs.s));
    DWF_HIP(hipStreamWaitEvent(user_st, ev_in.e, 0));
    DWF_HIP(hipStreamSynchronize(cs.s));
    bool all_ok = true;
    for (int v = 0; v < ns; ++v) {
        const double tr = b2[v] > 0 ? std::sqrt((r2e[v] + r2o[v]) / b2[v]) : 0.0;
        const bool conv = odone[v] != 0 || tr <= tol;
        all_ok = all_ok && conv;
        if (infos) {
            dwf_solve_info& f = infos[v];
            f.iters = iters[v];
            f.outer_iters = outer[v];
            f.fallback_used = fallback;
            f.converged = conv ? 1 : 0;
            f.true_res5 = tr;
            f.seconds = ms * 1e-3;
            f.final_rel_res_even = inner_rel[v];
            f.final_inner_prec = I->kp;
        }
    }
    if (nan_seen) throw Error{DWF_ENAN, "NaN/Inf in a batched CG reduction"};
    return all_ok ? DWF_OK : DWF_NOT_CONVERGED;
}

}  // namespace dwf
