// Internal declarations of libdwf (host and device).
//
// Internal field layout ("half field"): for one parity, one right-hand side,
//   elem[(s*12 + comp)*Vhp + site], comp = spin*3 + colour, site = internal
// site index of that parity (see build_geometry: spatial bricks of about
// 8^3, swept in t; lex_of_site gives the lexicographic site),
// complex stored as (re, im) pairs of the storage type.  Multi-RHS fields put
// the RHS index outermost: elem[((r*Ls + s)*12 + comp)*Vhp + site].
// Vhp >= Vh is the padded row stride (32 times an odd number): with a
// power-of-two stride every row of a site falls into the same L2 set and
// the hop thrashes the cache by conflict.  Padding entries stay zero.
//
// Links per output parity p ("hop links"):
//   link[((p*8 + d)*9 + row*3 + col)*Vhp + site],
//   d = 0..3: U_mu(x) (forward hop to x+mu), d = 4..7: U_mu(x-mu)^dag,
// with the antiperiodic time phase folded in.
// Neighbours: nbr[(p*8 + d)*Vhp + site] = internal index (other parity) of x+mu
// (d < 4) or x-mu (d >= 4).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dwf.h"

namespace dwf {

// ---------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
    int code;
    std::string msg;
};

#define DWF_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            throw ::dwf::Error{DWF_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define DWF_REQUIRE(cond, code, msg)                                               \
    do {                                                                           \
        if (!(cond)) throw ::dwf::Error{(code), (msg)};                            \
    } while (0)

// ---------------------------------------------------------------------
// device buffer (RAII)
// ---------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n) {
        release();
        if (n == 0) return;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error{DWF_ENOMEM, "hipMalloc(" + std::to_string(n) + " bytes) failed"};
        }
        bytes = n;
        // fields keep zero padding beyond the last site of every row
        e = hipMemset(p, 0, n);
        if (e != hipSuccess) throw Error{DWF_EHIP, "hipMemset failed"};
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------
// fifth-dimension matrices (host FP64), built in fifth_dim.cpp
// ---------------------------------------------------------------------
constexpr int LS_MAX = 16;   // the fused hop pads s to 16 rows (one MFMA tile)

struct FifthDim {
    int Ls = 0;
    // per chirality chi (0: P+ = spins 0,1; 1: P- = spins 2,3), row-major Ls x Ls
    std::vector<double> T[2], M5[2], K[2], N[2], M[2], Minv[2], Q[2];
};
// b, c: the coefficients b_s, c_s of D_+^(s), D_-^(s), s = 0..Ls-1
FifthDim build_fifth_dim(int Ls, double M0, double m, const std::vector<double>& b, const std::vector<double>& c,
                         double alpha);

enum StoreKind { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };

// ---------------------------------------------------------------------
// lattice / operator objects
// ---------------------------------------------------------------------
}  // namespace dwf

struct dwf_lattice {
    int dims[4];
    int antiperiodic_t;
    long V, Vh, Vhp;   // sites, sites per parity, padded row stride
    int brick[3] = {0, 0, 0};       // spatial brick extents of the internal site order
    int site_order = 0;             // 0 bricks swept in t, 1 t columns (build_geometry)
    std::vector<int> lex_of_site;   // host [2][Vh]: lexicographic index of internal site
    std::vector<int> nbr_host;    // host [2][8][Vh]
    dwf::DevBuf nbr;              // device [2][8][Vh]
    dwf::DevBuf lex_of_site_dev;    // device [2][Vh]
    dwf::DevBuf links[3];         // per storage kind: [2][8][9][Vh] complex
    bool has_gauge = false;
};

// Slots of the dense per-chirality s-matrices kept on the device, each
// [2][16][16] in the compute type (zero padded beyond Ls).
enum MatSlot {
    MAT_Q = 0, MAT_QT, MAT_MQMINV, MAT_G5MIT, MAT_G5MIT_MQMINV, MAT_MQG5KT, MAT_G5MT, MAT_HALFMINV,
    MAT_MINV, MAT_M, MAT_MT, MAT_MHALFI, MAT_MHALFKTG5, MAT_IDENT, MAT_CHALF, MAT_SRCLOC, MAT_MIT, NMAT
};
// Slots of the sparse pre-mix coefficient sets, each [d0 | d1 | e0 | e1] x 16.
enum PreSlot { PRE_K = 0, PRE_G5 = 1, NPRE };
constexpr int MAT_ELEMS = 2 * 16 * 16;
constexpr int PRE_ELEMS = 4 * 16;

struct dwf_op {
    dwf_lattice* lat = nullptr;
    int Ls = 0;
    double M0 = 0, m = 0, alpha = 1;
    std::vector<double> b, c;   // b_s, c_s, s = 0..Ls-1 (Sec. 2.2; constant for s-independent (b, c))
    bool any_c() const {
        for (double v : c)
            if (v != 0.0) return true;
        return false;
    }
    dwf::FifthDim fd;
    dwf::DevBuf mats[2];   // compute kind 0: double, 1: float; NMAT * MAT_ELEMS
    dwf::DevBuf pres[2];   // NPRE * PRE_ELEMS
    std::vector<double> mats_host;   // NMAT * MAT_ELEMS, FP64
    // solve workspace kept between solves on this operator (solver.cpp owns
    // the type); solves on one operator run one at a time
    mutable std::shared_ptr<void> solve_ws;
    mutable std::mutex solve_mu;
    const void* mat(int store_kind, int slot) const {
        const int ck = store_kind == dwf::ST_F64 ? 0 : 1;
        const size_t esz = ck == 0 ? 8 : 4;
        return static_cast<const char*>(mats[ck].p) + (size_t)slot * MAT_ELEMS * esz;
    }
    const void* pre(int store_kind, int slot) const {
        const int ck = store_kind == dwf::ST_F64 ? 0 : 1;
        const size_t esz = ck == 0 ? 8 : 4;
        return static_cast<const char*>(pres[ck].p) + (size_t)slot * PRE_ELEMS * esz;
    }
};
