// Lattice geometry, gauge-link packing and operator coefficient setup.
#include <algorithm>
#include <cmath>
#include <complex>
#include <utility>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "dwf_internal.h"
#include "precision.h"

namespace dwf {

using cd = std::complex<double>;

static uint16_t host_f32_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// Internal site order.  Two orders exist; both are bijections onto the
// sites of each parity, and every kernel goes through the site and
// neighbour tables, so the choice only changes cache behaviour.
//
// "brick": the spatial volume is cut into bricks and every brick is swept
// in t (brick index slowest, then t, z, y, x).  With bricks of the whole
// spatial volume this is the lexicographic order.  Smaller bricks keep the
// t neighbours of the sites a GPU die has in flight inside its L2 (a t slice
// of 24^3 sites is ~10 MB of FP32 input at Ls = 16, beyond an XCD's 4 MB L2)
// at the cost of re-reading brick faces.  Measured on MI355X (fused hop,
// Ls = 16): on 16^3x32 bricks of 1024 sites per slice beat whole slices
// (FP64 193 -> 185 us, FP32 84 -> 78 us); on 24^3x48 bricks of 4096 sites
// are best (FP32 479 us vs 519 us at 2048 and 546 us at 1024; larger bricks
// are slower: 440 us vs 459 us at 8192 and 501 us for whole slices).
// Brick limit: 1024 sites up to 16^3 spatial sites, 4096 above
// ($DWF_BRICK_SITES overrides).
//
// "tcol": t columns.  The sites of one parity at one spatial position (every
// other t) are consecutive, so a block of 16 sites is (most of) one t
// column: its t neighbours are the column of the other parity at the same
// position, and each spatial neighbour direction maps the block onto one
// column of a neighbouring position.  Spatial positions are visited octant
// by octant (one octant per XCD under the block remap of the hop), tile by
// tile inside an octant and x-fastest inside a tile, so that the columns a
// die reads are re-read while they are still in its L2.  Tile extents
// ($DWF_TCOL_TILE="tx,ty,tz", default 4,4,4) are shrunk to divide the
// octant; $DWF_TCOL_CURVE=morton visits an octant's positions along the
// Morton (bit-interleaved) curve instead of by tiles.
static void choose_brick(const int dims[4], int b[3]) {
    b[0] = dims[0];
    b[1] = dims[1];
    b[2] = dims[2];
    long fmax = (long)dims[0] * dims[1] * dims[2] <= 4096 ? 1024L : 4096L;   // sites (both parities) per brick slice
    if (const char* e = std::getenv("DWF_BRICK_SITES")) {
        const long v = std::atol(e);
        if (v >= 8) fmax = v;
    }
    while ((long)b[0] * b[1] * b[2] > fmax) {
        int best = -1;
        for (int mu = 2; mu >= 0; --mu)   // prefer z, then y, then x on ties
            if (b[mu] % 4 == 0 && (best < 0 || b[mu] > b[best])) best = mu;
        if (best < 0) break;
        b[best] /= 2;
    }
}

static int site_order_kind() {
    const char* e = std::getenv("DWF_SITE_ORDER");
    if (e && std::strcmp(e, "tcol") == 0) return 1;
    return 0;
}

static int gcd_int(int a, int b) {
    while (b) { const int t = a % b; a = b; b = t; }
    return a;
}

// spatial positions (x, y, z) in the visiting order of the t-column order
static std::vector<int> tcol_spatial_order(const int dims[4]) {
    int oct[3], tile[3] = {4, 4, 4};
    if (const char* e = std::getenv("DWF_TCOL_TILE")) {
        int a = 0, b = 0, c = 0;
        if (std::sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0) {
            tile[0] = a; tile[1] = b; tile[2] = c;
        }
    }
    for (int mu = 0; mu < 3; ++mu) {
        oct[mu] = dims[mu] % 2 == 0 && dims[mu] >= 4 ? dims[mu] / 2 : dims[mu];
        tile[mu] = gcd_int(oct[mu], tile[mu]);
    }
    std::vector<int> order;
    order.reserve((size_t)dims[0] * dims[1] * dims[2]);
    const char* curve = std::getenv("DWF_TCOL_CURVE");
    if (curve && std::strcmp(curve, "morton") == 0) {
        // inside each octant, positions sorted by the Morton code of their
        // octant-relative coordinates (bit-interleaved x, y, z)
        auto morton = [](unsigned x, unsigned y, unsigned z) {
            unsigned long long code = 0;
            for (int bit = 0; bit < 10; ++bit)
                code |= ((unsigned long long)((x >> bit) & 1u) << (3 * bit)) |
                        ((unsigned long long)((y >> bit) & 1u) << (3 * bit + 1)) |
                        ((unsigned long long)((z >> bit) & 1u) << (3 * bit + 2));
            return code;
        };
        for (int oz = 0; oz < dims[2]; oz += oct[2])
            for (int oy = 0; oy < dims[1]; oy += oct[1])
                for (int ox = 0; ox < dims[0]; ox += oct[0]) {
                    std::vector<std::pair<unsigned long long, int>> v;
                    for (int z = oz; z < oz + oct[2]; ++z)
                        for (int y = oy; y < oy + oct[1]; ++y)
                            for (int x = ox; x < ox + oct[0]; ++x)
                                v.push_back({morton(x - ox, y - oy, z - oz), x + dims[0] * (y + dims[1] * z)});
                    std::sort(v.begin(), v.end());
                    for (const auto& e : v) order.push_back(e.second);
                }
        return order;
    }
    for (int oz = 0; oz < dims[2]; oz += oct[2])
        for (int oy = 0; oy < dims[1]; oy += oct[1])
            for (int ox = 0; ox < dims[0]; ox += oct[0])
                for (int tz = oz; tz < oz + oct[2]; tz += tile[2])
                    for (int ty = oy; ty < oy + oct[1]; ty += tile[1])
                        for (int tx = ox; tx < ox + oct[0]; tx += tile[0])
                            for (int z = tz; z < tz + tile[2]; ++z)
                                for (int y = ty; y < ty + tile[1]; ++y)
                                    for (int x = tx; x < tx + tile[0]; ++x)
                                        order.push_back(x + dims[0] * (y + dims[1] * z));
    return order;
}

void build_geometry(dwf_lattice* L) {
    const int Lx = L->dims[0], Ly = L->dims[1], Lz = L->dims[2], Lt = L->dims[3];
    const long V = L->V, Vh = L->Vh;
    choose_brick(L->dims, L->brick);
    L->site_order = site_order_kind();
    // row stride: 32 x odd, so consecutive rows of a field land in different cache sets
    L->Vhp = ((Vh + 31) / 32) * 32;
    if ((L->Vhp / 32) % 2 == 0) L->Vhp += 32;
    const long Vhp = L->Vhp;
    const int bx = L->brick[0], by = L->brick[1], bz = L->brick[2];
    L->lex_of_site.assign(2 * Vh, -1);
    std::vector<int> site_of_lex(V, -1);
    long next[2] = {0, 0};
    auto place = [&](int x, int y, int z, int t) {
        const int p = (x + y + z + t) & 1;
        const long lex = x + (long)Lx * (y + (long)Ly * (z + (long)Lz * t));
        const long i = next[p]++;
        L->lex_of_site[p * Vh + i] = (int)lex;
        site_of_lex[lex] = (int)i;
    };
    if (L->site_order == 1) {
        for (const int pos : tcol_spatial_order(L->dims)) {
            const int x = (int)(pos % Lx), y = (int)((pos / Lx) % Ly), z = (int)(pos / ((long)Lx * Ly));
            for (int t = 0; t < Lt; ++t) place(x, y, z, t);
        }
    } else {
        for (int zb = 0; zb < Lz / bz; ++zb)
            for (int yb = 0; yb < Ly / by; ++yb)
                for (int xb = 0; xb < Lx / bx; ++xb)
                    for (int t = 0; t < Lt; ++t)
                        for (int z = zb * bz; z < (zb + 1) * bz; ++z)
                            for (int y = yb * by; y < (yb + 1) * by; ++y)
                                for (int x = xb * bx; x < (xb + 1) * bx; ++x) place(x, y, z, t);
    }
    DWF_REQUIRE(next[0] == Vh && next[1] == Vh, DWF_EDIMS, "internal site order is not a bijection");
    L->nbr_host.assign(2 * 8 * Vhp, 0);
    const int ext[4] = {Lx, Ly, Lz, Lt};
    for (int p = 0; p < 2; ++p)
        for (long i = 0; i < Vh; ++i) {
            const long x = L->lex_of_site[p * Vh + i];
            int c[4];
            long r = x;
            for (int mu = 0; mu < 4; ++mu) { c[mu] = r % ext[mu]; r /= ext[mu]; }
            for (int d = 0; d < 8; ++d) {
                const int mu = d & 3, dir = d < 4 ? +1 : -1;
                int cc[4] = {c[0], c[1], c[2], c[3]};
                cc[mu] = (cc[mu] + dir + ext[mu]) % ext[mu];
                const long y = cc[0] + (long)Lx * (cc[1] + (long)Ly * (cc[2] + (long)Lz * cc[3]));
                L->nbr_host[(p * 8 + d) * Vhp + i] = site_of_lex[y];
            }
        }
    L->nbr.alloc(sizeof(int) * 2 * 8 * Vhp);
    DWF_HIP(hipMemcpy(L->nbr.p, L->nbr_host.data(), L->nbr.bytes, hipMemcpyHostToDevice));
    L->lex_of_site_dev.alloc(sizeof(int) * 2 * Vh);
    DWF_HIP(hipMemcpy(L->lex_of_site_dev.p, L->lex_of_site.data(), L->lex_of_site_dev.bytes, hipMemcpyHostToDevice));
}

// Hop links per output parity: forward U_mu(x), backward U_mu(x-mu)^dag,
// antiperiodic t phase folded into the links that cross the boundary.
void upload_gauge(dwf_lattice* L, const cd* U) {
    const int ext[4] = {L->dims[0], L->dims[1], L->dims[2], L->dims[3]};
    const long Vh = L->Vh, Vhp = L->Vhp;
    const size_t nl = (size_t)2 * 8 * 9 * Vhp;
    std::vector<cd> hl(nl, cd(0.0, 0.0));
    for (int p = 0; p < 2; ++p)
        for (long i = 0; i < Vh; ++i) {
            const long x = L->lex_of_site[p * Vh + i];
            int c[4];
            long r = x;
            for (int mu = 0; mu < 4; ++mu) { c[mu] = r % ext[mu]; r /= ext[mu]; }
            for (int d = 0; d < 8; ++d) {
                const int mu = d & 3;
                double phase = 1.0;
                const cd* src;
                if (d < 4) {
                    src = U + (x * 4 + mu) * 9;
                    if (mu == 3 && L->antiperiodic_t && c[3] == ext[3] - 1) phase = -1.0;
                } else {
                    int cc[4] = {c[0], c[1], c[2], c[3]};
                    cc[mu] = (cc[mu] - 1 + ext[mu]) % ext[mu];
                    const long y = cc[0] + (long)ext[0] * (cc[1] + (long)ext[1] * (cc[2] + (long)ext[2] * cc[3]));
                    src = U + (y * 4 + mu) * 9;
                    if (mu == 3 && L->antiperiodic_t && c[3] == 0) phase = -1.0;
                }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        cd u = d < 4 ? src[a * 3 + b] : std::conj(src[b * 3 + a]);
                        hl[((size_t)(p * 8 + d) * 9 + a * 3 + b) * Vhp + i] = phase * u;
                    }
            }
        }
    // per storage kind: 16-byte groups of link elements (see precision.h)
    for (int kind : {ST_F64, ST_F32, ST_BF16}) {
        const int cb = (int)complex_bytes(kind);
        const long per = link_elems_parity(Vhp, cb);
        std::vector<double> re(2 * (size_t)per, 0.0), im(2 * (size_t)per, 0.0);
        for (int p = 0; p < 2; ++p)
            for (int d = 0; d < 8; ++d)
                for (int e = 0; e < 9; ++e)
                    for (long i = 0; i < Vh; ++i) {
                        const cd u = hl[((size_t)(p * 8 + d) * 9 + e) * Vhp + i];
                        const size_t k = (size_t)p * per + lidx(d, e, i, Vhp, cb);
                        re[k] = u.real();
                        im[k] = u.imag();
                    }
        const size_t n = 2 * (size_t)per;
        L->links[kind].alloc(n * cb);
        if (kind == ST_F64) {
            std::vector<double> h(2 * n);
            for (size_t k = 0; k < n; ++k) { h[2 * k] = re[k]; h[2 * k + 1] = im[k]; }
            DWF_HIP(hipMemcpy(L->links[kind].p, h.data(), n * cb, hipMemcpyHostToDevice));
        } else if (kind == ST_F32) {
            std::vector<float> h(2 * n);
            for (size_t k = 0; k < n; ++k) { h[2 * k] = (float)re[k]; h[2 * k + 1] = (float)im[k]; }
            DWF_HIP(hipMemcpy(L->links[kind].p, h.data(), n * cb, hipMemcpyHostToDevice));
        } else {
            std::vector<uint16_t> h(2 * n);
            for (size_t k = 0; k < n; ++k) {
                h[2 * k] = host_f32_to_bf16((float)re[k]);
                h[2 * k + 1] = host_f32_to_bf16((float)im[k]);
            }
            DWF_HIP(hipMemcpy(L->links[kind].p, h.data(), n * cb, hipMemcpyHostToDevice));
        }
    }
    L->has_gauge = true;
}

// ---------------------------------------------------------------------
// operator coefficients
// ---------------------------------------------------------------------
static void put_dense(std::vector<double>& buf, int slot, int Ls,
                      const std::vector<double> (&A)[2], const double g5sign[2], double scale) {
    for (int chi = 0; chi < 2; ++chi)
        for (int r = 0; r < Ls; ++r)
            for (int c = 0; c < Ls; ++c)
                buf[(size_t)slot * MAT_ELEMS + (chi * 16 + r) * 16 + c] = scale * g5sign[chi] * A[chi][r * Ls + c];
}

static std::vector<double> transpose(const std::vector<double>& A, int n) {
    std::vector<double> T(n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) T[j * n + i] = A[i * n + j];
    return T;
}

static std::vector<double> mm(const std::vector<double>& A, const std::vector<double>& B, int n) {
    std::vector<double> C(n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) C[i * n + j] += A[i * n + k] * B[k * n + j];
    return C;
}

void setup_op(dwf_op* op) {
    const int Ls = op->Ls;
    op->fd = build_fifth_dim(Ls, op->M0, op->m, op->b, op->c, op->alpha);
    const FifthDim& f = op->fd;
    std::vector<double> h((size_t)NMAT * MAT_ELEMS, 0.0);
    const double one[2] = {1.0, 1.0}, g5[2] = {1.0, -1.0};
    std::vector<double> Qt[2], Mit[2], Kt[2], Mt[2], I[2], MitMinv[2];
    for (int chi = 0; chi < 2; ++chi) {
        Qt[chi] = transpose(f.Q[chi], Ls);
        Mit[chi] = transpose(f.Minv[chi], Ls);
        Kt[chi] = transpose(f.K[chi], Ls);
        Mt[chi] = transpose(f.M[chi], Ls);
        I[chi].assign(Ls * Ls, 0.0);
        for (int s = 0; s < Ls; ++s) I[chi][s * Ls + s] = 1.0;
        MitMinv[chi] = mm(Mit[chi], f.Minv[chi], Ls);
    }
    put_dense(h, MAT_Q, Ls, f.Q, one, 1.0);
    put_dense(h, MAT_QT, Ls, Qt, one, 1.0);
    put_dense(h, MAT_MQMINV, Ls, f.Minv, one, -0.25);
    put_dense(h, MAT_G5MIT, Ls, Mit, g5, 1.0);
    put_dense(h, MAT_G5MIT_MQMINV, Ls, MitMinv, g5, -0.25);
    put_dense(h, MAT_MQG5KT, Ls, Kt, g5, -0.25);
    put_dense(h, MAT_G5MT, Ls, Mt, g5, 1.0);
    put_dense(h, MAT_HALFMINV, Ls, f.Minv, one, 0.5);
    put_dense(h, MAT_MINV, Ls, f.Minv, one, 1.0);
    put_dense(h, MAT_M, Ls, f.M, one, 1.0);
    put_dense(h, MAT_MT, Ls, Mt, one, 1.0);
    put_dense(h, MAT_MHALFI, Ls, I, one, -0.5);
    put_dense(h, MAT_MHALFKTG5, Ls, Kt, g5, -0.5);
    put_dense(h, MAT_IDENT, Ls, I, one, 1.0);
    put_dense(h, MAT_MIT, Ls, Mit, one, 1.0);
    // the source pair (s = 1 and s = Ls as slices 0 and 1):
    // -D_-^(s) y = (c_s / 2) H y + (1 - c_s (4 - M0)) y on each slice
    const double cf = op->c[0], cl = op->c[Ls - 1];
    for (int chi = 0; chi < 2; ++chi) {
        h[(size_t)MAT_CHALF * MAT_ELEMS + (chi * 16 + 0) * 16 + 0] = 0.5 * cf;
        h[(size_t)MAT_CHALF * MAT_ELEMS + (chi * 16 + 1) * 16 + 1] = 0.5 * cl;
        h[(size_t)MAT_SRCLOC * MAT_ELEMS + (chi * 16 + 0) * 16 + 0] = 1.0 - cf * (4.0 - op->M0);
        h[(size_t)MAT_SRCLOC * MAT_ELEMS + (chi * 16 + 1) * 16 + 1] = 1.0 - cl * (4.0 - op->M0);
    }
    op->mats_host = h;

    std::vector<double> pre((size_t)NPRE * PRE_ELEMS, 0.0);
    for (int s = 0; s < Ls; ++s) {
        // K: diagonal and the cyclic neighbour (s-1 for chi 0, s+1 for chi 1)
        const int sm = (s - 1 + Ls) % Ls, sp = (s + 1) % Ls;
        pre[PRE_K * PRE_ELEMS + 0 * 16 + s] = f.K[0][s * Ls + s];
        pre[PRE_K * PRE_ELEMS + 1 * 16 + s] = f.K[1][s * Ls + s];
        pre[PRE_K * PRE_ELEMS + 2 * 16 + s] = f.K[0][s * Ls + sm];
        pre[PRE_K * PRE_ELEMS + 3 * 16 + s] = f.K[1][s * Ls + sp];
        pre[PRE_G5 * PRE_ELEMS + 0 * 16 + s] = 1.0;
        pre[PRE_G5 * PRE_ELEMS + 1 * 16 + s] = -1.0;
    }
    op->mats[0].alloc(h.size() * 8);
    DWF_HIP(hipMemcpy(op->mats[0].p, h.data(), h.size() * 8, hipMemcpyHostToDevice));
    std::vector<float> hf(h.begin(), h.end());
    op->mats[1].alloc(hf.size() * 4);
    DWF_HIP(hipMemcpy(op->mats[1].p, hf.data(), hf.size() * 4, hipMemcpyHostToDevice));
    op->pres[0].alloc(pre.size() * 8);
    DWF_HIP(hipMemcpy(op->pres[0].p, pre.data(), pre.size() * 8, hipMemcpyHostToDevice));
    std::vector<float> pf(pre.begin(), pre.end());
    op->pres[1].alloc(pf.size() * 4);
    DWF_HIP(hipMemcpy(op->pres[1].p, pf.data(), pf.size() * 4, hipMemcpyHostToDevice));
}

}  // namespace dwf
