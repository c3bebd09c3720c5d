// Fused half-lattice domain-wall hop with fifth-dimension mixing on MFMA.
//
// One launch computes, for every site x of the output parity p and every s,
//
//   out(x, .) = POST . H(PRE . in)(x, .)  +  LOCMIX . loc(x, .)
//   out2(x,.) = POST2 . H(PRE . in)(x, .) +  LOCMIX2 . loc(x, .)     (optional)
//
// where H is the 4D Wilson hopping term of the paper's Wilson operator
// (Sec. 2.1, eq. Wilson_matrix without the -1/2 and the mass term):
//
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
//              + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu),
//
// applied on every s slice, and POST, LOCMIX, POST2, LOCMIX2 are real Ls x Ls
// matrices acting on s per chirality (the 5D-local algebra of the domain-wall
// operator, Sec. 2.2 and Sec. 2.3).  PRE is either nothing, a diagonal in s,
// or the cyclic bidiagonal pattern of K = (b + c M5) T.
//
// Wave layout (64 lanes): lane = 16 * sc + j, j = site within a group of 16
// consecutive even-odd sites, sc = 0..3; a wave computes the hop for one
// group of 4 slices s = 4 kk + sc (or KPW groups).  Memory access: every
// lane-dependent offset (site, slice) is in the vector offset of a buffer
// load and only wave-uniform offsets are scalar, so no load is serialised
// over lanes; fields hold spin-colour components in 16-byte groups per site
// (FP64 one, FP32 a pair, BF16 a quad), so a wave reads 16 consecutive sites
// of a group with one 128-bit load per lane, and the block's links (also in
// 16-byte groups) are staged once in LDS.  The hop results go to LDS as
// hs[kk][real][lane], which is exactly the B operand of v_mfma_*_16x16x4
// (B[k][n] = lane n + 16 k: k = slice within the group, n = site), so the
// dense s-mixing C = A * h reads each operand with one LDS load per MFMA.
// After the MFMA a lane holds rows s = 4*sc + i, i = 0..3, of the result for
// its site (f32); the f64 MFMA leaves rows sc + 4*i instead (see out_row).
#include <type_traits>
#include "dwf_internal.h"
#include "hop.h"
#include "precision.h"

#include <algorithm>
#include <cstdlib>

namespace dwf {

// Tuning knobs (compile time): occupancy target per precision, 4-slice
// groups per wave in the hop phase (KPW > 1: each link load serves KPW
// groups), unrolling of the direction loop, and whether the 8 neighbour
// indices are loaded up front.  Defaults are the best of sweeps on MI355X:
// one slice group per wave; the single-lattice kernels run the pipelined
// direction loop (below) in FP32 at 4 waves per SIMD (<= 127 VGPRs) and in
// BF16 at 5 (<= 95), FP64 runs the rolled loop at 3 (<= 168); without the
// pipelining, unrolling only lets the compiler hoist the loads of several
// directions and spill.  The work-list kernels, whose pre-mix mode is a
// runtime value, keep 4 waves (FP64: 2).
#ifndef DWF_HOP_WAVES_PER_EU
#define DWF_HOP_WAVES_PER_EU 4
#endif
#ifndef DWF_HOP_BATCHN_WPE
#define DWF_HOP_BATCHN_WPE 4
#endif
#ifndef DWF_HOP_WAVES_PER_EU64
#define DWF_HOP_WAVES_PER_EU64 3
#endif
// FP64 kernels whose pre-mix mode is a runtime value (work lists) or 2
#ifndef DWF_HOP_WAVES_PER_EU64_BATCH
#define DWF_HOP_WAVES_PER_EU64_BATCH 2
#endif
#ifndef DWF_HOP_WAVES_PER_EU16
#define DWF_HOP_WAVES_PER_EU16 5
#endif
#ifndef DWF_HOP_UNROLL
#define DWF_HOP_UNROLL 1
#endif
#ifndef DWF_HOP_KPW
#define DWF_HOP_KPW 1
#endif
#ifndef DWF_HOP_KPW64
#define DWF_HOP_KPW64 1
#endif
#ifndef DWF_HOP_NBR_PRELOAD
#define DWF_HOP_NBR_PRELOAD 1
#endif
// Software pipelining of the direction loop: the neighbour spinors of
// direction d+1 are loaded (raw 16-byte groups, decoded at use) while
// direction d is computed, so every wave keeps one direction's loads in
// flight during its arithmetic instead of exposing the memory latency once
// per direction.  1: a rolled ping-pong loop; 2: the eight directions
// unrolled with compile-time spin structure.  Single-lattice launches only
// (their pre-mix mode is a template constant; with the mode a runtime value
// the extra registers spill).  Measured on 24^3x48, Ls = 16 (hop us):
// FP32 451 (off, 5 waves) / 437 (2, 4 waves) / 469 (2, 5 waves, spills);
// BF16 292 (off) / 266 (2, 5 waves); FP64 spills with it (951 -> 5189) and
// takes 910 at 3 waves without it.
#ifndef DWF_HOP_PREFETCH
#define DWF_HOP_PREFETCH 2
#endif
#ifndef DWF_HOP_PREFETCH64
#define DWF_HOP_PREFETCH64 0
#endif
// Pipelined loop: request the first two directions' neighbour spinors in the
// block prologue, together with the link staging loads, instead of after the
// block barrier that publishes the staged tables.  Measured slower (FP32 hop
// 409 -> 419 us on 24^3x48, Ls = 16): off.
#ifndef DWF_HOP_EARLY
#define DWF_HOP_EARLY 0
#endif
// Staging of the tile's links and neighbour indices with every load issued
// before the first LDS write (1), or as a loop over the block's threads (0:
// the loop waits for each load in turn).  FP32 hop on 24^3x48, Ls = 16:
// 422 -> 409 us; FP64 869 -> 881 us, so FP64 keeps the loop.
#ifndef DWF_HOP_STAGE_BATCH
#define DWF_HOP_STAGE_BATCH 1
#endif
#ifndef DWF_HOP_STAGE_BATCH64
#define DWF_HOP_STAGE_BATCH64 0
#endif
// FP32 chained and update stages: request the local term right after the
// direction loop, before the block barriers (see hop_tile).
#ifndef DWF_HOP_LOC_EARLY32
#define DWF_HOP_LOC_EARLY32 1
#endif
// ... and the update stage its old residual values as well
#ifndef DWF_HOP_UPD_EARLY32
#define DWF_HOP_UPD_EARLY32 1
#endif
// Single-lattice launches of the fused CG stages use kernels compiled for
// their epilogue kind (epilogue_kind below); 0: every launch tests its flags
// at run time.
#ifndef DWF_HOP_EK
#define DWF_HOP_EK 1
#endif
// FP32: stage the dense s-mix matrices in LDS with the links (the second
// phase then reads them from LDS instead of waiting for L2 after the block
// barriers).
#ifndef DWF_HOP_COEF_LDS32
#define DWF_HOP_COEF_LDS32 1
#endif
// FP32: the hop results (hs) in LDS of their own rather than over the staged
// links, which saves one block barrier.  With the staged s-mix matrices a
// block then takes 42.8 KB of LDS, so 3 blocks (12 waves) fit per CU instead
// of 4.  Measured on 24^3x48, Ls = 16: the plain hop unchanged (390 us), the
// DC-FP32 solve 2-3 % faster; the same 3-block cap without the separate
// region gives most of that (the fused CG stages run better with fewer blocks
// in flight per CU), the saved barrier the rest.  Ls = 16 (4-wave blocks)
// only: with 3-wave blocks (Ls = 12) it takes 5 blocks per CU down to 4, and
// a batch of 12 Ls = 12 solves was 2 % slower.
#ifndef DWF_HOP_HS_SEP32
#define DWF_HOP_HS_SEP32 1
#endif
// Cache policy of the streamed accesses (the outputs, the local term and
// the fused update, each touched once): 0 default, 2 non-temporal, so that
// they do not displace the neighbour lines that later tiles re-read from L2.
#ifndef DWF_HOP_NT_STORE
#define DWF_HOP_NT_STORE 2
#endif
#ifndef DWF_HOP_NT_LOAD
#define DWF_HOP_NT_LOAD 2
#endif
// the tile's links and neighbour indices (each read by one block only)
#ifndef DWF_HOP_NT_LINK
#define DWF_HOP_NT_LINK 0
#endif
// Load the phase-2 MFMA A operands once per wave (see hop_tile): 1 when all
// its components share a chirality, 2 also when they straddle the two.
#ifndef DWF_HOP_COEF_HOIST
#define DWF_HOP_COEF_HOIST 2
#endif
// Stage the block's links and neighbour indices in LDS once (all lanes of a
// block need the same 16 sites' links; loaded per lane they would be fetched
// by every slice group of every wave).
#ifndef DWF_HOP_LDS_LINKS
#define DWF_HOP_LDS_LINKS 1
#endif
// FP32/BF16: stage the local-term field of the tile in LDS with 16-byte loads
// at block start, and write the outputs through an LDS tile so that every
// global store is a whole 16-byte group (the MFMA leaves one complex number
// per lane, which would otherwise be written by 2-4 partial stores per group).
// Wave index marked uniform (readfirstlane).  Off: with it the FP64 CG solve
// was measured not bit-reproducible run to run on MI355X (the generated code
// differs in scheduling and register assignment only).
#ifndef DWF_HOP_W_UNIFORM
#define DWF_HOP_W_UNIFORM 0
#endif
#ifndef DWF_HOP_TILE_IO
#define DWF_HOP_TILE_IO 1
#endif
// Local-term tile in LDS for BF16 / FP32 launches.  Off for FP32: its 24 KB
// tile costs a block per CU, and the solve was measured faster without it.
#ifndef DWF_HOP_LOC_LDS16
#define DWF_HOP_LOC_LDS16 1
#endif
#ifndef DWF_HOP_LOC_LDS32
#define DWF_HOP_LOC_LDS32 0
#endif
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <class R> struct Vec4;
template <> struct Vec4<float> { using T = v4f; };
template <> struct Vec4<double> { using T = v4d; };

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma4(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Orders LDS accesses of the lanes of one wave (data passed between lanes
// through LDS without a block barrier): the compiler reasons per lane and
// would otherwise move another lane's read across this lane's write.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row of the 16x16 result held in accumulator slot i of a lane with
// sc = lane / 16 (column = lane % 16 for both).  Measured on gfx950:
// v_mfma_f32_16x16x4f32 keeps rows 4*sc .. 4*sc+3, v_mfma_f64_16x16x4f64
// keeps rows sc, sc+4, sc+8, sc+12.  The A and B operand layouts are the
// same for both: A[m][k] from lane m + 16k, B[k][n] from lane n + 16k.
template <class R>
__device__ __forceinline__ int out_row(int sc, int i) {
    if constexpr (sizeof(R) == 8) return sc + 4 * i;
    else return 4 * sc + i;
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8), and each XCD has its own L2.  Remap so that XCD x sweeps one
// contiguous range of logical blocks: the y/z/t neighbours a block reads
// were then mostly fetched by the same XCD a few blocks earlier.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + j;
}

// ---------------------------------------------------------------------
// One hop direction: h += (1 + SG*gamma_MU) * U * p, spin-projected.
// Chiral basis gamma_mu = [[0, B],[B^dag, 0]] on (upper spins 0,1 | lower 2,3)
// with B = -i sigma_1, -i sigma_2, -i sigma_3, 1 for mu = x, y, z, t:
//   w     = p_up + SG * B p_lo          (half spinor, 2 spins x 3 colours)
//   h_up += U w,   h_lo += SG * B^dag (U w)
// p, h: 12 complex as 24 reals, index (spin*3 + colour)*2 + reim.
// U: 9 complex as 18 reals, index (row*3 + col)*2 + reim.
// kr scales the lower half spinor (a diagonal pre-mix d_lo/d_up whose d_up
// the caller applies to the sum of all directions); 1 otherwise.  The colour
// products are explicit FMA chains: written as re += ur*xr - ui*xi the
// compiler keeps a separate product and an add of the running sum per term.
// ---------------------------------------------------------------------
template <class R> __device__ __forceinline__ R fmad(R a, R b, R c);
template <> __device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <> __device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The direction loop runs over a wave-uniform d; only the spin structure
// depends on mu = d % 4, so the code is split into a projection and a
// reconstruction per mu around common colour products (a switch over all
// eight (mu, sign) variants of the whole update leaves the accumulators in
// different registers per case and costs 24 copies per direction).
//   w = p_up + skr * B_MU p_lo            (skr = SG * kr)
template <int MU, class R>
__device__ __forceinline__ void hop_project(const R* __restrict__ p, R skr, R* __restrict__ w) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R v0r = p[(6 + c) * 2], v0i = p[(6 + c) * 2 + 1];
        const R v1r = p[(9 + c) * 2], v1i = p[(9 + c) * 2 + 1];
        R b0r, b0i, b1r, b1i;
        if constexpr (MU == 0) {        // B v = (-i v1, -i v0)
            b0r = v1i; b0i = -v1r; b1r = v0i; b1i = -v0r;
        } else if constexpr (MU == 1) { // B v = (-v1, v0)
            b0r = -v1r; b0i = -v1i; b1r = v0r; b1i = v0i;
        } else if constexpr (MU == 2) { // B v = (-i v0, i v1)
            b0r = v0i; b0i = -v0r; b1r = -v1i; b1i = v1r;
        } else {                        // B v = v
            b0r = v0r; b0i = v0i; b1r = v1r; b1i = v1i;
        }
        w[c * 2] = fmad(skr, b0r, p[c * 2]);
        w[c * 2 + 1] = fmad(skr, b0i, p[c * 2 + 1]);
        w[(3 + c) * 2] = fmad(skr, b1r, p[(3 + c) * 2]);
        w[(3 + c) * 2 + 1] = fmad(skr, b1i, p[(3 + c) * 2 + 1]);
    }
}
//   h_lo += sg * B_MU^dag u
template <int MU, class R>
__device__ __forceinline__ void hop_reconstruct(const R* __restrict__ u, R sg, R* __restrict__ h) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R u0r = u[c * 2], u0i = u[c * 2 + 1];
        const R u1r = u[(3 + c) * 2], u1i = u[(3 + c) * 2 + 1];
        R* h0 = h + (6 + c) * 2;
        R* h1 = h + (9 + c) * 2;
        if constexpr (MU == 0) {        // (i u1, i u0)
            h0[0] = fmad(-sg, u1i, h0[0]); h0[1] = fmad(sg, u1r, h0[1]);
            h1[0] = fmad(-sg, u0i, h1[0]); h1[1] = fmad(sg, u0r, h1[1]);
        } else if constexpr (MU == 1) { // (u1, -u0)
            h0[0] = fmad(sg, u1r, h0[0]); h0[1] = fmad(sg, u1i, h0[1]);
            h1[0] = fmad(-sg, u0r, h1[0]); h1[1] = fmad(-sg, u0i, h1[1]);
        } else if constexpr (MU == 2) { // (i u0, -i u1)
            h0[0] = fmad(-sg, u0i, h0[0]); h0[1] = fmad(sg, u0r, h0[1]);
            h1[0] = fmad(sg, u1i, h1[0]); h1[1] = fmad(-sg, u1r, h1[1]);
        } else {
            h0[0] = fmad(sg, u0r, h0[0]); h0[1] = fmad(sg, u0i, h0[1]);
            h1[0] = fmad(sg, u1r, h1[0]); h1[1] = fmad(sg, u1i, h1[1]);
        }
    }
}

// h += (1 + SG gamma_mu) U p for a wave-uniform direction d (mu = d % 4,
// SG = -1 for d < 4, +1 otherwise), spin-projected as described above.
template <class R>
__device__ __forceinline__ void hop_dir(int d, const R* __restrict__ U, const R* __restrict__ p,
                                        R* __restrict__ h, R kr) {
    const R sg = d < 4 ? R(-1) : R(1);
    const R skr = sg * kr;
    R w[12];
    switch (d & 3) {   // wave-uniform
        case 0: hop_project<0, R>(p, skr, w); break;
        case 1: hop_project<1, R>(p, skr, w); break;
        case 2: hop_project<2, R>(p, skr, w); break;
        default: hop_project<3, R>(p, skr, w); break;
    }
    R u[12];
#pragma unroll
    for (int hs = 0; hs < 2; ++hs)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R* Ua = U + a * 6;
            const R* x = w + hs * 6;
            R re = Ua[0] * x[0], im = Ua[0] * x[1];
            re = fmad(-Ua[1], x[1], re);
            im = fmad(Ua[1], x[0], im);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                re = fmad(Ua[2 * b], x[2 * b], re);
                re = fmad(-Ua[2 * b + 1], x[2 * b + 1], re);
                im = fmad(Ua[2 * b], x[2 * b + 1], im);
                im = fmad(Ua[2 * b + 1], x[2 * b], im);
            }
            u[(hs * 3 + a) * 2] = re;
            u[(hs * 3 + a) * 2 + 1] = im;
        }
#pragma unroll
    for (int k = 0; k < 12; ++k) h[k] += u[k];   // h_up += U w
    switch (d & 3) {
        case 0: hop_reconstruct<0, R>(u, sg, h); break;
        case 1: hop_reconstruct<1, R>(u, sg, h); break;
        case 2: hop_reconstruct<2, R>(u, sg, h); break;
        default: hop_reconstruct<3, R>(u, sg, h); break;
    }
}

// Pre-mix mode of a launch: a template constant for the single-lattice
// kernel (PM >= 0: the code of the other modes, and the registers it would
// hold, is not generated), the launch parameter for work-list launches
// (PM < 0: the items of one launch may differ).
template <int PM>
__device__ __forceinline__ int pre_mode_of(const HopParams& P) {
    if constexpr (PM >= 0) return PM;
    else return P.pre_mode;
}

// Buffer descriptors of one hop launch (wave-uniform, scalar registers).
struct HopRes {
    __amdgpu_buffer_rsrc_t in, loc, out, out2, upd, links, nbr;
};

template <class S, int G, int PM>
__device__ __forceinline__ void hop_direction(const HopParams& P, const HopRes& R_, unsigned gb, unsigned sx,
                                              int D, unsigned ynb, const int (&s)[G],
                                              const typename Traits<S>::R (&pd)[G][2],
                                              const typename Traits<S>::R (&pe)[G][2],
                                              const typename Traits<S>::R (&kr)[G],
                                              typename Traits<S>::R (&h)[G][24], const u32x4* lnk,
                                              const unsigned* lnbr, int j) {
    using R = typename Traits<S>::R;
    constexpr unsigned CB = cbytes<S>();
    constexpr unsigned NG = link_ng(CB);
    const int Ls = P.Ls;
    const unsigned Vhp = (unsigned)P.Vhp;
    R U[18];
    unsigned y;
    if constexpr (DWF_HOP_LDS_LINKS) {
        y = lnbr[D * 16 + j];
#pragma unroll
        for (unsigned g = 0; g < NG; ++g) decode_link_group<S>(lnk[(D * NG + g) * 16 + j], (int)g, U);
    } else {
        y = DWF_HOP_NBR_PRELOAD ? ynb : __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, sx * 4u, (unsigned)D * Vhp * 4u, 0);
        constexpr unsigned LGB = link_lp(CB) * CB;   // bytes of one link group per site
        bload_link<S>(R_.links, sx * LGB, (unsigned)D * NG * Vhp * LGB, Vhp * LGB, U);
    }
    constexpr int PK = fpack<S>();             // components per group
    constexpr int NGR = 12 / PK;               // groups per slice
    const unsigned yg = y * (unsigned)PK * CB; // byte offset of the neighbour in a group row
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // Slices beyond Ls (Ls not a multiple of 4) read slice 0 (finite
        // values; branch-free, so the loads of all lanes are issued together)
        // and their hop result is zeroed once after the last direction.
        const int sg_ = s[g] < Ls ? s[g] : 0;
        R p[24];
        // lane-dependent offsets (site, slice) go to the vector operand, the
        // wave-uniform group offset to the scalar one
        const unsigned vb = yg + (unsigned)sg_ * NGR * gb;
#pragma unroll
        for (int q = 0; q < NGR; ++q) {
            R v[8];
            bload_group<S>(R_.in, vb, (unsigned)q * gb, v);
#pragma unroll
            for (int k = 0; k < 2 * PK; ++k) p[2 * PK * q + k] = v[k];
        }
        if (pre_mode_of<PM>(P) == 2) {   // mode 1 (diagonal) enters through kr and a final scale
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] *= pd[g][0];
#pragma unroll
            for (int k = 12; k < 24; ++k) p[k] *= pd[g][1];
        }
        if (pre_mode_of<PM>(P) == 2) {
            // K pattern: upper chirality (components 0-5) couples s-1, lower
            // (6-11) s+1 (cyclic); groups that straddle the boundary are read
            // from both slices
            const unsigned sm = (unsigned)(sg_ == 0 ? Ls - 1 : sg_ - 1) * NGR * gb;
            const unsigned sp = (unsigned)(sg_ == Ls - 1 ? 0 : sg_ + 1) * NGR * gb;
#pragma unroll
            for (int q = 0; q < NGR; ++q) {
                if (PK * q < 6) {
                    R v[8];
                    bload_group<S>(R_.in, yg + sm, (unsigned)q * gb, v);
#pragma unroll
                    for (int k = 0; k < PK; ++k)
                        if (PK * q + k < 6) {
                            p[2 * (PK * q + k)] += pe[g][0] * v[2 * k];
                            p[2 * (PK * q + k) + 1] += pe[g][0] * v[2 * k + 1];
                        }
                }
                if (PK * q + PK > 6) {
                    R v[8];
                    bload_group<S>(R_.in, yg + sp, (unsigned)q * gb, v);
#pragma unroll
                    for (int k = 0; k < PK; ++k)
                        if (PK * q + k >= 6) {
                            p[2 * (PK * q + k)] += pe[g][1] * v[2 * k];
                            p[2 * (PK * q + k) + 1] += pe[g][1] * v[2 * k + 1];
                        }
                }
            }
        }
        hop_dir<R>(D, U, p, h[g], kr[g]);
    }
}

// Pipelined form of hop_direction (DWF_HOP_PREFETCH): hop_fetch issues the
// neighbour loads of direction D for the wave's slice groups into raw
// 16-byte words; hop_apply decodes them and does the rest of hop_direction
// (the K pre-mix, the link from LDS, the spin-projected colour products).
template <class S>
__device__ __forceinline__ void decode_group(u32x4 w, typename Traits<S>::R (&v)[8]) {
    if constexpr (sizeof(S) == 8) {
        v[0] = __hiloint2double(w.y, w.x);
        v[1] = __hiloint2double(w.w, w.z);
    } else if constexpr (sizeof(S) == 4) {
        v[0] = __uint_as_float(w.x);
        v[1] = __uint_as_float(w.y);
        v[2] = __uint_as_float(w.z);
        v[3] = __uint_as_float(w.w);
    } else {
        const unsigned u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = bf16_to_f32(u[k] & 0xffffu);
            v[2 * k + 1] = bf16_to_f32(u[k] >> 16);
        }
    }
}

// neighbour site index y given (hop_fetch_at) or read from the staged table
template <class S, int G>
__device__ __forceinline__ void hop_fetch_at(const HopParams& P, const HopRes& R_, unsigned gb, unsigned y,
                                             const int (&s)[G], u32x4 (&raw)[G][12 / fpack<S>()], unsigned& yg) {
    constexpr unsigned CB = cbytes<S>();
    constexpr int PK = fpack<S>();
    constexpr int NGR = 12 / PK;
    static_assert(PK * CB == 16, "16-byte field groups expected");
    yg = y * (unsigned)PK * CB;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int sg_ = s[g] < P.Ls ? s[g] : 0;   // slices past Ls read slice 0 (zeroed later)
        const unsigned vb = yg + (unsigned)sg_ * NGR * gb;
#pragma unroll
        for (int q = 0; q < NGR; ++q) raw[g][q] = __builtin_amdgcn_raw_buffer_load_b128(R_.in, vb, (unsigned)q * gb, 0);
    }
}

template <class S, int G>
__device__ __forceinline__ void hop_fetch(const HopParams& P, const HopRes& R_, unsigned gb, int D, const int (&s)[G],
                                          const unsigned* lnbr, int j, u32x4 (&raw)[G][12 / fpack<S>()],
                                          unsigned& yg) {
    hop_fetch_at<S, G>(P, R_, gb, lnbr[D * 16 + j], s, raw, yg);
}

template <class S, int G, int PM>
__device__ __forceinline__ void hop_apply(const HopParams& P, const HopRes& R_, unsigned gb, int D, const int (&s)[G],
                                          const typename Traits<S>::R (&pd)[G][2],
                                          const typename Traits<S>::R (&pe)[G][2],
                                          const typename Traits<S>::R (&kr)[G],
                                          typename Traits<S>::R (&h)[G][24], const u32x4* lnk,
                                          const u32x4 (&raw)[G][12 / fpack<S>()], unsigned yg, int j) {
    using R = typename Traits<S>::R;
    constexpr unsigned CB = cbytes<S>();
    constexpr unsigned NG = link_ng(CB);
    constexpr int PK = fpack<S>();
    constexpr int NGR = 12 / PK;
    const int Ls = P.Ls;
    R U[18];
#pragma unroll
    for (unsigned g = 0; g < NG; ++g) decode_link_group<S>(lnk[(D * NG + g) * 16 + j], (int)g, U);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int sg_ = s[g] < Ls ? s[g] : 0;
        R p[24];
#pragma unroll
        for (int q = 0; q < NGR; ++q) {
            R v[8];
            decode_group<S>(raw[g][q], v);
#pragma unroll
            for (int k = 0; k < 2 * PK; ++k) p[2 * PK * q + k] = v[k];
        }
        if (pre_mode_of<PM>(P) == 2) {
#pragma unroll
            for (int k = 0; k < 12; ++k) p[k] *= pd[g][0];
#pragma unroll
            for (int k = 12; k < 24; ++k) p[k] *= pd[g][1];
            const unsigned sm = (unsigned)(sg_ == 0 ? Ls - 1 : sg_ - 1) * NGR * gb;
            const unsigned sp = (unsigned)(sg_ == Ls - 1 ? 0 : sg_ + 1) * NGR * gb;
#pragma unroll
            for (int q = 0; q < NGR; ++q) {
                if (PK * q < 6) {
                    R v[8];
                    bload_group<S>(R_.in, yg + sm, (unsigned)q * gb, v);
#pragma unroll
                    for (int k = 0; k < PK; ++k)
                        if (PK * q + k < 6) {
                            p[2 * (PK * q + k)] += pe[g][0] * v[2 * k];
                            p[2 * (PK * q + k) + 1] += pe[g][0] * v[2 * k + 1];
                        }
                }
                if (PK * q + PK > 6) {
                    R v[8];
                    bload_group<S>(R_.in, yg + sp, (unsigned)q * gb, v);
#pragma unroll
                    for (int k = 0; k < PK; ++k)
                        if (PK * q + k >= 6) {
                            p[2 * (PK * q + k)] += pe[g][1] * v[2 * k];
                            p[2 * (PK * q + k) + 1] += pe[g][1] * v[2 * k + 1];
                        }
                }
            }
        }
        hop_dir<R>(D, U, p, h[g], kr[g]);
    }
}

// Number of 4-slice groups each wave computes in the hop phase, and waves
// per block, for KK = ceil(Ls/4) groups.
__host__ __device__ constexpr int hop_kpw(int KK, bool f64) {
    return f64 ? (KK % DWF_HOP_KPW64 == 0 ? DWF_HOP_KPW64 : 1) : (KK % DWF_HOP_KPW == 0 ? DWF_HOP_KPW : 1);
}
__host__ __device__ constexpr int hop_waves(int KK, bool f64) { return KK / hop_kpw(KK, f64); }

// Block = KK waves = 16 sites x all s (KK = ceil(Ls/4)).
//  phase 1: wave w computes the hop for s = 4w + sc at site j of the block
//           (lane = 16 sc + j) and stores it to LDS as hs[w][real r][lane];
//           that is exactly the MFMA B operand for k-step w.
//  phase 2: wave w takes 12/KK of the 12 spin-colour components; for each it
//           runs the dense s-mixes as KK MFMAs per real part with B read back
//           from LDS, plus the local term as more MFMAs, and stores (FP32 and
//           BF16 through LDS, as whole 16-byte groups).
// Keeping one 4-slice group per wave (instead of all Ls slices) keeps the
// data a wave touches, and its registers, four times smaller; that lets an
// XCD's 4 MB L2 hold the neighbour reuse window.
// TAG only renames the symbol: TAG = 1 is the instance launched by the
// stand-alone hop benchmark, so profilers report it apart from the solver's.
//
// hop_tile computes one such block's work: sites 16*tile .. 16*tile+15 of
// right-hand side `rhs`; part_out (or nullptr) receives the block's partial
// norm.  Both kernels below call it.
template <class S> constexpr int lnk_entries() { return 8 * link_ng(cbytes<S>()) * 16; }

// Epilogue kinds compiled with their flags as constants: the fused stages of
// the CG iteration (the generic kernel, EK = -1, tests every flag at run
// time).  EK_PLAIN: out only.  EK_CHAIN: the D^ stage, out2 = POST2 . (POST .
// H + loc_scale loc) with |first result|^2 reduced.  EK_UPD: the last stage,
// upd -= alpha (POST . H + LOCMIX . loc) with |upd|^2 reduced.
constexpr int EK_PLAIN = 1, EK_CHAIN = 2, EK_UPD = 3;
inline int epilogue_kind(const HopParams& P) {
    if (P.out && !P.loc && !P.out2 && !P.upd && !P.partial && P.reduce == 0) return EK_PLAIN;
    if (!P.out && P.loc && !P.locmix && P.out2 && P.chain2 && !P.upd && P.partial && P.reduce == 1) return EK_CHAIN;
    if (!P.out && P.loc && P.locmix && !P.out2 && P.upd && P.partial && P.reduce == 3) return EK_UPD;
    return -1;
}

// Shared memory of one block (dynamic, bytes from the host):
//   [0, r0)       phase 1: the tile's links and neighbour indices;
//                 then hs, the hop result (MFMA B operand), hs[kk][r][lane]
//                 at kk * HSK + r * 64 + lane (HSK padded so that the four
//                 slice groups of a wave fall on different banks);
//                 FP32/BF16 then reuse the rows 2 cp, 2 cp + 1 of every kk
//                 (read only by the wave that owns component cp) for the
//                 output of component cp: slice 4 kk + i, site jj at
//                 complex (i * 16 + jj) of that 128-value run
//   [r0, r0+32)   per-wave partial norms
//   [r0+32, ...)  local-term tile, 16-byte groups [s][group][site]
//                 (FP32/BF16 launches with a local term only)
template <class S, int KK> struct HopSmem {
    using R = typename Traits<S>::R;
    static constexpr bool TIO = DWF_HOP_TILE_IO && sizeof(S) < 8;
    static constexpr bool LOC = TIO && (sizeof(S) == 2 ? DWF_HOP_LOC_LDS16 : DWF_HOP_LOC_LDS32);
    static constexpr int PK = fpack<S>();
    static constexpr int NGR = 12 / PK;
    static constexpr int HSK = 24 * 64 + (sizeof(R) == 4 ? 16 : 8);
    static constexpr unsigned hs_b = KK * HSK * sizeof(R);
    static constexpr unsigned lnk_b = lnk_entries<S>() * 16 + 128 * 4;
    // SEP: hs after the staged tables instead of over them (no block
    // barrier between the last link read and the first hs write)
    static constexpr bool SEP = sizeof(S) == 4 && DWF_HOP_HS_SEP32 && KK == 4;
    static constexpr unsigned hs_off = SEP ? ((lnk_b + 15u) & ~15u) : 0u;
    static constexpr unsigned mx = SEP ? hs_off + hs_b : (hs_b > lnk_b ? hs_b : lnk_b);
    static constexpr unsigned r0 = (mx + 15u) & ~15u;
    static constexpr unsigned red_off = r0;
    // FP32: the dense s-mixes (POST, LOCMIX, POST2, LOCMIX2; [2][16][16]
    // each) staged with the links, read back in the second phase
    static constexpr bool CST = sizeof(S) == 4 && DWF_HOP_COEF_LDS32 && DWF_HOP_STAGE_BATCH && DWF_HOP_LDS_LINKS;
    static constexpr unsigned cst_off = r0 + 32;
    static constexpr unsigned cst_b = CST ? 4u * MAT_ELEMS * 4u : 0u;
    static constexpr unsigned loc_off = cst_off + cst_b;
    static constexpr unsigned loc_b = LOC ? KK * 4 * NGR * 16 * 16 : 0u;
    static constexpr unsigned bytes(bool has_loc) { return loc_off + (has_loc ? loc_b : 0u); }
};

// A block may hold several such tiles of one item, one per right-hand side
// (the shared-link work-list kernel): group `sub` of NW waves computes
// right-hand side `rhs` in its own shared-memory region smem + sub * region,
// while the tile's links and neighbour indices are staged once, by every
// thread of the block, into the first region.  An inactive group (a
// right-hand side past the item's count or already converged) runs the same
// code, barriers included, on zero-size buffer descriptors: its loads read
// zeros and its stores are dropped.  The reduction runs when P.partial is set
// (the same for every group of a block); part_out = nullptr skips the write.
template <class S, int KK, int PM = -1, int EK = -1>
__device__ __forceinline__ void hop_tile(const HopParams& P, long tile, int rhs, double* part_out,
                                         unsigned char* smem, int sub = 0, unsigned region = 0,
                                         bool active = true) {
    using R = typename Traits<S>::R;
    using V = typename Vec4<R>::T;
    using L = HopSmem<S, KK>;
    // which outputs, local terms and reductions the launch has: compile-time
    // constants for the epilogue kinds below, else read from P
    constexpr bool EKC = EK >= 0;
    const bool f_out = EKC ? EK == EK_PLAIN : P.out != nullptr;
    const bool f_loc = EKC ? (EK == EK_CHAIN || EK == EK_UPD) : P.loc != nullptr;
    const bool f_dense = EKC ? EK == EK_UPD : (P.loc != nullptr && P.locmix != nullptr);
    const bool f_out2 = EKC ? EK == EK_CHAIN : P.out2 != nullptr;
    const bool f_chain = EKC ? EK == EK_CHAIN : (P.out2 != nullptr && P.chain2 != 0);
    const bool f_upd = EKC ? EK == EK_UPD : P.upd != nullptr;
    const int f_reduce = EKC ? (EK == EK_CHAIN ? 1 : (EK == EK_UPD ? 3 : 0)) : P.reduce;
    const bool f_partial = EKC ? EK != EK_PLAIN : P.partial != nullptr;
    constexpr int NW = hop_waves(KK, sizeof(S) == 8);
    constexpr int NTHR = 64 * NW;
    unsigned char* own = smem + (size_t)sub * region;
    R* hs = reinterpret_cast<R*>(own + L::hs_off);   // hs[kk][r][lane] at kk * HSK + r * 64 + lane
    constexpr int HSK = L::HSK;
    u32x4* lnk = reinterpret_cast<u32x4*>(smem);
    unsigned* lnbr = reinterpret_cast<unsigned*>(smem + lnk_entries<S>() * 16);
    double* red = reinterpret_cast<double*>(own + L::red_off);
    u32x4* locT = reinterpret_cast<u32x4*>(own + L::loc_off);
    const int lane = threadIdx.x & 63;
    const int tid = (int)threadIdx.x - sub * NTHR;   // thread index within the group
#if DWF_HOP_W_UNIFORM
    const int w = __builtin_amdgcn_readfirstlane(((int)threadIdx.x >> 6) - sub * NW);   // wave-uniform
#else
    const int w = ((int)threadIdx.x >> 6) - sub * NW;
#endif
    const int j = lane & 15, sc = lane >> 4;
    const long Vh = P.Vh;
    const int Ls = P.Ls;
    const long site = tile * 16 + j;
    const bool valid = site < Vh;
    const long sx = valid ? site : Vh - 1;
    constexpr unsigned CB = cbytes<S>();
    constexpr unsigned PK = fpack<S>();
    const unsigned gb = (unsigned)P.Vhp * PK * CB;             // bytes of one group row (PK components of a slice)
    const unsigned fieldb = (unsigned)Ls * (12u / PK) * gb;    // bytes of one right-hand side
    const unsigned fieldb_a = active ? fieldb : 0u;             // zero-size descriptors when inactive
    const size_t rhsb = (size_t)rhs * fieldb;                  // bytes of the preceding RHS
    const unsigned sxb = (unsigned)sx * PK * CB;               // this site's offset in a group row
    HopRes R_;
    R_.in = make_rsrc(static_cast<const char*>(P.in) + rhsb, fieldb_a);
    R_.loc = make_rsrc(P.loc ? static_cast<const char*>(P.loc) + rhsb : nullptr, P.loc ? fieldb_a : 0u);
    R_.out = make_rsrc(P.out ? static_cast<const char*>(P.out) + rhsb : nullptr, P.out ? fieldb_a : 0u);
    R_.out2 = make_rsrc(P.out2 ? static_cast<const char*>(P.out2) + rhsb : nullptr, P.out2 ? fieldb_a : 0u);
    // fused CG update target: compute type in its own layout
    constexpr unsigned PKU = fpack<typename std::conditional<sizeof(R) == 8, double, float>::type>();
    const unsigned fieldu = (unsigned)Ls * 12u * (unsigned)P.Vhp * 2u * (unsigned)sizeof(R);
    R_.upd = make_rsrc(P.upd ? static_cast<char*>(P.upd) + (size_t)rhs * fieldu : nullptr,
                       (P.upd && active) ? fieldu : 0u);
    R_.links = make_rsrc(P.links, 8u * link_ng(CB) * (unsigned)P.Vhp * link_lp(CB) * CB);
    R_.nbr = make_rsrc(P.nbr, 8u * (unsigned)P.Vhp * 4u);

    // Slice groups of this wave, and the pipelined loop's first two
    // directions (EARLY: their neighbour spinors are requested before the
    // block barrier, with the neighbour indices read per lane).
    constexpr int G = hop_kpw(KK, sizeof(S) == 8);
    constexpr int PF = PM < 0 ? 0 : (sizeof(S) == 8 ? DWF_HOP_PREFETCH64 : DWF_HOP_PREFETCH);
    constexpr bool EARLY = DWF_HOP_EARLY && PF == 2 && DWF_HOP_LDS_LINKS &&
                           (sizeof(S) == 8 ? DWF_HOP_STAGE_BATCH64 : DWF_HOP_STAGE_BATCH);
    constexpr int NGR_ = 12 / fpack<S>();
    int sg[G];
#pragma unroll
    for (int g = 0; g < G; ++g) sg[g] = 4 * (w * G + g) + sc;
    u32x4 ra[G][NGR_], rb[G][NGR_];
    unsigned ya = 0, yb = 0;
    // pre-mix coefficients of the wave's slices (read before the tile's
    // loads, so that waiting for them does not wait for the spinors)
    R pd[G][2], pe[G][2], kr[G];
    {
        const R* pre = static_cast<const R*>(P.pre);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int sc_ = min(sg[g], LS_MAX - 1);
            pd[g][0] = pre ? pre[0 * 16 + sc_] : R(1);
            pd[g][1] = pre ? pre[1 * 16 + sc_] : R(1);
            pe[g][0] = pre ? pre[2 * 16 + sc_] : R(0);
            pe[g][1] = pre ? pre[3 * 16 + sc_] : R(0);
            // diagonal pre-mix (mode 1; the host guarantees d_up != 0 on valid
            // slices): lower/upper ratio inside the projection, d_up at the end
            kr[g] = (pre_mode_of<PM>(P) == 1 && pd[g][0] != R(0)) ? pd[g][1] / pd[g][0] : R(1);
        }
    }

    constexpr bool SBATCH = sizeof(S) == 8 ? DWF_HOP_STAGE_BATCH64 : DWF_HOP_STAGE_BATCH;
    if constexpr (DWF_HOP_LDS_LINKS && SBATCH) {
        // the tile's links (16-byte groups) and neighbour indices, once per
        // block; every lane-dependent offset is in the vector operand.  All
        // loads are issued before the first LDS write (a loop with a runtime
        // trip count would wait for each load in turn).  Threads past the
        // table's end read and rewrite its last entry.
        const unsigned Vhp = (unsigned)P.Vhp;
        constexpr int NE = lnk_entries<S>();
        constexpr int IT = (NE + NTHR - 1) / NTHR;    // blockDim.x >= NTHR
        constexpr int IB = (128 + NTHR - 1) / NTHR;
        unsigned y0 = 0, y1 = 0;
        if constexpr (EARLY) {
            y0 = __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, (unsigned)sx * 4u, 0u, DWF_HOP_NT_LINK);
            y1 = __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, (unsigned)sx * 4u, Vhp * 4u, DWF_HOP_NT_LINK);
        }
        u32x4 lv[IT];
        unsigned nv[IB];
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int e = min((int)threadIdx.x + i * (int)blockDim.x, NE - 1);
            const int dg = e >> 4, jj = e & 15;
            const long se = tile * 16 + jj;
            const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
            lv[i] = __builtin_amdgcn_raw_buffer_load_b128(R_.links, sxe * 16u + (unsigned)dg * Vhp * 16u, 0u,
                                                          DWF_HOP_NT_LINK);
        }
#pragma unroll
        for (int i = 0; i < IB; ++i) {
            const int e = min((int)threadIdx.x + i * (int)blockDim.x, 127);
            const int d = e >> 4, jj = e & 15;
            const long se = tile * 16 + jj;
            const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
            nv[i] = __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, sxe * 4u + (unsigned)d * Vhp * 4u, 0u,
                                                         DWF_HOP_NT_LINK);
        }
        // dense s-mixes (FP32): 4 x 128 groups of 16 bytes; a missing matrix
        // reads POST instead (never used)
        constexpr int IC = L::CST ? (4 * MAT_ELEMS / 4 + NTHR - 1) / NTHR : 1;
        u32x4 cv[IC];
        if constexpr (L::CST) {
            const u32x4* m0 = static_cast<const u32x4*>(P.post);
            const u32x4* m1 = P.locmix ? static_cast<const u32x4*>(P.locmix) : m0;
            const u32x4* m2 = P.post2 ? static_cast<const u32x4*>(P.post2) : m0;
            const u32x4* m3 = P.locmix2 ? static_cast<const u32x4*>(P.locmix2) : m0;
#pragma unroll
            for (int i = 0; i < IC; ++i) {
                const int e = min((int)threadIdx.x + i * (int)blockDim.x, 4 * MAT_ELEMS / 4 - 1);
                const int m = e >> 7;   // MAT_ELEMS / 4 = 128 groups per matrix
                const u32x4* src = m == 0 ? m0 : (m == 1 ? m1 : (m == 2 ? m2 : m3));
                cv[i] = src[e & 127];
            }
        }
        if constexpr (EARLY) {
            hop_fetch_at<S, G>(P, R_, gb, y0, sg, ra, ya);
            hop_fetch_at<S, G>(P, R_, gb, y1, sg, rb, yb);
        }
        // unconditional stores (a guarded store lets the compiler sink its
        // load behind the guard and wait for it there)
#pragma unroll
        for (int i = 0; i < IT; ++i) lnk[min((int)threadIdx.x + i * (int)blockDim.x, NE - 1)] = lv[i];
#pragma unroll
        for (int i = 0; i < IB; ++i) lnbr[min((int)threadIdx.x + i * (int)blockDim.x, 127)] = nv[i];
        if constexpr (L::CST) {
            u32x4* cdst = reinterpret_cast<u32x4*>(smem + L::cst_off);
#pragma unroll
            for (int i = 0; i < IC; ++i) cdst[min((int)threadIdx.x + i * (int)blockDim.x, 4 * MAT_ELEMS / 4 - 1)] = cv[i];
        }
    }
    if constexpr (DWF_HOP_LDS_LINKS && !SBATCH) {
        // the same tables, one entry per thread and step
        const unsigned Vhp = (unsigned)P.Vhp;
        for (int e = threadIdx.x; e < lnk_entries<S>(); e += blockDim.x) {
            const int dg = e >> 4, jj = e & 15;
            const long se = tile * 16 + jj;
            const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
            lnk[e] = __builtin_amdgcn_raw_buffer_load_b128(R_.links, sxe * 16u + (unsigned)dg * Vhp * 16u, 0u,
                                                           DWF_HOP_NT_LINK);
        }
        for (int e = threadIdx.x; e < 128; e += blockDim.x) {
            const int d = e >> 4, jj = e & 15;
            const long se = tile * 16 + jj;
            const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
            lnbr[e] = __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, sxe * 4u + (unsigned)d * Vhp * 4u, 0u,
                                                           DWF_HOP_NT_LINK);
        }
    }
    if constexpr (L::LOC) {
        // local-term tile: group (s, q) of site jj at locT[(s * NGR + q) * 16 + jj];
        // slices s >= Ls are zero (they meet zero columns of the local mixes)
        if (f_loc) {
            constexpr int NL = KK * 4 * L::NGR * 16;
            constexpr int IL = (NL + NTHR - 1) / NTHR;
            u32x4 lt[IL];
#pragma unroll
            for (int i = 0; i < IL; ++i) {
                const int e = min(tid + i * NTHR, NL - 1);
                const int jj = e & 15, g = e >> 4;
                const long se = tile * 16 + jj;
                const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
                const int gc = g < Ls * L::NGR ? g : 0;
                lt[i] = __builtin_amdgcn_raw_buffer_load_b128(R_.loc, sxe * 16u + (unsigned)gc * gb, 0u, DWF_HOP_NT_LOAD);
            }
#pragma unroll
            for (int i = 0; i < IL; ++i) {
                const int e = min(tid + i * NTHR, NL - 1);
                const u32x4 z = {0u, 0u, 0u, 0u};
                locT[e] = (e >> 4) < Ls * L::NGR ? lt[i] : z;
            }
        }
    }
    if constexpr (DWF_HOP_LDS_LINKS || L::LOC) __syncthreads();

    // FP32 local term of the chained and update stages (per-component global
    // reads, not tiled in LDS): requested right after the direction loop, so
    // that the reads are in flight across the block barriers instead of
    // after them.  Compiled only for those epilogue kinds (a no-local-term
    // launch would still issue the reads).
    constexpr int CPW_ = 12 / hop_waves(KK, sizeof(S) == 8);
    constexpr bool LOCE = DWF_HOP_LOC_EARLY32 && sizeof(S) == 4 && !L::LOC && (EK == EK_CHAIN || EK == EK_UPD);
    R lre[LOCE ? CPW_ : 1][LOCE ? KK : 1], lie[LOCE ? CPW_ : 1][LOCE ? KK : 1];
    // the update stage's old values (its 16-byte groups of this thread),
    // requested with the local term
    constexpr bool UPDE = LOCE && DWF_HOP_UPD_EARLY32 && EK == EK_UPD;
    constexpr int IUE = UPDE ? (4 * KK * 6 * 16 + NTHR - 1) / NTHR : 1;
    u32x4 uve[IUE];
    R h[G][24];
    {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int k = 0; k < 24; ++k) h[g][k] = 0;
        // Loop over the 8 hop directions.  Its unrolling (DWF_HOP_UNROLL)
        // trades registers for loads in flight: with 1, nothing of direction
        // d+1 (its links in particular) is hoisted above direction d.
        unsigned ynb[8];
#pragma unroll
        for (int d = 0; d < 8; ++d)
            ynb[d] = (DWF_HOP_NBR_PRELOAD && !DWF_HOP_LDS_LINKS)
                         ? __builtin_amdgcn_raw_buffer_load_b32(R_.nbr, (unsigned)sx * 4u, (unsigned)d * (unsigned)P.Vhp * 4u, 0)
                         : 0u;
        if constexpr (PF == 2 && DWF_HOP_LDS_LINKS) {
            // fully unrolled, double-buffered: direction d is a compile-time
            // constant in each step (its spin structure folds), and the loads
            // of d+1 are issued before the arithmetic of d
            if constexpr (!EARLY) {
                hop_fetch<S, G>(P, R_, gb, 0, sg, lnbr, j, ra, ya);
                hop_fetch<S, G>(P, R_, gb, 1, sg, lnbr, j, rb, yb);
            }
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 0, sg, pd, pe, kr, h, lnk, ra, ya, j);
            hop_fetch<S, G>(P, R_, gb, 2, sg, lnbr, j, ra, ya);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 1, sg, pd, pe, kr, h, lnk, rb, yb, j);
            hop_fetch<S, G>(P, R_, gb, 3, sg, lnbr, j, rb, yb);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 2, sg, pd, pe, kr, h, lnk, ra, ya, j);
            hop_fetch<S, G>(P, R_, gb, 4, sg, lnbr, j, ra, ya);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 3, sg, pd, pe, kr, h, lnk, rb, yb, j);
            hop_fetch<S, G>(P, R_, gb, 5, sg, lnbr, j, rb, yb);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 4, sg, pd, pe, kr, h, lnk, ra, ya, j);
            hop_fetch<S, G>(P, R_, gb, 6, sg, lnbr, j, ra, ya);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 5, sg, pd, pe, kr, h, lnk, rb, yb, j);
            hop_fetch<S, G>(P, R_, gb, 7, sg, lnbr, j, rb, yb);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 6, sg, pd, pe, kr, h, lnk, ra, ya, j);
            __builtin_amdgcn_sched_barrier(0);
            hop_apply<S, G, PM>(P, R_, gb, 7, sg, pd, pe, kr, h, lnk, rb, yb, j);
        } else if constexpr (PF == 1 && DWF_HOP_LDS_LINKS) {
            // ping-pong over two raw buffers: the loads of the next direction
            // are in flight while the current one is computed
            hop_fetch<S, G>(P, R_, gb, 0, sg, lnbr, j, ra, ya);
#pragma unroll 1
            for (int d = 0; d < 8; d += 2) {
                hop_fetch<S, G>(P, R_, gb, d + 1, sg, lnbr, j, rb, yb);
                __builtin_amdgcn_sched_barrier(0);
                hop_apply<S, G, PM>(P, R_, gb, d, sg, pd, pe, kr, h, lnk, ra, ya, j);
                if (d + 2 < 8) hop_fetch<S, G>(P, R_, gb, d + 2, sg, lnbr, j, ra, ya);
                __builtin_amdgcn_sched_barrier(0);
                hop_apply<S, G, PM>(P, R_, gb, d + 1, sg, pd, pe, kr, h, lnk, rb, yb, j);
            }
        } else {
#pragma unroll DWF_HOP_UNROLL
            for (int d = 0; d < 8; ++d) {
                hop_direction<S, G, PM>(P, R_, gb, (unsigned)sx, d, ynb[d], sg, pd, pe, kr, h, lnk, lnbr, j);
                // unrolled: keep each direction's loads after the previous one's
                // arithmetic (hoisting them all raises the register count past
                // the occupancy target)
                if constexpr (DWF_HOP_UNROLL > 1) {
                    asm volatile("" ::: "memory");
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (pre_mode_of<PM>(P) == 1) {
#pragma unroll
                for (int k = 0; k < 24; ++k) h[g][k] *= pd[g][0];
            }
            const bool inval = sg[g] >= Ls;
#pragma unroll
            for (int k = 0; k < 24; ++k) h[g][k] = inval ? R(0) : h[g][k];
        }
    }
    if constexpr (LOCE) {
        // slices past Ls read slice 0 and are zeroed (branch-free: measured,
        // a branch among these reads made the register allocator spill
        // across the direction loop)
#pragma unroll
        for (int q = 0; q < CPW_; ++q)
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int cp = w * CPW_ + q, s_ = sc + 4 * kk;
                const unsigned off = sxb + (unsigned)(s_ < Ls ? s_ : 0) * (12u / PK) * gb +
                                     (unsigned)(cp / PK) * gb + (unsigned)(cp % PK) * CB;
                const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(R_.loc, off, 0u, 0);
                lre[q][kk] = s_ < Ls ? __uint_as_float(v.x) : R(0);
                lie[q][kk] = s_ < Ls ? __uint_as_float(v.y) : R(0);
            }
        if constexpr (UPDE) {
            const unsigned gbu = (unsigned)P.Vhp * 16u;
            const int nU = Ls * 6 * 16;
#pragma unroll
            for (int i = 0; i < IUE; ++i) {
                const int e = min(tid + i * NTHR, nU - 1);
                const int jj = e & 15, g = e >> 4;
                const long se = tile * 16 + jj;
                const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
                uve[i] = __builtin_amdgcn_raw_buffer_load_b128(R_.upd, sxe * 16u + (unsigned)g * gbu, 0u, DWF_HOP_NT_LOAD);
            }
        }
    }
    if constexpr (!L::SEP) __syncthreads();   // hs shares storage with the staged links

#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < 24; ++k) hs[(w * G + g) * HSK + k * 64 + lane] = h[g][k];
    __syncthreads();

    // A operands: A[m][k] = MAT[chi][row m = j][col 4*kk + sc].  A dense
    // local mix (LOCMIX, LOCMIX2) enters as more MFMAs with B = the local
    // field in the hs layout; loc_scale times the identity is a plain add
    // when the local tile is in LDS, else one more MFMA set.
    const R* post = static_cast<const R*>(P.post);
    const R* lmix = static_cast<const R*>(P.locmix);
    const R* post2 = static_cast<const R*>(P.post2);
    const R* lmix2 = static_cast<const R*>(P.locmix2);
    const bool has_loc = f_loc;
    const bool dense_loc = f_dense;
    const bool has_out2 = f_out2;
    const bool chain = f_chain;
    const R lscale = R(P.loc_scale);
    constexpr int CPW = 12 / hop_waves(KK, sizeof(S) == 8);
    // per-component accesses: one instruction covers whole lines only in FP64
    // (one complex per 16-byte group); in FP32/BF16 a group holds several
    // components, read or written by different instructions, and a
    // non-temporal line can leave L2 before the second one (measured: the
    // FP32 solve 2 % slower with it)
    constexpr int WAUX = sizeof(S) == 8 ? DWF_HOP_NT_LOAD : 0;
    constexpr int SAUX = sizeof(S) == 8 ? DWF_HOP_NT_STORE : 0;

    // FP32/BF16: the primary output (out, else out2) goes through LDS; a
    // second output, if any, is stored directly
    const bool upd = f_upd;
    const R ua = upd ? R(P.upd_alpha[(long)rhs * P.upd_stride]) : R(0);
    const bool tile_out = L::TIO && (f_out || has_out2 || upd);
    // byte offset of component cp of slice s of this lane's site; the whole
    // offset goes to the vector operand (cp depends on the wave index, which
    // the compiler does not treat as uniform: a scalar operand would be
    // split into a loop over lanes)
    auto coff = [&](int s, int cp) -> unsigned {
        return sxb + (unsigned)s * (12u / PK) * gb + (unsigned)(cp / PK) * gb + (unsigned)(cp % PK) * CB;
    };
    double nrm = 0.0;
    // A operands of one chirality, loaded once per wave before the component
    // loop (per-lane loads are vector-memory instructions, and the compiler
    // cannot see that the per-component loads repeat).  When the components
    // of a wave all have the same chirality (6 divisible by CPW) one set is
    // loaded; otherwise a wave whose components straddle the two chiralities
    // loads a second set and each component selects its own.
    constexpr bool CHI_W = DWF_HOP_COEF_HOIST && (6 % CPW) == 0;
    constexpr bool CHI_2 = DWF_HOP_COEF_HOIST >= 2 && !CHI_W;
    const R* cst = reinterpret_cast<const R*>(smem + L::cst_off);   // block-wide (region 0)
    auto load_a = [&](int chi, R (&ap)[KK], R (&al)[KK], R (&ap2)[KK], R (&al2)[KK]) {
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const int idx = (chi * 16 + j) * 16 + 4 * kk + sc;
            if constexpr (L::CST) {
                ap[kk] = cst[idx];
                al[kk] = dense_loc ? cst[MAT_ELEMS + idx] : ((has_loc && !L::LOC && j == 4 * kk + sc) ? lscale : R(0));
                ap2[kk] = has_out2 ? cst[2 * MAT_ELEMS + idx] : R(0);
                al2[kk] = (has_out2 && has_loc && !chain) ? cst[3 * MAT_ELEMS + idx] : R(0);
            } else {
                ap[kk] = post[idx];
                al[kk] = dense_loc ? lmix[idx] : ((has_loc && !L::LOC && j == 4 * kk + sc) ? lscale : R(0));
                ap2[kk] = has_out2 ? post2[idx] : R(0);
                al2[kk] = (has_out2 && has_loc && !chain) ? lmix2[idx] : R(0);
            }
        }
    };
    R apw[KK], alw[KK], ap2w[KK], al2w[KK];
    R apv[KK], alv[KK], ap2v[KK], al2v[KK];
    const int chi_a = w * CPW >= 6 ? 1 : 0;             // first component of the wave
    const int chi_b = w * CPW + CPW - 1 >= 6 ? 1 : 0;   // last component of the wave
    if constexpr (CHI_W || CHI_2) load_a(chi_a, apw, alw, ap2w, al2w);
    if constexpr (CHI_2) {
        if (chi_b != chi_a) {   // wave-uniform
            load_a(chi_b, apv, alv, ap2v, al2v);
        } else {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                apv[kk] = apw[kk];
                alv[kk] = alw[kk];
                ap2v[kk] = ap2w[kk];
                al2v[kk] = al2w[kk];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
        const int cp = w * CPW + q;
        const int chi = cp >= 6 ? 1 : 0;
        R ap[KK], al[KK], ap2[KK], al2[KK];
        if constexpr (CHI_W) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                ap[kk] = apw[kk];
                al[kk] = alw[kk];
                ap2[kk] = ap2w[kk];
                al2[kk] = al2w[kk];
            }
        } else if constexpr (CHI_2) {
            const bool second = chi != chi_a;
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                ap[kk] = second ? apv[kk] : apw[kk];
                al[kk] = second ? alv[kk] : alw[kk];
                ap2[kk] = second ? ap2v[kk] : ap2w[kk];
                al2[kk] = second ? al2v[kk] : al2w[kk];
            }
        } else {
            load_a(chi, ap, al, ap2, al2);
        }
        // local values in the B layout: slice 4 kk + sc of site j
        R lr[KK], li[KK];
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) { lr[kk] = 0; li[kk] = 0; }
        const bool loc_mfma = dense_loc || (has_loc && !L::LOC);
        if (loc_mfma || (has_out2 && has_loc && !chain)) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int s = sc + 4 * kk;
                if constexpr (L::LOC) {
                    const int e = (s * L::NGR + cp / L::PK) * 16 + j;
                    if constexpr (sizeof(S) == 4) {
                        const u32x2 v = reinterpret_cast<const u32x2*>(locT)[e * 2 + cp % 2];
                        lr[kk] = __uint_as_float(v.x);
                        li[kk] = __uint_as_float(v.y);
                    } else {
                        const unsigned v = reinterpret_cast<const unsigned*>(locT)[e * 4 + cp % 4];
                        lr[kk] = bf16_to_f32(v & 0xffffu);
                        li[kk] = bf16_to_f32(v >> 16);
                    }
                } else if constexpr (LOCE) {
                    lr[kk] = lre[q][kk];
                    li[kk] = lie[q][kk];
                } else {
                    if (s < Ls) bload<S, WAUX>(R_.loc, coff(s, cp), 0u, lr[kk], li[kk]);
                }
            }
        }
        V cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            cr = mfma4(ap[kk], hs[kk * HSK + (2 * cp) * 64 + lane], cr);
            ci = mfma4(ap[kk], hs[kk * HSK + (2 * cp + 1) * 64 + lane], ci);
        }
        if (loc_mfma) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                cr = mfma4(al[kk], lr[kk], cr);
                ci = mfma4(al[kk], li[kk], ci);
            }
        }
        if constexpr (L::LOC) {
            if (has_loc && !dense_loc) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {   // row layout: slice out_row(sc, i) of site j
                    const int e = (out_row<R>(sc, i) * L::NGR + cp / L::PK) * 16 + j;
                    R xr, xi;
                    if constexpr (sizeof(S) == 4) {
                        const u32x2 v = reinterpret_cast<const u32x2*>(locT)[e * 2 + cp % 2];
                        xr = __uint_as_float(v.x);
                        xi = __uint_as_float(v.y);
                    } else {
                        const unsigned v = reinterpret_cast<const unsigned*>(locT)[e * 4 + cp % 4];
                        xr = bf16_to_f32(v & 0xffffu);
                        xi = bf16_to_f32(v >> 16);
                    }
                    cr[i] += lscale * xr;
                    ci[i] += lscale * xi;
                }
            }
        }
        V dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
        if (chain) {
            // the first result back to the B layout through the rows 2 cp,
            // 2 cp + 1 of hs, which only this wave reads (no block barrier),
            // then out2 = POST2 . result
            wave_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int s = out_row<R>(sc, i);
                if (s < 4 * KK) {
                    hs[(s >> 2) * HSK + (2 * cp) * 64 + 16 * (s & 3) + j] = cr[i];
                    hs[(s >> 2) * HSK + (2 * cp + 1) * 64 + 16 * (s & 3) + j] = ci[i];
                }
            }
            wave_sync();
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                dr = mfma4(ap2[kk], hs[kk * HSK + (2 * cp) * 64 + lane], dr);
                di = mfma4(ap2[kk], hs[kk * HSK + (2 * cp + 1) * 64 + lane], di);
            }
        } else if (has_out2) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                dr = mfma4(ap2[kk], hs[kk * HSK + (2 * cp) * 64 + lane], dr);
                di = mfma4(ap2[kk], hs[kk * HSK + (2 * cp + 1) * 64 + lane], di);
            }
            if (has_loc) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    dr = mfma4(al2[kk], lr[kk], dr);
                    di = mfma4(al2[kk], li[kk], di);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = out_row<R>(sc, i);
            if (valid && s < Ls) {
                if (f_reduce == 1) nrm += double(cr[i]) * double(cr[i]) + double(ci[i]) * double(ci[i]);
                if (f_reduce == 2) nrm += double(dr[i]) * double(dr[i]) + double(di[i]) * double(di[i]);
                if (!tile_out) {
                    if (upd) {   // FP64: upd has the layout of out
                        R ur, ui;
                        bload<S, WAUX>(R_.upd, coff(s, cp), 0u, ur, ui);
                        ur -= ua * cr[i];
                        ui -= ua * ci[i];
                        bstore<S, SAUX>(R_.upd, coff(s, cp), 0u, ur, ui);
                        if (f_reduce == 3) nrm += double(ur) * double(ur) + double(ui) * double(ui);
                    }
                    if (f_out) bstore<S, SAUX>(R_.out, coff(s, cp), 0u, cr[i], ci[i]);
                    if (has_out2) bstore<S, SAUX>(R_.out2, coff(s, cp), 0u, dr[i], di[i]);
                } else if (f_out && has_out2) {
                    bstore<S, SAUX>(R_.out2, coff(s, cp), 0u, dr[i], di[i]);
                }
            }
        }
        if constexpr (L::TIO) {
            if (tile_out) {
                // this wave alone read rows 2 cp, 2 cp + 1 of hs: overwrite them
                // with the component's output (slice 4 kk + i at i * 16 + jj)
                wave_sync();
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int s = out_row<R>(sc, i);
                    if (s >= Ls) continue;   // rows past Ls: zero columns, and past the hs runs when KK < 4
                    const R orr = (f_out || upd) ? cr[i] : dr[i];
                    const R oi = (f_out || upd) ? ci[i] : di[i];
                    R* run = hs + (s >> 2) * HSK + (2 * cp) * 64;
                    if (sizeof(S) == 4 || upd) {   // FP32 values (the update needs them unrounded)
                        reinterpret_cast<float2*>(run)[(s & 3) * 16 + j] = make_float2(orr, oi);
                    } else {
                        reinterpret_cast<unsigned*>(run)[(s & 3) * 16 + j] = pack_bf16(orr, oi);
                    }
                }
            }
        }
    }

    if constexpr (L::TIO) {
        if (upd) {
            // upd -= alpha * result over upd's own groups (FP32 pairs)
            static_assert(PKU == 2, "fused update expects FP32 fields in component pairs");
            __syncthreads();
            const unsigned gbu = (unsigned)P.Vhp * 16u;
            // every LDS and global read of the thread first, then the
            // updates (a loop with a runtime trip count would wait for each
            // iteration's reads in turn); threads past the end read the last
            // entry again and store nothing
            const int nU = Ls * 6 * 16;
            constexpr int IU = (4 * KK * 6 * 16 + NTHR - 1) / NTHR;
            float2 av[IU], bv[IU];
            u32x4 uv[IU];
#pragma unroll
            for (int i = 0; i < IU; ++i) {
                const int e = min(tid + i * NTHR, nU - 1);
                const int jj = e & 15, g = e >> 4;
                const int sl = g / 6, q2 = g - sl * 6;
                const long se = tile * 16 + jj;
                const float* run0 = hs + (sl >> 2) * HSK + 2 * ((sl & 3) * 16 + jj);
                av[i] = *reinterpret_cast<const float2*>(run0 + (2 * (2 * q2)) * 64);
                bv[i] = *reinterpret_cast<const float2*>(run0 + (2 * (2 * q2 + 1)) * 64);
                const unsigned sxe = (unsigned)(se < Vh ? se : Vh - 1);
                if constexpr (UPDE)
                    uv[i] = uve[i];
                else
                    uv[i] = __builtin_amdgcn_raw_buffer_load_b128(R_.upd, sxe * 16u + (unsigned)g * gbu, 0u,
                                                                  DWF_HOP_NT_LOAD);
            }
#pragma unroll
            for (int i = 0; i < IU; ++i) {
                const int e = tid + i * NTHR;
                const int jj = e & 15, g = e >> 4;
                const long se = tile * 16 + jj;
                if (e < nU && se < Vh) {
                    const unsigned off = (unsigned)se * 16u + (unsigned)g * gbu;
                    const u32x4 u = uv[i];
                    const float2 a = av[i], b = bv[i];
                    float v0 = __uint_as_float(u.x) - ua * a.x, v1 = __uint_as_float(u.y) - ua * a.y;
                    float v2 = __uint_as_float(u.z) - ua * b.x, v3 = __uint_as_float(u.w) - ua * b.y;
                    u32x4 o;
                    o.x = __float_as_uint(v0); o.y = __float_as_uint(v1); o.z = __float_as_uint(v2); o.w = __float_as_uint(v3);
                    __builtin_amdgcn_raw_buffer_store_b128(o, R_.upd, off, 0u, DWF_HOP_NT_STORE);
                    if (f_reduce == 3)
                        nrm += double(v0) * double(v0) + double(v1) * double(v1) + double(v2) * double(v2) +
                               double(v3) * double(v3);
                }
            }
        } else if (tile_out) {
            // whole 16-byte groups of 16 consecutive sites
            __syncthreads();
            const __amdgpu_buffer_rsrc_t dst = f_out ? R_.out : R_.out2;
            // all LDS reads first, then the stores (as in the update above)
            const int nO = Ls * L::NGR * 16;
            constexpr int IO = (4 * KK * L::NGR * 16 + NTHR - 1) / NTHR;
            u32x4 vv[IO];
#pragma unroll
            for (int i = 0; i < IO; ++i) {
                const int e = min(tid + i * NTHR, nO - 1);
                const int jj = e & 15, g = e >> 4;
                const int sl = g / L::NGR, q = g - sl * L::NGR;
                const R* run0 = hs + (sl >> 2) * HSK + (sl & 3) * 16 * (int)(CB / 4) + jj * (int)(CB / 4);
                if constexpr (sizeof(S) == 4) {
                    const u32x2 a = *reinterpret_cast<const u32x2*>(run0 + (2 * (2 * q)) * 64);
                    const u32x2 b = *reinterpret_cast<const u32x2*>(run0 + (2 * (2 * q + 1)) * 64);
                    vv[i].x = a.x; vv[i].y = a.y; vv[i].z = b.x; vv[i].w = b.y;
                } else {
                    const unsigned* r = reinterpret_cast<const unsigned*>(run0);
                    vv[i].x = r[(2 * (4 * q)) * 64];
                    vv[i].y = r[(2 * (4 * q + 1)) * 64];
                    vv[i].z = r[(2 * (4 * q + 2)) * 64];
                    vv[i].w = r[(2 * (4 * q + 3)) * 64];
                }
            }
#pragma unroll
            for (int i = 0; i < IO; ++i) {
                const int e = tid + i * NTHR;
                const int jj = e & 15, g = e >> 4;
                const long se = tile * 16 + jj;
                if (e < nO && se < Vh)
                    __builtin_amdgcn_raw_buffer_store_b128(vv[i], dst, (unsigned)se * 16u + (unsigned)g * gb, 0u,
                                                           DWF_HOP_NT_STORE);
            }
        }
    }

    if (f_partial) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        if (lane == 0) red[w] = nrm;
        __syncthreads();
        if (tid == 0 && part_out) {
            double t = 0.0;
            for (int ww = 0; ww < NW; ++ww) t += red[ww];
            *part_out = t;
        }
    }
}

// Waves per SIMD the single-lattice hop is compiled for.  The general
// pre-mix (mode 2, c != 0) holds the extra K row in registers: at the
// occupancy of modes 0/1 it spills in FP64 and BF16, so it runs one wave
// lower there.
template <class S, int PM>
constexpr int hop_waves_per_eu() {
    if (sizeof(S) == 8) return PM == 2 ? DWF_HOP_WAVES_PER_EU64_BATCH : DWF_HOP_WAVES_PER_EU64;
    if (sizeof(S) == 2) return PM == 2 ? DWF_HOP_WAVES_PER_EU16 - 1 : DWF_HOP_WAVES_PER_EU16;
    return DWF_HOP_WAVES_PER_EU;
}

template <class S, int KK, int TAG = 0, int PM = 1, int EK = -1>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(hop_waves_per_eu<S, PM>())))
void hop_mfma_kernel(HopParams P) {
    extern __shared__ u32x4 hop_smem[];
    hop_tile<S, KK, PM, EK>(P, xcd_block(blockIdx.x, gridDim.x), blockIdx.y,
                    P.partial ? P.partial + (long)blockIdx.y * gridDim.x + blockIdx.x : nullptr,
                    reinterpret_cast<unsigned char*>(hop_smem));
}

// Work-list form for batches: one launch covers several operators (lattices
// of any size with the same ceil(Ls/4)) and all their right-hand sides.
// meta[0..n] is the prefix sum of the blocks of each item, meta[n+1+i] its
// number of right-hand sides.  Item i takes ceil(nrhs/nrb) x tiles blocks;
// a block computes one tile for nrb consecutive right-hand sides, so the
// tile's links and neighbour indices are fetched from HBM once and re-read
// from cache for the others.  order 0 sweeps tiles fastest (neighbour reuse
// across tiles of one RHS), order 1 sweeps RHS chunks fastest (link reuse
// across chunks).  A right-hand side whose done flag is set is skipped
// (its partial is written as 0).
// PM as in hop_batch1_kernel below (the same arithmetic path, so that every
// schedule gives the same bits).
template <class S, int KK, int PM>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? DWF_HOP_WAVES_PER_EU64_BATCH : DWF_HOP_BATCHN_WPE)))
void hop_batch_kernel(const HopParams* __restrict__ items, const int* __restrict__ meta, int nitems, int nrb,
                      int order) {
    extern __shared__ u32x4 hop_smem[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int i = 0;
    while (i + 1 < nitems && b >= meta[i + 1]) ++i;
    const HopParams& P = items[i];   // read in place (wave-uniform address: scalar loads)
    const int nrhs = meta[nitems + 1 + i];
    const long tiles = (P.Vh + 15) / 16;
    const int chunks = (nrhs + nrb - 1) / nrb;
    const long local = b - meta[i];
    const long tile = order == 0 ? local % tiles : local / chunks;
    const int chunk = order == 0 ? (int)(local / tiles) : (int)(local % chunks);
    for (int q = 0; q < nrb; ++q) {
        const int r = chunk * nrb + q;
        if (r >= nrhs) break;
        double* part = P.partial ? P.partial + (long)r * P.pstride + tile : nullptr;
        if (P.done && P.done[(long)r * P.done_stride] != 0.0) {
            if (part && threadIdx.x == 0) *part = 0.0;
            continue;
        }
        hop_tile<S, KK, PM>(P, tile, r, part, reinterpret_cast<unsigned char*>(hop_smem));
        __syncthreads();   // shared memory is reused by the next right-hand side
    }
}

// The same work list with one right-hand side per block (nrb = 1): no loop
// around the tile, so nothing is live across right-hand sides.
#ifndef DWF_HOP_BATCH1_WPE
#define DWF_HOP_BATCH1_WPE 5
#endif
// PM >= 0: every item of the launch has that pre-mix mode (compiled in, with
// the single-lattice kernel's pipelined direction loop and occupancy);
// PM = -1: mixed modes, read per item.
template <class S, int PM>
constexpr int hop_batch1_waves_per_eu() {
    if (PM >= 0) return hop_waves_per_eu<S, PM>();
    return sizeof(S) == 8 ? DWF_HOP_WAVES_PER_EU64_BATCH : DWF_HOP_BATCH1_WPE;
}

template <class S, int KK, int PM, int EK = -1>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(hop_batch1_waves_per_eu<S, PM>())))
void hop_batch1_kernel(const HopParams* __restrict__ items, const int* __restrict__ meta, int nitems, int order) {
    extern __shared__ u32x4 hop_smem[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int i = 0;
    while (i + 1 < nitems && b >= meta[i + 1]) ++i;
    const HopParams& P = items[i];   // read in place (wave-uniform address: scalar loads)
    const int nrhs = meta[nitems + 1 + i];
    const int tiles = (int)((P.Vh + 15) / 16);
    int tile = b - meta[i], r = 0;
    if (order == 0) {
        // tiles fastest: a uniform subtraction loop (nrhs steps at most)
        // keeps tile and r in scalar registers, where a division would be
        // expanded on the vector unit
        while (tile >= tiles) { tile -= tiles; ++r; }
    } else {
        r = tile % nrhs;
        tile /= nrhs;
    }
    double* part = P.partial ? P.partial + (long)r * P.pstride + tile : nullptr;
    if (P.done && P.done[(long)r * P.done_stride] != 0.0) {
        if (part && threadIdx.x == 0) *part = 0.0;
        return;
    }
    hop_tile<S, KK, PM, EK>(P, tile, r, part, reinterpret_cast<unsigned char*>(hop_smem));
}

// The work list with NR right-hand sides per block sharing the tile's
// staged links and neighbour indices: group r of the block's NR groups of
// hop_waves(KK) waves computes right-hand side chunk * NR + r of the tile in
// its own shared-memory region (`region` bytes each).  Block -> (tile,
// chunk) as in hop_batch1_kernel with chunks of NR right-hand sides.
template <class S, int KK, int PM, int NR>
__global__ __launch_bounds__(1024)
__attribute__((amdgpu_waves_per_eu(hop_batch1_waves_per_eu<S, PM>())))
void hop_multi_kernel(const HopParams* __restrict__ items, const int* __restrict__ meta, int nitems, int order,
                      unsigned region) {
    extern __shared__ u32x4 hop_smem[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int i = 0;
    while (i + 1 < nitems && b >= meta[i + 1]) ++i;
    const HopParams& P = items[i];
    const int nrhs = meta[nitems + 1 + i];
    const int tiles = (int)((P.Vh + 15) / 16);
    const int chunks = (nrhs + NR - 1) / NR;
    int tile = b - meta[i], chunk = 0;
    if (order == 0) {
        while (tile >= tiles) { tile -= tiles; ++chunk; }
    } else {
        chunk = tile % chunks;
        tile /= chunks;
    }
    const int sub = (int)threadIdx.x / (64 * hop_waves(KK, sizeof(S) == 8));   // wave-uniform
    const int r = chunk * NR + sub;
    const bool in_range = r < nrhs;
    const int rr = in_range ? r : nrhs - 1;   // scalar reads of an out-of-range group stay in bounds
    const bool active = in_range && !(P.done && P.done[(long)rr * P.done_stride] != 0.0);
    // a converged right-hand side writes a zero partial (its loads read zeros)
    double* part = (P.partial && in_range) ? P.partial + (long)rr * P.pstride + tile : nullptr;
    hop_tile<S, KK, PM>(P, tile, rr, part, reinterpret_cast<unsigned char*>(hop_smem), sub, region, active);
}

// ---------------------------------------------------------------------
// Local dense s-mix on one half field: out = A . in (per chirality),
// same lane layout and MFMA use as the hop epilogue.  Optional reduction.
// ---------------------------------------------------------------------
template <class S, int KK>
__global__ __launch_bounds__(256) void mix_mfma_kernel(MixParams P) {
    using R = typename Traits<S>::R;
    using V = typename Vec4<R>::T;
    const int lane = threadIdx.x & 63;
    const int j = lane & 15, sc = lane >> 4;
    const long Vh = P.Vh;
    const int Ls = P.Ls;
    const long site = ((long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 16 + j;
    const bool valid = site < Vh;
    const long sx = valid ? site : Vh - 1;
    const long Vhp = P.Vhp;
    const long roff = (long)blockIdx.y * Ls * 12 * Vhp;
    const R* A = static_cast<const R*>(P.mat);
    R a[2][KK];
#pragma unroll
    for (int chi = 0; chi < 2; ++chi)
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) a[chi][kk] = A[(chi * 16 + j) * 16 + 4 * kk + sc];
    double nrm = 0.0;
#pragma unroll
    for (int cp = 0; cp < 12; ++cp) {
        const int chi = cp / 6;
        V cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            const int s = sc + 4 * kk;
            R xr = 0, xi = 0;
            if (s < Ls) cload<S>(P.in, roff + fidx((long)s * 12 + cp, sx, Vhp, fpack<S>()), xr, xi);
            cr = mfma4(a[chi][kk], xr, cr);
            ci = mfma4(a[chi][kk], xi, ci);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = out_row<R>(sc, i);
            if (valid && s < Ls) {
                cstore<S>(P.out, roff + fidx((long)s * 12 + cp, site, Vhp, fpack<S>()), cr[i], ci[i]);
                nrm += double(cr[i]) * double(cr[i]) + double(ci[i]) * double(ci[i]);
            }
        }
    }
    if (P.partial) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
        __shared__ double red[4];
        if (lane == 0) red[threadIdx.x >> 6] = nrm;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
            P.partial[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------
template <class S>
static unsigned hop_smem_bytes(int KK, bool loc) {
    switch (KK) {
        case 1: return HopSmem<S, 1>::bytes(loc);
        case 2: return HopSmem<S, 2>::bytes(loc);
        case 3: return HopSmem<S, 3>::bytes(loc);
        default: return HopSmem<S, 4>::bytes(loc);
    }
}

int hop_grid_blocks(long Vh) { return (int)((Vh + 15) / 16); }
int mix_grid_blocks(long Vh) { return (int)((Vh + 63) / 64); }

// Minimum shared memory per hop block ($DWF_HOP_MIN_LDS bytes, default 0):
// a larger request caps the blocks resident per CU (160 KB of LDS each),
// i.e. the sites an XCD has in flight, without changing the code.
static unsigned hop_min_lds() {
    static const unsigned v = [] {
        const char* e = std::getenv("DWF_HOP_MIN_LDS");
        const long x = e ? std::atol(e) : 0;
        return (unsigned)std::min<long>(std::max<long>(x, 0), 160 * 1024);
    }();
    return v;
}

template <class S, int TAG, int PM, int EK>
static void launch_hop_ek(const HopParams& P, int nrhs, hipStream_t st) {
    const int KK = (P.Ls + 3) / 4;
    dim3 grid(hop_grid_blocks(P.Vh), nrhs), block(64 * hop_waves(KK, sizeof(S) == 8));
    const unsigned smem_b = std::max(hop_smem_bytes<S>(KK, P.loc != nullptr), hop_min_lds());
    switch (KK) {
        // Ls <= 4: the generic kernel (the specialised chained stage spills there)
        case 1: hipLaunchKernelGGL((hop_mfma_kernel<S, 1, TAG, PM, -1>), grid, block, smem_b, st, P); break;
        case 2: hipLaunchKernelGGL((hop_mfma_kernel<S, 2, TAG, PM, EK>), grid, block, smem_b, st, P); break;
        case 3: hipLaunchKernelGGL((hop_mfma_kernel<S, 3, TAG, PM, EK>), grid, block, smem_b, st, P); break;
        case 4: hipLaunchKernelGGL((hop_mfma_kernel<S, 4, TAG, PM, EK>), grid, block, smem_b, st, P); break;
        default: throw Error{DWF_EDIMS, "Ls > 16 not supported by the fused hop"};
    }
    DWF_HIP(hipGetLastError());
}

// Epilogue kinds compiled per pre-mix mode: the plain hop for every mode of
// the solver's launches (FP64: mode 0 only), the chained and update stages
// for mode 0 (they never pre-mix); the stand-alone benchmark instance only as
// the plain mode-1 hop it times.
template <class S, int TAG, int PM>
static void launch_hop_pm(const HopParams& P, int nrhs, hipStream_t st) {
    const int ek = DWF_HOP_EK ? epilogue_kind(P) : -1;
    if constexpr ((TAG == 1 && PM != 1) || (sizeof(S) == 8 && PM != 0)) {
        // (FP64 pre-mixing hops: the specialised plain form spills one value)
        launch_hop_ek<S, TAG, PM, -1>(P, nrhs, st);
    } else if constexpr (TAG == 1 || PM != 0) {
        if (ek == EK_PLAIN) launch_hop_ek<S, TAG, PM, EK_PLAIN>(P, nrhs, st);
        else launch_hop_ek<S, TAG, PM, -1>(P, nrhs, st);
    } else {
        switch (ek) {
            case EK_PLAIN: launch_hop_ek<S, TAG, PM, EK_PLAIN>(P, nrhs, st); break;
            case EK_CHAIN: launch_hop_ek<S, TAG, PM, EK_CHAIN>(P, nrhs, st); break;
            case EK_UPD: launch_hop_ek<S, TAG, PM, EK_UPD>(P, nrhs, st); break;
            default: launch_hop_ek<S, TAG, PM, -1>(P, nrhs, st); break;
        }
    }
}

template <class S, int TAG>
static void launch_hop_t(const HopParams& P, int nrhs, hipStream_t st) {
    switch (P.pre_mode) {
        case 0: launch_hop_pm<S, TAG, 0>(P, nrhs, st); break;
        case 1: launch_hop_pm<S, TAG, 1>(P, nrhs, st); break;
        case 2: launch_hop_pm<S, TAG, 2>(P, nrhs, st); break;
        default: throw Error{DWF_EINVAL, "bad pre-mix mode"};
    }
}

template <class S, int PM, int EK>
static void launch_hop_batch1_ek(int KK, dim3 grid, dim3 block, unsigned smem_b, const HopParams* items,
                                 const int* meta, int nitems, int order, hipStream_t st) {
    switch (KK) {
        // Ls <= 4: the generic kernel, as for single lattices
        case 1: hipLaunchKernelGGL((hop_batch1_kernel<S, 1, PM, -1>), grid, block, smem_b, st, items, meta, nitems, order); break;
        case 2: hipLaunchKernelGGL((hop_batch1_kernel<S, 2, PM, EK>), grid, block, smem_b, st, items, meta, nitems, order); break;
        case 3: hipLaunchKernelGGL((hop_batch1_kernel<S, 3, PM, EK>), grid, block, smem_b, st, items, meta, nitems, order); break;
        case 4: hipLaunchKernelGGL((hop_batch1_kernel<S, 4, PM, EK>), grid, block, smem_b, st, items, meta, nitems, order); break;
        default: throw Error{DWF_EDIMS, "Ls > 16 not supported by the fused hop"};
    }
}

// ek: the items' common epilogue kind (-1: mixed or none), compiled in on
// the same terms as for single-lattice launches
template <class S, int PM>
static void launch_hop_batch1_pm(int KK, dim3 grid, dim3 block, unsigned smem_b, const HopParams* items,
                                 const int* meta, int nitems, int order, int ek, hipStream_t st) {
    if (!DWF_HOP_EK) ek = -1;
    if constexpr (PM < 0 || (sizeof(S) == 8 && PM != 0)) {
        launch_hop_batch1_ek<S, PM, -1>(KK, grid, block, smem_b, items, meta, nitems, order, st);
    } else if constexpr (PM != 0) {
        if (ek == EK_PLAIN) launch_hop_batch1_ek<S, PM, EK_PLAIN>(KK, grid, block, smem_b, items, meta, nitems, order, st);
        else launch_hop_batch1_ek<S, PM, -1>(KK, grid, block, smem_b, items, meta, nitems, order, st);
    } else {
        switch (ek) {
            case EK_PLAIN: launch_hop_batch1_ek<S, PM, EK_PLAIN>(KK, grid, block, smem_b, items, meta, nitems, order, st); break;
            case EK_CHAIN: launch_hop_batch1_ek<S, PM, EK_CHAIN>(KK, grid, block, smem_b, items, meta, nitems, order, st); break;
            case EK_UPD: launch_hop_batch1_ek<S, PM, EK_UPD>(KK, grid, block, smem_b, items, meta, nitems, order, st); break;
            default: launch_hop_batch1_ek<S, PM, -1>(KK, grid, block, smem_b, items, meta, nitems, order, st); break;
        }
    }
}

template <class S, int PM>
static void launch_hop_batchn_pm(int KK, dim3 grid, dim3 block, unsigned smem_b, const HopParams* items,
                                 const int* meta, int nitems, int nrb, int order, hipStream_t st) {
    switch (KK) {
        case 1: hipLaunchKernelGGL((hop_batch_kernel<S, 1, PM>), grid, block, smem_b, st, items, meta, nitems, nrb, order); break;
        case 2: hipLaunchKernelGGL((hop_batch_kernel<S, 2, PM>), grid, block, smem_b, st, items, meta, nitems, nrb, order); break;
        case 3: hipLaunchKernelGGL((hop_batch_kernel<S, 3, PM>), grid, block, smem_b, st, items, meta, nitems, nrb, order); break;
        case 4: hipLaunchKernelGGL((hop_batch_kernel<S, 4, PM>), grid, block, smem_b, st, items, meta, nitems, nrb, order); break;
        default: throw Error{DWF_EDIMS, "Ls > 16 not supported by the fused hop"};
    }
}

template <class S, int PM, int NR>
static void launch_hop_multi_pm(int KK, dim3 grid, unsigned region, const HopParams* items, const int* meta,
                                int nitems, int order, hipStream_t st) {
    const dim3 block(64 * hop_waves(KK, sizeof(S) == 8) * NR);
    const unsigned smem_b = region * NR;
    switch (KK) {
        case 1: hipLaunchKernelGGL((hop_multi_kernel<S, 1, PM, NR>), grid, block, smem_b, st, items, meta, nitems, order, region); break;
        case 2: hipLaunchKernelGGL((hop_multi_kernel<S, 2, PM, NR>), grid, block, smem_b, st, items, meta, nitems, order, region); break;
        case 3: hipLaunchKernelGGL((hop_multi_kernel<S, 3, PM, NR>), grid, block, smem_b, st, items, meta, nitems, order, region); break;
        case 4: hipLaunchKernelGGL((hop_multi_kernel<S, 4, PM, NR>), grid, block, smem_b, st, items, meta, nitems, order, region); break;
        default: throw Error{DWF_EDIMS, "Ls > 16 not supported by the fused hop"};
    }
}

// shared-link kernel for FP32 with 2 or 4 right-hand sides per block when
// the block (<= 1024 threads) and its shared memory fit; false otherwise
template <class S>
static bool launch_hop_multi(int KK, int blocks, int nrb, int order, bool loc, int pm, const HopParams* items,
                             const int* meta, int nitems, hipStream_t st) {
    if constexpr (!std::is_same<S, float>::value) {
        return false;
    } else {
        if (nrb != 2 && nrb != 4) return false;
        if (64 * hop_waves(KK, false) * nrb > 1024) return false;
        static const int max_lds = [] {
            int dev = 0, v = 65536;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
                v = 65536;
            return v;
        }();
        const unsigned region = (hop_smem_bytes<S>(KK, loc) + 15u) & ~15u;
        if ((long)region * nrb > (long)max_lds) return false;
        const dim3 grid(blocks);
#define DWF_MULTI(PMV)                                                                                   \
    (nrb == 2 ? launch_hop_multi_pm<S, PMV, 2>(KK, grid, region, items, meta, nitems, order, st)        \
              : launch_hop_multi_pm<S, PMV, 4>(KK, grid, region, items, meta, nitems, order, st))
        switch (pm) {
            case 0: DWF_MULTI(0); break;
            case 1: DWF_MULTI(1); break;
            case 2: DWF_MULTI(2); break;
            default: DWF_MULTI(-1); break;
        }
#undef DWF_MULTI
        DWF_HIP(hipGetLastError());
        return true;
    }
}

template <class S>
static void launch_hop_batch_t(int KK, const HopParams* items, const int* meta, int nitems, int blocks, int nrb,
                               int order, bool loc, int pm, int ek, hipStream_t st) {
    if (launch_hop_multi<S>(KK, blocks, nrb, order, loc, pm, items, meta, nitems, st)) return;
    dim3 grid(blocks), block(64 * hop_waves(KK, sizeof(S) == 8));
    const unsigned smem_b = hop_smem_bytes<S>(KK, loc);
    if (nrb == 1) {
        switch (pm) {
            case 0: launch_hop_batch1_pm<S, 0>(KK, grid, block, smem_b, items, meta, nitems, order, ek, st); break;
            case 1: launch_hop_batch1_pm<S, 1>(KK, grid, block, smem_b, items, meta, nitems, order, ek, st); break;
            case 2: launch_hop_batch1_pm<S, 2>(KK, grid, block, smem_b, items, meta, nitems, order, ek, st); break;
            default: launch_hop_batch1_pm<S, -1>(KK, grid, block, smem_b, items, meta, nitems, order, ek, st); break;
        }
        DWF_HIP(hipGetLastError());
        return;
    }
    switch (pm) {
        case 0: launch_hop_batchn_pm<S, 0>(KK, grid, block, smem_b, items, meta, nitems, nrb, order, st); break;
        case 1: launch_hop_batchn_pm<S, 1>(KK, grid, block, smem_b, items, meta, nitems, nrb, order, st); break;
        case 2: launch_hop_batchn_pm<S, 2>(KK, grid, block, smem_b, items, meta, nitems, nrb, order, st); break;
        default: launch_hop_batchn_pm<S, -1>(KK, grid, block, smem_b, items, meta, nitems, nrb, order, st); break;
    }
    DWF_HIP(hipGetLastError());
}

int hop_epilogue_kind(const HopParams& P) { return epilogue_kind(P); }

void launch_hop_batch(int kind, int KK, const HopParams* items, const int* meta, int nitems, int blocks, int nrb,
                      int order, bool has_loc, int pm, int ek, hipStream_t st) {
    if (blocks <= 0) return;
    switch (kind) {
        case ST_F64: launch_hop_batch_t<double>(KK, items, meta, nitems, blocks, nrb, order, has_loc, pm, ek, st); break;
        case ST_F32: launch_hop_batch_t<float>(KK, items, meta, nitems, blocks, nrb, order, has_loc, pm, ek, st); break;
        case ST_BF16: launch_hop_batch_t<bf16s>(KK, items, meta, nitems, blocks, nrb, order, has_loc, pm, ek, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}

void launch_hop(int kind, const HopParams& P, int nrhs, hipStream_t st, int bench_tag) {
    switch (kind) {
        case ST_F64:
            if (bench_tag) launch_hop_t<double, 1>(P, nrhs, st); else launch_hop_t<double, 0>(P, nrhs, st);
            break;
        case ST_F32:
            if (bench_tag) launch_hop_t<float, 1>(P, nrhs, st); else launch_hop_t<float, 0>(P, nrhs, st);
            break;
        case ST_BF16:
            if (bench_tag) launch_hop_t<bf16s, 1>(P, nrhs, st); else launch_hop_t<bf16s, 0>(P, nrhs, st);
            break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}

// Plain streaming copy (16-byte vectors), used to calibrate memory counters
// and as the measured streaming ceiling: every lane moves four 16-byte
// vectors whose loads are all issued before the first store, one block per
// 4 x 256 vectors (no grid-stride loop), the form that kept the most bytes
// in flight in a sweep of vectors per lane and block counts.
constexpr int COPY_VPL = 4;
__global__ __launch_bounds__(256) void copy_kernel(float4* __restrict__ dst, const float4* __restrict__ src, long n) {
    const long base = (long)blockIdx.x * (256 * COPY_VPL) + threadIdx.x;
    float4 v[COPY_VPL];
#pragma unroll
    for (int k = 0; k < COPY_VPL; ++k) {
        const long i = base + (long)k * 256;
        if (i < n) v[k] = src[i];
    }
#pragma unroll
    for (int k = 0; k < COPY_VPL; ++k) {
        const long i = base + (long)k * 256;
        if (i < n) dst[i] = v[k];
    }
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const long n = (long)(bytes / 16);
    const long blocks = (n + 256 * COPY_VPL - 1) / (256 * COPY_VPL);
    DWF_REQUIRE(blocks < (1L << 31), DWF_EINVAL, "copy too large");
    if (blocks == 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (float4*)dst, (const float4*)src, n);
    DWF_HIP(hipGetLastError());
}

template <class S>
static void launch_mix_t(const MixParams& P, int nrhs, hipStream_t st) {
    dim3 grid(mix_grid_blocks(P.Vh), nrhs), block(256);
    const int KK = (P.Ls + 3) / 4;
    switch (KK) {
        case 1: hipLaunchKernelGGL((mix_mfma_kernel<S, 1>), grid, block, 0, st, P); break;
        case 2: hipLaunchKernelGGL((mix_mfma_kernel<S, 2>), grid, block, 0, st, P); break;
        case 3: hipLaunchKernelGGL((mix_mfma_kernel<S, 3>), grid, block, 0, st, P); break;
        case 4: hipLaunchKernelGGL((mix_mfma_kernel<S, 4>), grid, block, 0, st, P); break;
        default: throw Error{DWF_EDIMS, "Ls > 16 not supported"};
    }
    DWF_HIP(hipGetLastError());
}

void launch_mix(int kind, const MixParams& P, int nrhs, hipStream_t st) {
    switch (kind) {
        case ST_F64: launch_mix_t<double>(P, nrhs, st); break;
        case ST_F32: launch_mix_t<float>(P, nrhs, st); break;
        case ST_BF16: launch_mix_t<bf16s>(P, nrhs, st); break;
        default: throw Error{DWF_EINVAL, "bad storage kind"};
    }
}

}  // namespace dwf
