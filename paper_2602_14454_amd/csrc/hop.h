// Launch interface of the fused hop and local-mix kernels (hop.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

// All matrices are compute-type (double for F64 storage, float otherwise),
// padded to [2 chirality][16][16]; `pre` is [d chi0 | d chi1 | e chi0 | e chi1] x 16.
// Stage 2 of D^dag D^ forms v = g5 Minv^T q from q itself (1) or as
// POST2 . h + LOCMIX2 . p (0).
#ifndef DWF_CHAIN2
#define DWF_CHAIN2 1
#endif
struct HopParams {
    const void* in;        // input half field, parity 1-p
    const void* loc;       // local half field, parity p (nullptr: none)
    void* out;             // output half field (nullptr: not stored)
    void* out2;            // second output (nullptr: none)
    const void* links;     // hop links of output parity p
    const int* nbr;        // neighbour table of output parity p
    const void* pre;       // sparse pre-mix coefficients (nullptr: identity)
    const void* post;      // dense POST (required)
    const void* locmix;    // dense LOCMIX (nullptr: loc_scale * identity)
    const void* post2;     // dense POST2 (required with out2)
    const void* locmix2;   // dense LOCMIX2 (required with out2 and loc)
    double* partial;       // per-block FP64 partial norms (nullptr: none)
    long Vh;               // sites of the output parity
    long Vhp;              // padded row stride of fields, links and neighbour table
    int Ls;
    int pre_mode;          // 0 identity, 1 diagonal d, 2 d + e (K sparsity)
    int reduce;            // 1: |out|^2, 2: |out2|^2, 3: |upd|^2 after the update
    int chain2;            // 1: out2 = POST2 . (the first result, local term included); LOCMIX2 unused
    double loc_scale;
    // fused CG update (nullptr: none; needs out == out2 == nullptr):
    // upd -= (*upd_alpha) * (first result), the result itself is not stored.
    // upd holds the compute type (FP64 for FP64 launches, FP32 otherwise) in
    // that type's own field layout.
    void* upd;
    const double* upd_alpha;   // alpha of right-hand side r at upd_alpha[r * upd_stride]
    long upd_stride;
    // work-list (batch) launches only
    const double* done;    // per-RHS done flags, done[r * done_stride] != 0: skip (nullptr: none)
    long done_stride;
    long pstride;          // partial of (rhs r, tile t) at partial[r * pstride + t]
};

struct MixParams {
    const void* in;
    void* out;
    const void* mat;       // dense [2][16][16] compute type
    double* partial;
    long Vh;
    long Vhp;
    int Ls;
};

int hop_grid_blocks(long Vh);
// blocks of a mix launch per right-hand side (partials it writes, with partial set)
int mix_grid_blocks(long Vh);
void launch_hop(int kind, const HopParams& P, int nrhs, hipStream_t st, int bench_tag = 0);
// One work-list launch over `nitems` HopParams (device array `items`, same
// ceil(Ls/4) = KK for all) with block prefix sums and RHS counts in `meta`
// (device, 2 * nitems + 1 ints); `blocks` = meta[nitems].  has_loc: the
// items carry a local term (all or none of them).  pm: the pre-mix mode
// every item has (0, 1, 2), or -1 when they differ.  ek: the epilogue kind
// every item has (hop_epilogue_kind), or -1 when they differ.
void launch_hop_batch(int kind, int KK, const HopParams* items, const int* meta, int nitems, int blocks, int nrb,
                      int order, bool has_loc, int pm, int ek, hipStream_t st);
// The epilogue kind of a launch that the hop kernels are compiled for (the
// fused stages of the CG iteration), or -1 (flags tested at run time).
int hop_epilogue_kind(const HopParams& P);
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
void launch_mix(int kind, const MixParams& P, int nrhs, hipStream_t st);

}  // namespace dwf
