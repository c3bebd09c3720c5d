// Slot-aware vector kernels for batched solves (slot_blas.hip).
//
// A batch is a list of slots; a slot is one right-hand side of one operator
// (lattices may differ in size and Ls).  Every batch vector is one buffer
// holding the slots' even half fields back to back: slot v occupies complex
// elements [off, off + n).  Each slot owns a block of CG scalars at
// scal[v * CG_NSLOTS] and a run of partial sums at partial[v * pstride].
// One launch covers all slots (block -> slot through block0); a slot whose
// CG_DONE flag is set is left untouched.
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

// extra per-slot CG scalars (after the ones in blas.h)
enum { CG_DONE = 9, CG_STOP = 10, CG_ITERS = 11 };

struct SlotDesc {
    long off;     // complex-element offset of the slot in every batch vector
    long n;       // complex elements of the slot (Ls * 12 * Vhp)
    int nb;       // vector-kernel blocks of the slot
    int block0;   // first vector-kernel block of the slot
    int nhop;     // partials written per hop launch (tiles of its lattice)
    int pad;
    long Vhp;     // row stride of its lattice (layout changes between storage kinds)
};

// blocks of one slot for the vector kernels
int slot_blocks(long n);

// partial[v * pstride + b] = |x_v|^2 over block b of slot v
void bnorm2(int kind, const void* x, const SlotDesc* slots, int nslots, int blocks, double* partial, long pstride,
            const double* scal, hipStream_t st);
// Direction ring of the batched CG: every batch vector of the ring holds one
// search direction of every slot (ring slot q at ring + q * N complex
// elements, N = elements of one batch vector).
// p_dst_v = r_v + beta_v p_src_v (slots not done)
void bcg_p2(int kx, int kp, void* p_dst, const void* p_src, const void* r, const SlotDesc* slots, int nslots,
            int blocks, const double* scal, hipStream_t st);
// x_v += alpha[v * astride + q] p_q for q = 0 .. cnt-1 in this order, with
// p_q ring slot q; a zero alpha (a slot already done) adds nothing
void bcg_accx(int kx, int kp, void* x, const void* ring, long N, const double* alpha, int astride, int cnt,
              const SlotDesc* slots, int nslots, int blocks, hipStream_t st);
// Per-slot reduction of the partials (count: nhop if from_hop, else nb) and
// CG scalar update, one block per slot:
//  mode 0: RR = RR0 = sum; STOP = tol2[v] * sum; ITERS = 0;
//          DONE = (sum == 0); NANFLAG = !finite(sum); a slot with
//          tol2[v] < 0 is retired (DONE = 1, RR = RR0 = STOP = ITERS =
//          NANFLAG = 0, partials not read); one with tol2[v] == 0 is left as it is
//  mode 1: QQ = sum; ALPHA = RR / QQ; alpha_out[v * astride] = ALPHA
//          (done slots: alpha_out[v * astride] = 0 and nothing else)
//  mode 2: RRNEW = sum; BETA = sum / RR; RROLD = RR; RR = sum; ITERS += 1;
//          sum <= STOP with ITERS a multiple of check_every: DONE = 1 (the
//          single solve's rule, which tests every check_every iterations);
//          non-finite: NANFLAG = DONE = 1
//  mode 4: TMP = sum (any slot, done or not)
void bfinalize(const double* partial, long pstride, const SlotDesc* slots, int nslots, double* scal, int mode,
               int from_hop, const double* tol2, hipStream_t st, double* alpha_out = nullptr, int astride = 0,
               int check_every = 1);

}  // namespace dwf
