// Learned-preconditioner objects (ptc.cpp).  dwf_ptc and dwf_ptc_pairs are
// the opaque handles of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "dwf_internal.h"

struct dwf_ptc {
    int H;                   // hidden channels
    long nw;                 // complex weights: W1 [11][H][1][16] then W2 [11][1][H][16]
    int step = 0;            // Adam steps taken
    int loss_kind = 1;       // 0: |M r - e|^2/|e|^2;  1: |A (M r - e)|^2/|r|^2 = |A M r - r|^2/|r|^2
    dwf::DevBuf W, G, Wt, m, v, stats, rows;
    int n2 = 0, n1e = 0, n1o = 0;
    long cap_n = 0;
    dwf::DevBuf he, ho, ghe, gho, y, g, lpartial, wpart, d, u, w, to, tv;

    explicit dwf_ptc(int hidden);
    const float2* W1() const;
    const float2* W2() const;
    void reserve(const dwf_op* op);
    // out = M r on FP32 internal even half fields (1 channel)
    void forward(const dwf_op* op, const float2* r, float2* out, hipStream_t st);
    // loss in stats[0] (and g = dL/dy unless value_only), dL/dW in G
    void loss(const dwf_op* op, const float2* r, const float2* e, bool value_only, hipStream_t st);
    void gradient(const dwf_op* op, const float2* r, const float2* e, hipStream_t st);
    void train_step(const dwf_op* op, const float2* r, const float2* e, double lr, hipStream_t st);
};

struct dwf_ptc_pairs {
    const dwf_op* op = nullptr;
    int count = 0;
    long n = 0;              // complex elements of one field
    dwf::DevBuf r, e;        // count FP32 internal even fields each
};

namespace dwf {
long ptc_field_elems(const dwf_op* op);
dwf_ptc* ptc_create(int hidden, unsigned long long seed, double scale);
dwf_ptc_pairs* ptc_pairs_create(const dwf_op* op, const void* b5, unsigned long long seed, int nsnap,
                                const int* snaps, hipStream_t st);
void ptc_train(dwf_ptc* M, int nsets, dwf_ptc_pairs* const* sets, int steps, double lr, unsigned long long seed,
               double* hist, hipStream_t st);
double ptc_eval(dwf_ptc* M, int nsets, dwf_ptc_pairs* const* sets, hipStream_t st);
void ptc_save(const dwf_ptc* M, const char* path);
dwf_ptc* ptc_load(const char* path);
}  // namespace dwf
