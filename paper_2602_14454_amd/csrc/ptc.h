// Launch interface of the parallel-transport convolution kernels (ptc_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

// One layer for the sites of one parity; see ptc_kernels.hip.
struct PtcLayerParams {
    const float2* in_loc;   // B channels on the output parity (paths 0, +s, -s), or nullptr
    const float2* in_hop;   // B channels on the other parity (the 8 link paths), or nullptr
    float2* out;            // A channels on the output parity
    const float2* W;        // [11][A][B][4][4] complex
    const float2* links;    // FP32 hop links of the output parity [8][9][Vhp]
    const int* nbr;         // neighbour table of the output parity [8][Vhp]
    long Vh, Vhp;
    int Ls, A, B;
    int accumulate;         // 1: out += result
};

void ptc_layer(const PtcLayerParams& P, hipStream_t st);
// weight-gradient rows: (path, b, first a) triples; a-group width ptc_wgrad_ac(A)
int ptc_wgrad_ac(int A);
int ptc_wgrad_blocks(const PtcLayerParams& P);
void ptc_wgrad(const PtcLayerParams& P, const float2* g, const int* rows_dev, int nrows, float* partial,
               float2* grad, hipStream_t st);
int ptc_loss_blocks(long n);
// stats[0] = |y-e|^2/|e|^2, stats[1] = |e|^2, stats[2] = |y-e|^2; g = 2(y-e)/|e|^2 (if g)
void ptc_loss(const float2* y, const float2* e, long n, double* partial, double* stats, float2* g, hipStream_t st);
// d = y - e;  stats[0] = |u|^2/|r|^2, stats[1] = |r|^2, stats[2] = |u|^2;  g = 2 w / stats[1]
void ptc_sub(const float2* y, const float2* e, long n, float2* d, hipStream_t st);
void ptc_norms(const float2* u, const float2* r, long n, double* partial, double* stats, hipStream_t st);
void ptc_scale_grad(const float2* w, long n, const double* stats, float2* g, hipStream_t st);
void ptc_adam(float* w, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, int step,
              hipStream_t st);
void ptc_adjoint(const float2* W, float2* Wt, int A, int B, hipStream_t st);

}  // namespace dwf
