// Launch interface of the vector kernels (blas.hip).  All `kind` arguments
// are StoreKind values; n counts complex elements.  Internal fields have
// Vh sites per row and row stride Vhp (zero padding in between).
#pragma once

#include <hip/hip_runtime.h>

namespace dwf {

// Slots of the device-resident CG scalar block (doubles).
enum { CG_RR = 0, CG_QQ = 1, CG_ALPHA = 2, CG_BETA = 3, CG_RRNEW = 4, CG_NANFLAG = 5, CG_RR0 = 6,
       CG_TMP = 7, CG_RROLD = 8, CG_NSLOTS = 16 };

int blas_grid(long n);
void pack_full(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long nslices,
               hipStream_t st);
void unpack_full(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long V, long nslices,
                 hipStream_t st);
void pack_half(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long nslices,
               hipStream_t st);
void unpack_half(int kind, void* dst, const void* src, const int* lex, long Vh, long Vhp, long nslices,
                 hipStream_t st);
void pack_chiral_pair_f64(void* dst, const void* b4, const int* lex, long Vh, long Vhp, hipStream_t st);
void project_4d(void* x4, const void* x5, long V, int Ls, hipStream_t st);
void embed_4d(void* e5, const void* y, long V, int Ls, hipStream_t st);
// dst = src in another storage kind; Vhp (row stride) is needed when the two
// kinds group components differently (FP64 vs FP32/BF16)
void convert(int kd, int ks, void* dst, const void* src, long n, hipStream_t st, long Vhp = 0);
void norm2_partial(int kind, const void* x, long n, double* partial, hipStream_t st);
void dot_partial(int kind, const void* x, const void* y, long n, double* partial, hipStream_t st);
// y = a x + b y; a = *sa if sa else ha (same for b); optional partial |y|^2
void axpby(int ky, int kx, void* y, const void* x, long n, const double* sa, double ha, const double* sb,
           double hb, double* partial, hipStream_t st, long Vhp = 0);
// (Vhp: row stride, needed when the operands' layouts differ, FP32 with BF16)
void cg_update_xr(int kx, int kp, void* x, void* r, const void* p, const void* w, long n, const double* alpha,
                  double* partial, hipStream_t st, long Vhp = 0);
void cg_update_p(int kr, int kp, void* p, const void* r, long n, const double* beta, hipStream_t st, long Vhp = 0);
// p_dst = r + beta p_src (r of kind kr; p_src, p_dst of kind kp, distinct buffers)
void cg_update_p2(int kr, int kp, void* p_dst, const void* p_src, const void* r, long n, const double* beta,
                  hipStream_t st, long Vhp = 0);
// x += sum_{i < cnt} alpha[i] p_i, p_i = p_ring + i * n elements of kind kp, added in order i = 0, 1, ...
// with x (kind kx) rounded after each term, as cnt successive x += alpha p updates
void cg_accumulate_x(int kx, int kp, void* x, const void* p_ring, const double* alpha, int cnt, long n,
                     hipStream_t st, long Vhp = 0);
// x += alpha p; p = r + beta p (x, r of kind kx; p of kind kp)
void cg_update_px(int kx, int kp, void* x, void* p, const void* r, long n, const double* alpha, const double* beta,
                  hipStream_t st, long Vhp = 0);
// y += (ar + i ai) x
void caxpy(int kind, void* y, const void* x, long n, double ar, double ai, hipStream_t st);
// FP64 half field(s) of `rows` rows: uniform [-1,1) real and imaginary parts on valid sites
void random_fill_f64(void* v, long rows, long Vh, long Vhp, unsigned long long seed, hipStream_t st);
// mode 0: out[0] = sum; 1: alpha step; 2: beta step; 3: beta after a residual
// replacement (RR = sum, BETA = sum / RROLD) (see CG slots)
void finalize(const double* partial, int nparts, int stride, double* out, int mode, hipStream_t st,
              double* alpha_copy = nullptr);

}  // namespace dwf
