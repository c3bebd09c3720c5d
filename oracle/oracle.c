/*
 * FP64 CPU oracle for the domain-wall fermion solve -- TEST INFRASTRUCTURE ONLY.
 * See oracle.h for what is computed, the conventions and who may call this.
 *
 * Plain C99 + OpenMP (parallel loops over lattice sites only).  Every
 * operator is evaluated from its definition in the paper; nothing is
 * factorised, fused or reordered.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define I_ _Complex_I

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

long or_volume(const int dims[4]) {
    return (long)dims[0] * dims[1] * dims[2] * dims[3];
}

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

static void coords_of(const int dims[4], long lex, int c[4]) {
    c[0] = (int)(lex % dims[0]); lex /= dims[0];
    c[1] = (int)(lex % dims[1]); lex /= dims[1];
    c[2] = (int)(lex % dims[2]); lex /= dims[2];
    c[3] = (int)lex;
}

static long lex_of(const int dims[4], const int c[4]) {
    return c[0] + (long)dims[0] * (c[1] + (long)dims[1] * (c[2] + (long)dims[2] * c[3]));
}

static int parity_of(const int dims[4], long lex) {
    int c[4];
    coords_of(dims, lex, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* Neighbour x + dir*mu_hat with periodic wrap; *phase = -1 when an
 * antiperiodic t boundary is crossed. */
static long neighbor(const int dims[4], int apbc, long lex, int mu, int dir, double* phase) {
    int c[4];
    coords_of(dims, lex, c);
    int v = c[mu] + dir;
    *phase = 1.0;
    if (v >= dims[mu]) { v -= dims[mu]; if (mu == 3 && apbc) *phase = -1.0; }
    if (v < 0)         { v += dims[mu]; if (mu == 3 && apbc) *phase = -1.0; }
    c[mu] = v;
    return lex_of(dims, c);
}

void or_site_maps(const int dims[4], int* parity, int* eo, int* lex_of_eo_even, int* lex_of_eo_odd) {
    long V = or_volume(dims);
    for (long x = 0; x < V; ++x) {
        int p = parity_of(dims, x);
        parity[x] = p;
        eo[x] = (int)(x >> 1);
        if (p == 0) lex_of_eo_even[x >> 1] = (int)x;
        else        lex_of_eo_odd[x >> 1] = (int)x;
    }
}

void or_neighbors(const int dims[4], int* nbr) {
    long V = or_volume(dims);
    for (long x = 0; x < V; ++x)
        for (int mu = 0; mu < 4; ++mu) {
            double ph;
            nbr[x * 8 + 2 * mu + 0] = (int)neighbor(dims, 0, x, mu, +1, &ph);
            nbr[x * 8 + 2 * mu + 1] = (int)neighbor(dims, 0, x, mu, -1, &ph);
        }
}

/* ------------------------------------------------------------------ */
/* Gamma matrices, chiral basis (Sec. 2.1: gamma_5 = g1 g2 g3 g4)       */
/* ------------------------------------------------------------------ */

static void matmul4(const or_cplx* a, const or_cplx* b, or_cplx* out) {
    or_cplx t[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            or_cplx s = 0;
            for (int k = 0; k < 4; ++k) s += a[i * 4 + k] * b[k * 4 + j];
            t[i * 4 + j] = s;
        }
    memcpy(out, t, sizeof t);
}

void or_gamma(int mu, or_cplx out[16]) {
    /* Pauli matrices */
    const or_cplx sig[3][4] = {
        {0, 1, 1, 0},
        {0, -I_, I_, 0},
        {1, 0, 0, -1},
    };
    memset(out, 0, 16 * sizeof(or_cplx));
    if (mu >= 0 && mu < 3) {
        /* [[0, -i sigma],[i sigma, 0]] */
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                out[i * 4 + (j + 2)] = -I_ * sig[mu][i * 2 + j];
                out[(i + 2) * 4 + j] = I_ * sig[mu][i * 2 + j];
            }
    } else if (mu == 3) {
        out[0 * 4 + 2] = out[1 * 4 + 3] = out[2 * 4 + 0] = out[3 * 4 + 1] = 1;
    } else {
        or_cplx g[4][16];
        for (int k = 0; k < 4; ++k) or_gamma(k, g[k]);
        or_cplx t[16];
        matmul4(g[0], g[1], t);
        matmul4(t, g[2], t);
        matmul4(t, g[3], out);
    }
}

/* (1 + sign*gamma_mu) as a full 4x4 matrix */
static void one_pm_gamma(int mu, double sign, or_cplx out[16]) {
    or_gamma(mu, out);
    for (int i = 0; i < 16; ++i) out[i] *= sign;
    for (int i = 0; i < 4; ++i) out[i * 4 + i] += 1.0;
}

/* P_+ = (1 + gamma_5)/2, P_- = (1 - gamma_5)/2 as full 4x4 matrices */
static void chiral_projector(double sign, or_cplx out[16]) {
    or_cplx g5[16];
    or_gamma(4, g5);
    for (int i = 0; i < 16; ++i) out[i] = 0.5 * sign * g5[i];
    for (int i = 0; i < 4; ++i) out[i * 4 + i] += 0.5;
}

/* ------------------------------------------------------------------ */
/* Wilson operator D_W(-M0), Sec. 2.1 eq. Wilson_matrix with M = -M0    */
/*   D_W psi(x) = (4 - M0) psi(x)                                        */
/*     - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)                       */
/*                  + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]              */
/* Adjoint: swap (1 - g_mu) <-> (1 + g_mu) (gamma Hermitian).            */
/* parity_mask: bit 0 -> compute even outputs, bit 1 -> odd outputs;     */
/* outputs of the other parity are set to zero.                          */
/* ------------------------------------------------------------------ */

void or_wilson(const or_params* p, const or_cplx* U, const or_cplx* in, or_cplx* out,
               int dagger, int parity_mask) {
    const long V = or_volume(p->dims);
    or_cplx fwd[4][16], bwd[4][16];
    for (int mu = 0; mu < 4; ++mu) {
        double sf = dagger ? +1.0 : -1.0;
        one_pm_gamma(mu, sf, fwd[mu]);   /* (1 - g) or (1 + g) for the x+mu hop */
        one_pm_gamma(mu, -sf, bwd[mu]);  /* (1 + g) or (1 - g) for the x-mu hop */
    }
    const double diag = 4.0 - p->M0;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x) {
        or_cplx* o = out + x * 12;
        int par = parity_of(p->dims, x);
        if (!((parity_mask >> par) & 1)) {
            for (int k = 0; k < 12; ++k) o[k] = 0;
            continue;
        }
        or_cplx acc[12];
        for (int k = 0; k < 12; ++k) acc[k] = 0;
        for (int mu = 0; mu < 4; ++mu) {
            for (int dir = 0; dir < 2; ++dir) {
                double ph;
                long y = neighbor(p->dims, p->antiperiodic_t, x, mu, dir == 0 ? +1 : -1, &ph);
                /* colour part: U_mu(x) psi(y) or U_mu(y)^dag psi(y) */
                or_cplx cpsi[12];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        or_cplx s = 0;
                        for (int b = 0; b < 3; ++b) {
                            or_cplx u = (dir == 0) ? U[(x * 4 + mu) * 9 + a * 3 + b]
                                                   : conj(U[(y * 4 + mu) * 9 + b * 3 + a]);
                            s += u * in[y * 12 + sp * 3 + b];
                        }
                        cpsi[sp * 3 + a] = s;
                    }
                /* spin part: full 4x4 (1 -/+ gamma_mu) */
                const or_cplx* S = (dir == 0) ? fwd[mu] : bwd[mu];
                for (int sp = 0; sp < 4; ++sp)
                    for (int a = 0; a < 3; ++a) {
                        or_cplx s = 0;
                        for (int tp = 0; tp < 4; ++tp) s += S[sp * 4 + tp] * cpsi[tp * 3 + a];
                        acc[sp * 3 + a] += ph * s;
                    }
            }
        }
        for (int k = 0; k < 12; ++k) o[k] = diag * in[x * 12 + k] - 0.5 * acc[k];
    }
}

/* ------------------------------------------------------------------ */
/* 5D domain-wall operator as a block matrix in s (Sec. 2.3,            */
/* eq. domainwall_neff; alpha = 1 is eq. domainwall_general of Sec. 2.2)*/
/* Each block is coef * D_kind * S with D_kind in {D_+, D_-} and S a    */
/* 4x4 spin matrix; D_+ = b D_W + 1, D_- = c D_W - 1.                    */
/* ------------------------------------------------------------------ */

typedef struct {
    int row, col;
    int kind;        /* 0: D_+, 1: D_- */
    double coef;
    or_cplx S[16];
} or_block;

static void spin_lincomb(const or_cplx* A, double a, const or_cplx* B, double b, or_cplx* out) {
    for (int i = 0; i < 16; ++i) out[i] = a * A[i] + b * B[i];
}

/* Returns number of blocks written to blk (at most 3*Ls). */
static int build_blocks(const or_params* p, or_block* blk) {
    const int Ls = p->Ls;
    const double al = p->alpha;
    or_cplx Pp[16], Pm[16], one[16];
    chiral_projector(+1.0, Pp);
    chiral_projector(-1.0, Pm);
    memset(one, 0, sizeof one);
    for (int i = 0; i < 4; ++i) one[i * 4 + i] = 1.0;
    int n = 0;
#define ADD(r, c_, k, cf, Smat) do { blk[n].row = (r); blk[n].col = (c_); blk[n].kind = (k); \
        blk[n].coef = (cf); memcpy(blk[n].S, (Smat), sizeof(or_cplx) * 16); ++n; } while (0)
    for (int r = 0; r < Ls; ++r) {
        /* diagonal block */
        if (r == 0) {
            or_cplx S[16]; spin_lincomb(Pm, 1.0, Pp, al, S);   /* D_+ (P_- + alpha P_+) */
            ADD(r, r, 0, 1.0, S);
        } else if (r == Ls - 1) {
            or_cplx S[16]; spin_lincomb(Pp, 1.0, Pm, al, S);   /* D_+ (P_+ + alpha P_-) */
            ADD(r, r, 0, 1.0, S);
        } else {
            ADD(r, r, 0, al, one);                             /* alpha D_+ */
        }
        /* super-diagonal alpha D_- P_- and sub-diagonal alpha D_- P_+ */
        if (r + 1 < Ls) ADD(r, r + 1, 1, al, Pm);
        if (r - 1 >= 0) ADD(r, r - 1, 1, al, Pp);
    }
    /* corner blocks, unchanged by alpha: -m D_- P_+ (top right), -m D_- P_- (bottom left) */
    ADD(0, Ls - 1, 1, -p->m, Pp);
    ADD(Ls - 1, 0, 1, -p->m, Pm);
#undef ADD
    return n;
}

/* coefficients of D_+^(i) and D_-^(i) in row i (i = 0..Ls-1) */
static double coef_b(const or_params* p, int i) { return p->bs ? p->bs[i] : p->b; }
static double coef_c(const or_params* p, int i) { return p->cs ? p->cs[i] : p->c; }

static void apply_spin(const or_cplx* S, const or_cplx* in4, or_cplx* out4, long V, int adjoint) {
#pragma omp parallel for schedule(static)
    for (long x = 0; x < V; ++x)
        for (int sp = 0; sp < 4; ++sp)
            for (int a = 0; a < 3; ++a) {
                or_cplx s = 0;
                for (int tp = 0; tp < 4; ++tp) {
                    or_cplx m = adjoint ? conj(S[tp * 4 + sp]) : S[sp * 4 + tp];
                    s += m * in4[x * 12 + tp * 3 + a];
                }
                out4[x * 12 + sp * 3 + a] = s;
            }
}

void or_dwf_apply(const or_params* p, const or_cplx* U, const or_cplx* in5, or_cplx* out5,
                  int dagger, int parity_mask) {
    const long V = or_volume(p->dims);
    const int Ls = p->Ls;
    const long n4 = V * 12;
    or_block* blk = (or_block*)malloc(sizeof(or_block) * (3 * Ls + 2));
    int nb = build_blocks(p, blk);
    or_cplx* t1 = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    or_cplx* t2 = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    memset(out5, 0, sizeof(or_cplx) * n4 * Ls);
    for (int k = 0; k < nb; ++k) {
        const or_block* B = &blk[k];
        /* coefficient of D_W in D_kind of this block's row */
        const double dw = B->kind == 0 ? coef_b(p, B->row) : coef_c(p, B->row);
        const double id = B->kind == 0 ? 1.0 : -1.0;    /* coefficient of 1 in D_kind   */
        if (!dagger) {
            /* out_row += coef * D_kind (S in_col) */
            apply_spin(B->S, in5 + B->col * n4, t1, V, 0);
            or_wilson(p, U, t1, t2, 0, parity_mask);
            or_cplx* o = out5 + B->row * n4;
#pragma omp parallel for schedule(static)
            for (long x = 0; x < V; ++x) {
                if (!((parity_mask >> parity_of(p->dims, x)) & 1)) continue;
                for (int j = 0; j < 12; ++j)
                    o[x * 12 + j] += B->coef * (dw * t2[x * 12 + j] + id * t1[x * 12 + j]);
            }
        } else {
            /* adjoint of block (row,col) acts from row to col:
             * out_col += coef * S^dag D_kind^dag in_row, D_kind^dag = dw D_W^dag + id */
            or_wilson(p, U, in5 + B->row * n4, t2, 1, 3);
            const or_cplx* ir = in5 + B->row * n4;
#pragma omp parallel for schedule(static)
            for (long x = 0; x < V; ++x)
                for (int j = 0; j < 12; ++j) t2[x * 12 + j] = dw * t2[x * 12 + j] + id * ir[x * 12 + j];
            apply_spin(B->S, t2, t1, V, 1);
            or_cplx* o = out5 + B->col * n4;
#pragma omp parallel for schedule(static)
            for (long x = 0; x < V; ++x) {
                if (!((parity_mask >> parity_of(p->dims, x)) & 1)) continue;
                for (int j = 0; j < 12; ++j) o[x * 12 + j] += B->coef * t1[x * 12 + j];
            }
        }
    }
    free(t1);
    free(t2);
    free(blk);
}

/* ------------------------------------------------------------------ */
/* Site-diagonal block D_ee = D_oo: the block matrix with D_W replaced  */
/* by its site-diagonal part (4 - M0) * 1.  Matrix over (s, spin), the  */
/* colour index is a spectator.  Mloc[(r*4+sp)*(4Ls) + (c*4+tp)].        */
/* ------------------------------------------------------------------ */

void or_local_block(const or_params* p, or_cplx* Mloc) {
    const int Ls = p->Ls, n = 4 * Ls;
    or_block* blk = (or_block*)malloc(sizeof(or_block) * (3 * Ls + 2));
    int nb = build_blocks(p, blk);
    memset(Mloc, 0, sizeof(or_cplx) * n * n);
    const double dwdiag = 4.0 - p->M0;
    for (int k = 0; k < nb; ++k) {
        const or_block* B = &blk[k];
        double dw = B->kind == 0 ? coef_b(p, B->row) : coef_c(p, B->row);
        double id = B->kind == 0 ? 1.0 : -1.0;
        double f = B->coef * (dw * dwdiag + id);
        for (int sp = 0; sp < 4; ++sp)
            for (int tp = 0; tp < 4; ++tp)
                Mloc[(B->row * 4 + sp) * n + (B->col * 4 + tp)] += f * B->S[sp * 4 + tp];
    }
    free(blk);
}

/* Gauss-Jordan elimination with partial pivoting. Returns 0 on success. */
int or_invert_dense(int n, const or_cplx* A, or_cplx* Ainv) {
    or_cplx* a = (or_cplx*)malloc(sizeof(or_cplx) * n * n);
    memcpy(a, A, sizeof(or_cplx) * n * n);
    for (int i = 0; i < n * n; ++i) Ainv[i] = 0;
    for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = cabs(a[col * n + col]);
        for (int r = col + 1; r < n; ++r)
            if (cabs(a[r * n + col]) > best) { best = cabs(a[r * n + col]); piv = r; }
        if (best == 0.0) { free(a); return -1; }
        if (piv != col)
            for (int j = 0; j < n; ++j) {
                or_cplx t = a[col * n + j]; a[col * n + j] = a[piv * n + j]; a[piv * n + j] = t;
                t = Ainv[col * n + j]; Ainv[col * n + j] = Ainv[piv * n + j]; Ainv[piv * n + j] = t;
            }
        or_cplx inv = 1.0 / a[col * n + col];
        for (int j = 0; j < n; ++j) { a[col * n + j] *= inv; Ainv[col * n + j] *= inv; }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            or_cplx f = a[r * n + col];
            if (f == 0) continue;
            for (int j = 0; j < n; ++j) {
                a[r * n + j] -= f * a[col * n + j];
                Ainv[r * n + j] -= f * Ainv[col * n + j];
            }
        }
    }
    free(a);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Even-odd pieces (Sec. 2.3, eq. eo_decomposition and                 */
/* eq. even-odd_linear_equation), all by restriction of or_dwf_apply.   */
/* ------------------------------------------------------------------ */

static void half_to_full(const or_params* p, const or_cplx* h, int parity, or_cplx* full) {
    const long V = or_volume(p->dims), Vh = V / 2;
    memset(full, 0, sizeof(or_cplx) * V * 12 * p->Ls);
    for (int s = 0; s < p->Ls; ++s)
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x)
            if (parity_of(p->dims, x) == parity)
                memcpy(full + (s * V + x) * 12, h + (s * Vh + (x >> 1)) * 12, sizeof(or_cplx) * 12);
}

static void full_to_half(const or_params* p, const or_cplx* full, int parity, or_cplx* h) {
    const long V = or_volume(p->dims), Vh = V / 2;
    for (int s = 0; s < p->Ls; ++s)
#pragma omp parallel for schedule(static)
        for (long x = 0; x < V; ++x)
            if (parity_of(p->dims, x) == parity)
                memcpy(h + (s * Vh + (x >> 1)) * 12, full + (s * V + x) * 12, sizeof(or_cplx) * 12);
}

/* y = Minv x per (site, colour) on a half-lattice vector; adjoint uses Minv^dag */
static void apply_local_inverse(const or_params* p, const or_cplx* Minv, const or_cplx* x,
                                or_cplx* y, int adjoint) {
    const long Vh = or_volume(p->dims) / 2;
    const int Ls = p->Ls, n = 4 * Ls;
#pragma omp parallel for schedule(static)
    for (long e = 0; e < Vh; ++e)
        for (int a = 0; a < 3; ++a)
            for (int r = 0; r < Ls; ++r)
                for (int sp = 0; sp < 4; ++sp) {
                    or_cplx acc = 0;
                    for (int c = 0; c < Ls; ++c)
                        for (int tp = 0; tp < 4; ++tp) {
                            int i = r * 4 + sp, j = c * 4 + tp;
                            or_cplx m = adjoint ? conj(Minv[j * n + i]) : Minv[i * n + j];
                            acc += m * x[((c * Vh + e) * 4 + tp) * 3 + a];
                        }
                    y[((r * Vh + e) * 4 + sp) * 3 + a] = acc;
                }
}

static or_cplx* local_inverse(const or_params* p) {
    const int n = 4 * p->Ls;
    or_cplx* M = (or_cplx*)malloc(sizeof(or_cplx) * n * n);
    or_cplx* Minv = (or_cplx*)malloc(sizeof(or_cplx) * n * n);
    or_local_block(p, M);
    or_invert_dense(n, M, Minv);
    free(M);
    return Minv;
}

/* D_{dst,src} x_src (restriction of the 5D operator), or its adjoint block */
static void offdiag(const or_params* p, const or_cplx* U, const or_cplx* x_src, int src_parity,
                    or_cplx* y_dst, int dagger, or_cplx* fa, or_cplx* fb) {
    half_to_full(p, x_src, src_parity, fa);
    or_dwf_apply(p, U, fa, fb, dagger, 1 << (1 - src_parity));
    full_to_half(p, fb, 1 - src_parity, y_dst);
}

/* D^hat = 1 - D_ee^-1 D_eo D_oo^-1 D_oe (dagger: 1 - D_oe^dag D_oo^-dag D_eo^dag D_ee^-dag) */
void or_dhat(const or_params* p, const or_cplx* U, const or_cplx* in_e, or_cplx* out_e, int dagger) {
    const long V = or_volume(p->dims), Vh = V / 2;
    const long nh = Vh * 12 * p->Ls;
    or_cplx* Minv = local_inverse(p);
    or_cplx* fa = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* fb = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* h1 = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* h2 = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    if (!dagger) {
        offdiag(p, U, in_e, 0, h1, 0, fa, fb);      /* D_oe x_e          */
        apply_local_inverse(p, Minv, h1, h2, 0);    /* D_oo^-1 ...       */
        offdiag(p, U, h2, 1, h1, 0, fa, fb);        /* D_eo ...          */
        apply_local_inverse(p, Minv, h1, h2, 0);    /* D_ee^-1 ...       */
    } else {
        apply_local_inverse(p, Minv, in_e, h1, 1);  /* D_ee^-dag x_e     */
        offdiag(p, U, h1, 0, h2, 1, fa, fb);        /* D_eo^dag ...      */
        apply_local_inverse(p, Minv, h2, h1, 1);    /* D_oo^-dag ...     */
        offdiag(p, U, h1, 1, h2, 1, fa, fb);        /* D_oe^dag ...      */
    }
    for (long i = 0; i < nh; ++i) out_e[i] = in_e[i] - h2[i];
    free(Minv); free(fa); free(fb); free(h1); free(h2);
}

/* b~_e = D_ee^-1 (b_e - D_eo D_oo^-1 b_o) */
void or_schur_rhs(const or_params* p, const or_cplx* U, const or_cplx* b5, or_cplx* bt_e) {
    const long V = or_volume(p->dims), Vh = V / 2;
    const long nh = Vh * 12 * p->Ls;
    or_cplx* Minv = local_inverse(p);
    or_cplx* fa = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* fb = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* be = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* bo = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* h = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    full_to_half(p, b5, 0, be);
    full_to_half(p, b5, 1, bo);
    apply_local_inverse(p, Minv, bo, h, 0);
    offdiag(p, U, h, 1, bo, 0, fa, fb);           /* bo <- D_eo D_oo^-1 b_o */
    for (long i = 0; i < nh; ++i) be[i] -= bo[i];
    apply_local_inverse(p, Minv, be, bt_e, 0);
    free(Minv); free(fa); free(fb); free(be); free(bo); free(h);
}

/* x_o = D_oo^-1 (b_o - D_oe x_e); x5 = (x_e, x_o) on the full lattice */
void or_reconstruct(const or_params* p, const or_cplx* U, const or_cplx* x_e,
                    const or_cplx* b5, or_cplx* x5) {
    const long V = or_volume(p->dims), Vh = V / 2;
    const long nh = Vh * 12 * p->Ls;
    or_cplx* Minv = local_inverse(p);
    or_cplx* fa = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* fb = (or_cplx*)malloc(sizeof(or_cplx) * V * 12 * p->Ls);
    or_cplx* bo = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* h = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* xo = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    full_to_half(p, b5, 1, bo);
    offdiag(p, U, x_e, 0, h, 0, fa, fb);
    for (long i = 0; i < nh; ++i) bo[i] -= h[i];
    apply_local_inverse(p, Minv, bo, xo, 0);
    half_to_full(p, x_e, 0, x5);
    half_to_full(p, xo, 1, fa);
    for (long i = 0; i < V * 12 * p->Ls; ++i) x5[i] += fa[i];
    free(Minv); free(fa); free(fb); free(bo); free(h); free(xo);
}

static double norm2(const or_cplx* v, long n) {
    double s = 0;
    for (long i = 0; i < n; ++i) s += creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]);
    return s;
}

/* CG on D^dag D x_e = D^dag b~_e from x_e = 0 (Sec. 2.3, CGNR paragraph).
 * Stops when |r|/|D^dag b~_e| < tol on the recursive residual.
 * Returns the iteration count, or -1 if maxiter was reached. */
int or_cgnr_even(const or_params* p, const or_cplx* U, const or_cplx* bt_e, or_cplx* x_e,
                 double tol, int maxiter) {
    const long nh = or_volume(p->dims) / 2 * 12 * p->Ls;
    or_cplx* r = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* pv = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* q = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* s = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_dhat(p, U, bt_e, r, 1);
    double rhs2 = norm2(r, nh), rr = rhs2;
    for (long i = 0; i < nh; ++i) { x_e[i] = 0; pv[i] = r[i]; }
    int k = 0, done = (rhs2 == 0.0);
    while (!done && k < maxiter) {
        or_dhat(p, U, pv, q, 0);
        double a = rr / norm2(q, nh);
        or_dhat(p, U, q, s, 1);
        for (long i = 0; i < nh; ++i) { x_e[i] += a * pv[i]; r[i] -= a * s[i]; }
        double rr_new = norm2(r, nh);
        ++k;
        if (rr_new <= tol * tol * rhs2) { done = 1; break; }
        double b = rr_new / rr;
        rr = rr_new;
        for (long i = 0; i < nh; ++i) pv[i] = r[i] + b * pv[i];
    }
    free(r); free(pv); free(q); free(s);
    return done ? k : -1;
}

double or_true_residual(const or_params* p, const or_cplx* U, const or_cplx* x5, const or_cplx* b5) {
    const long n = or_volume(p->dims) * 12 * p->Ls;
    or_cplx* t = (or_cplx*)malloc(sizeof(or_cplx) * n);
    or_dwf_apply(p, U, x5, t, 0, 3);
    for (long i = 0; i < n; ++i) t[i] = b5[i] - t[i];
    double r = sqrt(norm2(t, n) / norm2(b5, n));
    free(t);
    return r;
}

/* Full solve D^(alpha) x5 = b5: Schur RHS, CGNR, reconstruction, then
 * defect-correction restarts (all FP64) until the true 5D relative
 * residual is <= tol.  Returns total CG iterations (negative if maxiter hit). */
int or_solve(const or_params* p, const or_cplx* U, const or_cplx* b5, or_cplx* x5,
             double tol, int maxiter, double* true_res) {
    const long V = or_volume(p->dims), n = V * 12 * p->Ls, nh = n / 2;
    or_cplx* bt = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* xe = (or_cplx*)malloc(sizeof(or_cplx) * nh);
    or_cplx* r5 = (or_cplx*)malloc(sizeof(or_cplx) * n);
    or_cplx* dx = (or_cplx*)malloc(sizeof(or_cplx) * n);
    const double b2 = norm2(b5, n);
    memset(x5, 0, sizeof(or_cplx) * n);
    memcpy(r5, b5, sizeof(or_cplx) * n);
    int total = 0, ok = 0;
    double res = 1.0;
    for (int outer = 0; outer < 20 && total < maxiter; ++outer) {
        or_schur_rhs(p, U, r5, bt);
        int it = or_cgnr_even(p, U, bt, xe, 0.1 * tol, maxiter - total);
        total += it < 0 ? (maxiter - total) : it;
        or_reconstruct(p, U, xe, r5, dx);
        for (long i = 0; i < n; ++i) x5[i] += dx[i];
        or_dwf_apply(p, U, x5, r5, 0, 3);
        for (long i = 0; i < n; ++i) r5[i] = b5[i] - r5[i];
        res = sqrt(norm2(r5, n) / b2);
        if (res <= tol) { ok = 1; break; }
    }
    if (true_res) *true_res = res;
    free(bt); free(xe); free(r5); free(dx);
    return ok ? total : -total;
}

/* b5 = (-D_-) P^dag (0,...,0,b4)^T: b5(s=1) = -D_- P_+ b4, b5(s=Ls) = -D_- P_- b4 */
void or_source_4d(const or_params* p, const or_cplx* U, const or_cplx* b4, or_cplx* b5) {
    const long V = or_volume(p->dims), n4 = V * 12;
    or_cplx Pp[16], Pm[16];
    chiral_projector(+1.0, Pp);
    chiral_projector(-1.0, Pm);
    or_cplx* t = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    or_cplx* w = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    memset(b5, 0, sizeof(or_cplx) * n4 * p->Ls);
    for (int side = 0; side < 2; ++side) {
        int s = side == 0 ? 0 : p->Ls - 1;
        apply_spin(side == 0 ? Pp : Pm, b4, t, V, 0);
        or_wilson(p, U, t, w, 0, 3);
        /* -D_-^(s) t = -(c_s D_W t - t) */
        const double cs = coef_c(p, s);
        for (long i = 0; i < n4; ++i) b5[s * n4 + i] += -(cs * w[i] - t[i]);
    }
    free(t);
    free(w);
}

/* x4 = [P^dag x5]_{s=1} = P_- x5(s=1) + P_+ x5(s=Ls) */
void or_project_4d(const or_params* p, const or_cplx* x5, or_cplx* x4) {
    const long V = or_volume(p->dims), n4 = V * 12;
    or_cplx Pp[16], Pm[16];
    chiral_projector(+1.0, Pp);
    chiral_projector(-1.0, Pm);
    or_cplx* t = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    apply_spin(Pm, x5, x4, V, 0);
    apply_spin(Pp, x5 + (long)(p->Ls - 1) * n4, t, V, 0);
    for (long i = 0; i < n4; ++i) x4[i] += t[i];
    free(t);
}

/* 4D residual of the projected solution.  With
 *   D_eff(m) y = [P^dag D(m=1)^-1 D(m) P (y,0,...,0)]_{s=1}   (alpha = 1),
 * the map G: b4 -> x4 satisfies (1-m) G + 1 = D_eff^-1, so
 *   r4 = b4 - D_eff((1-m) x4 + b4)
 * vanishes for the exact x4 of any alpha.  The inner m = 1 solve runs to
 * tol_inner.  Returns |r4| / |b4|. */
double or_residual_4d(const or_params* p, const or_cplx* U, const or_cplx* x4,
                      const or_cplx* b4, double tol_inner) {
    const long V = or_volume(p->dims), n4 = V * 12, n = n4 * p->Ls;
    or_params pm = *p, p1 = *p;
    pm.alpha = 1.0;
    p1.alpha = 1.0;
    p1.m = 1.0;
    or_cplx Pp[16], Pm[16];
    chiral_projector(+1.0, Pp);
    chiral_projector(-1.0, Pm);
    or_cplx* y = (or_cplx*)malloc(sizeof(or_cplx) * n4);
    or_cplx* e5 = (or_cplx*)malloc(sizeof(or_cplx) * n);
    or_cplx* z5 = (or_cplx*)malloc(sizeof(or_cplx) * n);
    or_cplx* v5 = (or_cplx*)malloc(sizeof(or_cplx) * n);
    for (long i = 0; i < n4; ++i) y[i] = (1.0 - p->m) * x4[i] + b4[i];
    /* P (y, 0, ..., 0): first block column of P is (P_-, 0, ..., 0, P_+) */
    memset(e5, 0, sizeof(or_cplx) * n);
    apply_spin(Pm, y, e5, V, 0);
    apply_spin(Pp, y, e5 + (long)(p->Ls - 1) * n4, V, 0);
    or_dwf_apply(&pm, U, e5, z5, 0, 3);
    double tr;
    or_solve(&p1, U, z5, v5, tol_inner, 100000, &tr);
    or_project_4d(p, v5, y);
    double num = 0, den = 0;
    for (long i = 0; i < n4; ++i) {
        or_cplx d = b4[i] - y[i];
        num += creal(d) * creal(d) + cimag(d) * cimag(d);
        den += creal(b4[i]) * creal(b4[i]) + cimag(b4[i]) * cimag(b4[i]);
    }
    free(y); free(e5); free(z5); free(v5);
    return sqrt(num / den);
}
