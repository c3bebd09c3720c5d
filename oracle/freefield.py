"""Momentum-space closed forms for unit gauge links -- TEST INFRASTRUCTURE.

With U = 1 and psi(x) = exp(i p.x) u, the Wilson operator of the paper
(Sec. 2.1, eq. Wilson_matrix, mass -M0) acts as the 4x4 spin matrix

    D_W(p) = -M0 + sum_mu (1 - cos p_mu) + i sum_mu gamma_mu sin p_mu,

with p_mu = 2 pi n / L_mu for x, y, z and (2n+1) pi / L_t for an antiperiodic
t direction.  The 4D operator reached by the domain-wall solve with the
paper's source and projection (Sec. 2.2 eq. 4d_quark_field, Sec. 2.3
eq. 5D_linear_equation) has the closed form of the Moebius domain-wall
literature the paper builds on (its ref. Brower:2004xi):

    D_eff(m) = (1+m)/2 + (1-m)/2 gamma_5 eps_Ls(H),
    H        = gamma_5 (b+c) D_W (2 + (b-c) D_W)^-1   (Hermitian),
    eps_Ls(H) = [(1+H)^Ls - (1-H)^Ls] [(1+H)^Ls + (1-H)^Ls]^-1,

and the 4D solution is x4 = G b4 with (1-m) G + 1 = D_eff^-1.  Neither
formula mentions the fifth-dimension block structure, so they pin the
oracle's 5D operator, source, projection, Schur solve and CG from outside.
It also does not depend on alpha (Sec. 2.3, the 4D solution is unchanged).
"""
from __future__ import annotations

import itertools

import numpy as np

from . import gamma as _gamma


def gammas():
    return [_gamma(mu) for mu in range(4)], _gamma(4)


def momenta(dims, antiperiodic_t=True):
    """All lattice momenta (p_x, p_y, p_z, p_t)."""
    axes = []
    for mu, L in enumerate(dims):
        n = np.arange(L)
        if mu == 3 and antiperiodic_t:
            axes.append((2 * n + 1) * np.pi / L)
        else:
            axes.append(2 * n * np.pi / L)
    return [np.array(p) for p in itertools.product(*axes)]


def dw_of_p(p, M0):
    g, _ = gammas()
    D = (-M0 + np.sum(1 - np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        D = D + 1j * np.sin(p[mu]) * g[mu]
    return D


def hermitian_kernel(Dw, b, c):
    _, g5 = gammas()
    n = Dw.shape[0]
    G5 = np.kron(np.eye(n // 4), g5) if n != 4 else g5
    return G5 @ ((b + c) * Dw) @ np.linalg.inv(2 * np.eye(n) + (b - c) * Dw)


def eps_polar(H, Ls):
    w, v = np.linalg.eigh(0.5 * (H + H.conj().T))
    f = ((1 + w) ** Ls - (1 - w) ** Ls) / ((1 + w) ** Ls + (1 - w) ** Ls)
    return (v * f) @ v.conj().T


def deff_from_dw(Dw, Ls, m, b, c):
    """Closed-form D_eff for any D_W given as a dense matrix (spin-major blocks of 4)."""
    _, g5 = gammas()
    n = Dw.shape[0]
    G5 = np.kron(np.eye(n // 4), g5) if n != 4 else g5
    H = hermitian_kernel(Dw, b, c)
    return 0.5 * (1 + m) * np.eye(n) + 0.5 * (1 - m) * G5 @ eps_polar(H, Ls)


def g_from_dw(Dw, Ls, m, b, c):
    """The map b4 -> x4: G = (D_eff^-1 - 1) / (1 - m)."""
    D = deff_from_dw(Dw, Ls, m, b, c)
    n = D.shape[0]
    return (np.linalg.inv(D) - np.eye(n)) / (1 - m)


def plane_wave_4d(dims, p, u):
    """psi[lex, spin, colour] = exp(i p.x) u[spin, colour]."""
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    ph = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t)).reshape(-1)
    return ph[:, None, None] * np.asarray(u)[None, :, :]


# ---------------------------------------------------------------------------
# Momentum-space 5D operator and even-odd Schur complement (free field).
# On the even sub-lattice exp(i p.x) u is mapped by the Schur operator to
# exp(i p.x) D^(p) u, so the spectrum of D^dag D^ is the union over p of the
# squared singular values of the (4 Ls) x (4 Ls) matrix D^(p).
# ---------------------------------------------------------------------------

def _blocks5(Ls, m, alpha, Pp, Pm):
    """Block list (row, col, kind, coef, S) of the paper's Neff-form matrix."""
    one = np.eye(4)
    out = []
    for r in range(Ls):
        if r == 0:
            out.append((r, r, 0, 1.0, Pm + alpha * Pp))
        elif r == Ls - 1:
            out.append((r, r, 0, 1.0, Pp + alpha * Pm))
        else:
            out.append((r, r, 0, alpha, one))
        if r + 1 < Ls:
            out.append((r, r + 1, 1, alpha, Pm))
        if r - 1 >= 0:
            out.append((r, r - 1, 1, alpha, Pp))
    out.append((0, Ls - 1, 1, -m, Pp))
    out.append((Ls - 1, 0, 1, -m, Pm))
    return out


def dwf5_of(Dw_part, one_part, Ls, m, b, c, alpha):
    """5D block matrix with D_+ = b*Dw_part + one_part, D_- = c*Dw_part - one_part."""
    _, g5 = gammas()
    Pp = 0.5 * (np.eye(4) + g5)
    Pm = 0.5 * (np.eye(4) - g5)
    D = np.zeros((4 * Ls, 4 * Ls), dtype=np.complex128)
    for (r, cc, kind, coef, S) in _blocks5(Ls, m, alpha, Pp, Pm):
        Dk = (b * Dw_part + one_part) if kind == 0 else (c * Dw_part - one_part)
        D[4 * r:4 * r + 4, 4 * cc:4 * cc + 4] += coef * Dk @ S
    return D


def dhat_of_p(p, Ls, M0, m, b, c, alpha):
    g, _ = gammas()
    Hp = sum(2 * (np.cos(p[mu]) * np.eye(4) - 1j * np.sin(p[mu]) * g[mu]) for mu in range(4))
    Dee = dwf5_of((4 - M0) * np.eye(4), np.eye(4), Ls, m, b, c, alpha)
    Deo = dwf5_of(-0.5 * Hp, np.zeros((4, 4)), Ls, m, b, c, alpha)
    Di = np.linalg.inv(Dee)
    return np.eye(4 * Ls) - Di @ Deo @ Di @ Deo


def normal_spectrum_extremes(dims, Ls, M0, m, b, c, alpha, antiperiodic_t=True):
    lo, hi = np.inf, 0.0
    for p in momenta(dims, antiperiodic_t):
        s = np.linalg.svd(dhat_of_p(p, Ls, M0, m, b, c, alpha), compute_uv=False)
        lo = min(lo, s.min() ** 2)
        hi = max(hi, s.max() ** 2)
    return lo, hi


# ---------------------------------------------------------------------------
# s-dependent coefficients (Sec. 2.2: b_i, c_i depending on the row i).  For
# b_s - c_s = kappa independent of s (Moebius-type, including Chiu's
# b_s = c_s) the kernels H_s = (b_s + c_s) Ht with
# Ht = g5 D_W (2 + kappa D_W)^-1 commute, and the 4D operator is
#   D_eff = (1+m)/2 + (1-m)/2 g5 eps,
#   eps = (prod_s (1 + H_s) - prod_s (1 - H_s)) / (prod_s (1 + H_s) + prod_s (1 - H_s)).
# ---------------------------------------------------------------------------

def eps_product(Ht, a):
    """eps of the kernels a_s * Ht (Ht Hermitian), by eigendecomposition."""
    w, v = np.linalg.eigh(0.5 * (Ht + Ht.conj().T))
    P = np.prod(1 + np.outer(a, w), axis=0)
    Q = np.prod(1 - np.outer(a, w), axis=0)
    return (v * ((P - Q) / (P + Q))) @ v.conj().T


def deff_from_dw_sdep(Dw, m, bs, cs):
    bs, cs = np.asarray(bs, float), np.asarray(cs, float)
    kappa = bs[0] - cs[0]
    assert np.all(np.abs((bs - cs) - kappa) < 1e-14), "closed form needs b_s - c_s independent of s"
    _, g5 = gammas()
    n = Dw.shape[0]
    G5 = np.kron(np.eye(n // 4), g5) if n != 4 else g5
    Ht = hermitian_kernel(Dw, 0.5 * (1 + kappa), 0.5 * (1 - kappa))   # (b + c) = 1, (b - c) = kappa
    return 0.5 * (1 + m) * np.eye(n) + 0.5 * (1 - m) * G5 @ eps_product(Ht, bs + cs)


def g_from_deff(D, m):
    n = D.shape[0]
    return (np.linalg.inv(D) - np.eye(n)) / (1 - m)
