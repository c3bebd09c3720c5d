"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no solver arithmetic.  It produces the gauge links and the
sources that both sides take as inputs:

* a counter-based random stream (SplitMix64 applied to seed-keyed counters,
  Box-Muller for Gaussians), so every draw is a pure function of
  (seed, stream, index) and generation vectorises;
* random SU(3) links U = exp(i*eps*H), H = sum_a h_a lambda_a / 2 with
  h_a ~ N(0,1) (Gell-Mann lambda_a), re-projected onto SU(3);
* stout smearing of the links (paper Sec. 2.2, "Link smearing", eq. of the
  stout projection): C_mu = rho * sum of the six staples,
  U' = exp([C U^dagger]_AT) U, all links updated simultaneously;
* Gaussian 4D / 5D sources and spin-colour point sources;
* operator coefficients: Zolotarev's optimal rational sign function and the
  s-dependent weights omega_s (b_s = c_s, Chiu's optimal domain-wall choice of
  Sec. 2.2) that realise it.

Array layouts (lex = x + Lx*(y + Ly*(z + Lz*t))):
  links   complex128 (V, 4, 3, 3)   U[lex, mu, row, col], mu = x, y, z, t
  4D      complex128 (V, 4, 3)      [lex, spin, colour]
  5D      complex128 (Ls, V, 4, 3)  [s, lex, spin, colour]
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform01", "gaussian", "random_su3_links", "stout_smear", "plaquette",
    "gaussian_source_4d", "gaussian_source_5d", "point_source_4d",
    "unit_links", "make_links", "lattice_volume", "zolotarev_sign", "zolotarev_omega",
]

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on a uint64 array."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def _key(seed: int, stream: int) -> np.uint64:
    k = np.array([(int(seed) * 0x2545F4914F6CDD1D + int(stream) * 0x632BE59BD9B4E019)
                  & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return _mix64(k)[0]


def _raw(seed: int, stream: int, n: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        ctr = np.arange(1, n + 1, dtype=np.uint64)
        return _mix64(_key(seed, stream) + ctr * _GOLD)


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """n doubles in (0, 1]: the top 53 bits of each counter hash."""
    r = _raw(seed, stream, n)
    return ((r >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def gaussian(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normal doubles by Box-Muller over pairs of uniforms."""
    m = (n + 1) // 2
    u = uniform01(seed, stream, 2 * m)
    r = np.sqrt(-2.0 * np.log(u[0::2]))
    th = 2.0 * np.pi * u[1::2]
    out = np.empty(2 * m)
    out[0::2] = r * np.cos(th)
    out[1::2] = r * np.sin(th)
    return out[:n]


def lattice_volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return lam


def _expi_hermitian(h: np.ndarray, scale: float) -> np.ndarray:
    """exp(i*scale*h) for a batch of Hermitian 3x3 matrices (eigendecomposition)."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * scale * w)
    return np.einsum("nij,nj,nkj->nik", v, ph, v.conj(), optimize=True)


def project_su3(u: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 1-2, row3 = conj(row1 x row2): exact SU(3)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def unit_links(dims) -> np.ndarray:
    V = lattice_volume(dims)
    u = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    u[:, :, 0, 0] = u[:, :, 1, 1] = u[:, :, 2, 2] = 1.0
    return u


def random_su3_links(dims, eps: float, seed: int) -> np.ndarray:
    """U = exp(i*eps*H) per link, H = sum_a h_a lambda_a/2, h_a ~ N(0,1).

    Draw order: canonical link order (lex, mu), eight coefficients per link.
    """
    V = lattice_volume(dims)
    n = V * 4
    h = gaussian(seed, 1, 8 * n).reshape(n, 8)
    H = np.einsum("na,aij->nij", h, _gell_mann() * 0.5, optimize=True)
    H = 0.5 * (H + np.conj(np.swapaxes(H, -1, -2)))
    U = project_su3(_expi_hermitian(H, eps))
    return U.reshape(V, 4, 3, 3)


def _shift(field: np.ndarray, dims, mu: int, step: int) -> np.ndarray:
    """f(x + step*mu_hat) as an array over x (periodic), field indexed by lex."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    f = field.reshape((Lt, Lz, Ly, Lx) + field.shape[1:])
    axis = 3 - mu
    return np.roll(f, -step, axis=axis).reshape(field.shape)


def _dag(a: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(a, -1, -2))


def _staple_sum(U: np.ndarray, dims, mu: int) -> np.ndarray:
    """sum_{nu != mu} [U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
                       + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)]."""
    C = np.zeros_like(U[:, mu])
    Umu = U[:, mu]
    for nu in range(4):
        if nu == mu:
            continue
        Unu = U[:, nu]
        up = Unu @ _shift(Umu, dims, nu, 1) @ _dag(_shift(Unu, dims, mu, 1))
        Unu_m = _shift(Unu, dims, nu, -1)
        Umu_m = _shift(Umu, dims, nu, -1)
        Unu_mp = _shift(_shift(Unu, dims, nu, -1), dims, mu, 1)
        dn = _dag(Unu_m) @ Umu_m @ Unu_mp
        C += up + dn
    return C


def stout_smear(U: np.ndarray, dims, rho: float, nsteps: int) -> np.ndarray:
    """nsteps of stout smearing, every link updated from the previous step."""
    U = U.copy()
    eye = np.eye(3)
    for _ in range(nsteps):
        new = np.empty_like(U)
        for mu in range(4):
            C = rho * _staple_sum(U, dims, mu)
            Om = C @ _dag(U[:, mu])
            A = Om - _dag(Om)
            X = 0.5 * A - (np.trace(A, axis1=-2, axis2=-1)[:, None, None] / 6.0) * eye
            # X is anti-Hermitian traceless: exp(X) = exp(i * (-i X)), -iX Hermitian.
            E = _expi_hermitian(-1j * X, 1.0)
            new[:, mu] = project_su3(E @ U[:, mu])
        U = new
    return U


def plaquette(U: np.ndarray, dims) -> float:
    """Average Re tr(U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag) / 3."""
    tot = 0.0
    cnt = 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = (U[:, mu] @ _shift(U[:, nu], dims, mu, 1)
                 @ _dag(_shift(U[:, mu], dims, nu, 1)) @ _dag(U[:, nu]))
            tot += np.trace(P, axis1=-2, axis2=-1).real.sum() / 3.0
            cnt += U.shape[0]
    return tot / cnt


def make_links(dims, eps: float, seed: int, rho: float = 0.0, nsmear: int = 0) -> np.ndarray:
    U = random_su3_links(dims, eps, seed)
    if nsmear > 0:
        U = stout_smear(U, dims, rho, nsmear)
    return U


def gaussian_source_4d(dims, seed: int) -> np.ndarray:
    V = lattice_volume(dims)
    g = gaussian(seed, 2, 2 * V * 12)
    return (g[0::2] + 1j * g[1::2]).reshape(V, 4, 3)


def gaussian_source_5d(dims, Ls: int, seed: int) -> np.ndarray:
    V = lattice_volume(dims)
    g = gaussian(seed, 3, 2 * Ls * V * 12)
    return (g[0::2] + 1j * g[1::2]).reshape(Ls, V, 4, 3)


def point_source_4d(dims, spin: int, colour: int, site: int = 0) -> np.ndarray:
    V = lattice_volume(dims)
    b = np.zeros((V, 4, 3), dtype=np.complex128)
    b[site, spin, colour] = 1.0
    return b


# ---------------------------------------------------------------------------
# Operator coefficients (inputs of the operator, no solver arithmetic).
# ---------------------------------------------------------------------------

def _zolotarev_coeffs(Ls: int, k: float):
    from scipy.special import ellipj, ellipk
    kp2 = 1.0 - k * k
    Kp = ellipk(kp2)
    ls = np.arange(1, Ls)
    sn, cn, _, _ = ellipj(ls * Kp / Ls, kp2)
    c = k * k * sn ** 2 / cn ** 2

    def shape(x):
        x = np.asarray(x, dtype=np.float64)
        r = x.copy()
        for l, cl in zip(ls, c):
            r = r * (x * x + cl) if l % 2 == 0 else r / (x * x + cl)
        return r

    g = shape(np.geomspace(k, 1.0, 200001))
    d = 2.0 / (g.max() + g.min())
    delta = (g.max() - g.min()) / (g.max() + g.min())
    return (lambda x: d * shape(x)), delta


def zolotarev_sign(y, Ls: int, k: float):
    """Zolotarev's best uniform rational approximation of sign on [k, 1]
    (odd, numerator degree Ls or Ls - 1 by parity, denominator Ls - 1 or Ls):
        R(y) = d * y * prod_{l even} (y^2 + c_l) / prod_{l odd} (y^2 + c_l),
        c_l = k^2 sn^2(l K'/Ls; k') / cn^2(l K'/Ls; k'),  l = 1 .. Ls-1,
    with k' = sqrt(1 - k^2), K' the complete elliptic integral of modulus k'
    (Jacobi elliptic functions), and d fixed so that 1 - R equioscillates
    between +delta and -delta on [k, 1].  Returns (R(y), delta)."""
    R, delta = _zolotarev_coeffs(Ls, k)
    return R(y), delta


def zolotarev_omega(Ls: int, lmin: float, lmax: float) -> np.ndarray:
    """Chiu's optimal domain-wall weights: b_s = c_s = omega_s such that
    (prod(1 + w x) - prod(1 - w x)) / (prod(1 + w x) + prod(1 - w x)) is
    Zolotarev's approximation of sign(x) on lmin <= |x| <= lmax.  Both sides
    have (1 + R) / (1 - R) = prod (1 + w_s x) / (1 - w_s x), so 1 / omega_s
    are the Ls points of [lmin, lmax] where the approximation equals 1
    (found by bracketing on a grid and bisection).  Sorted descending."""
    k = lmin / lmax
    R, _ = _zolotarev_coeffs(Ls, k)
    y = np.geomspace(k, 1.0, 400001)
    f = R(y) - 1.0
    idx = np.nonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)[0]
    roots = []
    for i in idx:
        a, b = y[i], y[i + 1]
        fa = f[i]
        for _ in range(80):
            mid = 0.5 * (a + b)
            fm = float(R(np.array([mid]))[0]) - 1.0
            if np.sign(fm) == np.sign(fa):
                a, fa = mid, fm
            else:
                b = mid
        roots.append(0.5 * (a + b))
    if len(roots) != Ls:
        raise ValueError(f"expected {Ls} crossings of 1, found {len(roots)}")
    return np.sort(1.0 / (lmax * np.array(roots)))[::-1].copy()
