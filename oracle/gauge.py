"""Quenched gauge-field generator for the plaquette action -- TEST INFRASTRUCTURE.

Only tests/ may import this module; the HIP path never does and shares no
code with it.

The paper's ensembles are quenched configurations of the plaquette (Wilson)
gauge action at beta = 6.0 and 5.7 (Sec. 3.1),
    S = beta * sum_P (1 - Re tr U_P / 3),
U_P(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag; the paper does not say
how they were generated.  Reading taken: the standard local Monte Carlo,
written here from its definitions in plain numpy, FP64:

* a link U_mu(x) sees the staple sum
      A = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                       + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu),
  its action is -beta/3 Re tr(U A); the links of one direction on the sites
  of one parity do not appear in each other's staples and are updated
  together (order: mu = 0..3, parity 0 then 1);
* heatbath (Cabibbo-Marinari): U <- R U for R in the SU(2) subgroups on
  rows/columns (0,1), (0,2), (1,2) in turn, R drawn from
  exp(beta/3 Re tr(R W)), W = U A.  The 2x2 block r of W enters only through
  Re tr(X r) = k Re tr(X V^dag) (X, V in SU(2), k >= 0), so R = Y V with Y
  drawn from exp(2 beta k / 3 * y0) dY; y0 = 1 - delta with delta from the
  Gamma(3/2) density times sqrt(1 - delta/2) by rejection (Kennedy and
  Pendleton's sampler), the other three components uniform on the sphere of
  radius sqrt(1 - y0^2);
* over-relaxation: R = V^2, which leaves Re tr(R r) and hence the action
  unchanged;
* after every sweep the links are re-projected onto SU(3) (rows 0 and 1
  normalised and orthogonalised, row 2 = conj(row0 x row1)).

Random numbers: uniform doubles in (0, 1] from SplitMix64 (Steele, Lea and
Flood 2014) applied to counters: key = mix(seed * K1 + sweep * K2),
value = mix(key + (c + 1) * golden), c = ((lex * 4 + mu) * 3 + subgroup) * 4096
+ draw; attempt t of the sampler uses draws 4t .. 4t+3, the direction draws
4000 and 4001; a link whose sampler finds no acceptance in 1000 attempts keeps
that subgroup unchanged.
"""
from __future__ import annotations

import numpy as np

_GOLD = np.uint64(0x9E3779B97F4A7C15)
_K1 = 0x2545F4914F6CDD1D
_K2 = 0x632BE59BD9B4E019
NDRAW = 4096
MAX_ATTEMPTS = 1000
SUBGROUPS = ((0, 1), (0, 2), (1, 2))


def _mix(z):
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def sweep_key(seed: int, sweep: int) -> np.uint64:
    return _mix(np.array([(int(seed) * _K1 + int(sweep) * _K2) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]


def uniform(key, counters):
    """Uniform doubles in (0, 1] for integer counters (array)."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(key + (c + np.uint64(1)) * _GOLD)
    return ((z >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def _coords(dims):
    V = int(np.prod(dims))
    lex = np.arange(V)
    c = np.empty((V, 4), np.int64)
    r = lex.copy()
    for mu in range(4):
        c[:, mu] = r % dims[mu]
        r //= dims[mu]
    return c


def _lex(dims, c):
    return c[:, 0] + dims[0] * (c[:, 1] + dims[1] * (c[:, 2] + dims[2] * c[:, 3]))


def _shift(dims, c, mu, step):
    d = c.copy()
    d[:, mu] = (d[:, mu] + step) % dims[mu]
    return _lex(dims, d)


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def staples(U, dims, mu, sites):
    """Staple sum A of U_mu(x) for the given sites (array of lex)."""
    c = _coords(dims)[sites]
    A = np.zeros((len(sites), 3, 3), np.complex128)
    xpmu = _shift(dims, c, mu, +1)
    for nu in range(4):
        if nu == mu:
            continue
        xpnu = _shift(dims, c, nu, +1)
        xmnu = _shift(dims, c, nu, -1)
        cm = c.copy()
        cm[:, nu] = (cm[:, nu] - 1) % dims[nu]
        xpmu_mnu = _shift(dims, cm, mu, +1)
        A += U[xpmu, nu] @ _dag(U[xpnu, mu]) @ _dag(U[sites, nu])
        A += _dag(U[xpmu_mnu, nu]) @ _dag(U[xmnu, mu]) @ U[xmnu, nu]
    return A


def _quaternion_of_block(r):
    """c with Re tr(X r) = 2 (x0 c0 - x1 c1 - x2 c2 - x3 c3) for X in SU(2)."""
    c0 = 0.5 * (r[:, 0, 0] + r[:, 1, 1]).real
    c1 = 0.5 * (r[:, 0, 1] + r[:, 1, 0]).imag
    c2 = 0.5 * (r[:, 0, 1] - r[:, 1, 0]).real
    c3 = 0.5 * (r[:, 0, 0] - r[:, 1, 1]).imag
    return np.stack([c0, -c1, -c2, -c3], axis=1)   # parameters of V (times k)


def su2_matrix(q):
    """X = q0 + i (q1 s1 + q2 s2 + q3 s3) as 2x2 complex matrices."""
    X = np.empty((q.shape[0], 2, 2), np.complex128)
    X[:, 0, 0] = q[:, 0] + 1j * q[:, 3]
    X[:, 0, 1] = q[:, 2] + 1j * q[:, 1]
    X[:, 1, 0] = -q[:, 2] + 1j * q[:, 1]
    X[:, 1, 1] = q[:, 0] - 1j * q[:, 3]
    return X


def kp_sample(alpha, key, ctr0):
    """y0 with density ~ sqrt(1 - y0^2) exp(alpha y0) for each alpha (Kennedy-Pendleton);
    ctr0: counter base per sample.  Returns (y0, accepted)."""
    n = len(alpha)
    y0 = np.ones(n)
    done = np.zeros(n, bool)
    for t in range(MAX_ATTEMPTS):
        todo = np.nonzero(~done)[0]
        if len(todo) == 0:
            break
        base = ctr0[todo] + np.uint64(4 * t)
        r1 = uniform(key, base)
        r2 = uniform(key, base + np.uint64(1))
        r3 = uniform(key, base + np.uint64(2))
        r4 = uniform(key, base + np.uint64(3))
        delta = -(np.log(r1) + np.cos(2 * np.pi * r2) ** 2 * np.log(r3)) / alpha[todo]
        ok = r4 * r4 <= 1.0 - 0.5 * delta
        y0[todo[ok]] = 1.0 - delta[ok]
        done[todo[ok]] = True
    return y0, done


def _update_subgroup(U_l, W, i, j, beta, key, ctr0, heatbath):
    r = W[:, [i, j]][:, :, [i, j]]
    cq = _quaternion_of_block(r)
    k = np.sqrt(np.sum(cq * cq, axis=1))
    V = su2_matrix(cq / np.where(k > 0, k, 1.0)[:, None])
    if heatbath:
        alpha = 2.0 * beta * k / 3.0
        y0, ok = kp_sample(np.where(alpha > 0, alpha, 1e-300), key, ctr0)
        cth = 2.0 * uniform(key, ctr0 + np.uint64(4000)) - 1.0
        phi = 2.0 * np.pi * uniform(key, ctr0 + np.uint64(4001))
        rad = np.sqrt(np.maximum(0.0, 1.0 - y0 * y0))
        sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
        y = np.stack([y0, rad * sth * np.cos(phi), rad * sth * np.sin(phi), rad * cth], axis=1)
        R = su2_matrix(y) @ V
        R[~ok] = np.eye(2)
    else:
        R = V @ V
    for M in (U_l, W):
        rows = M[:, [i, j], :]
        M[:, [i, j], :] = R @ rows
    return U_l, W


def reunitarize(U):
    a = U[..., 0, :]
    a = a / np.linalg.norm(a, axis=-1, keepdims=True)
    b = U[..., 1, :]
    b = b - np.sum(np.conj(a) * b, axis=-1, keepdims=True) * a
    b = b / np.linalg.norm(b, axis=-1, keepdims=True)
    c = np.conj(np.cross(a, b))
    return np.stack([a, b, c], axis=-2)


def sweep(U, dims, beta, seed, sweep_index, heatbath=True):
    """One heatbath (or over-relaxation) sweep over all links, in place; U: (V, 4, 3, 3)."""
    V = int(np.prod(dims))
    c = _coords(dims)
    par = np.sum(c, axis=1) & 1
    key = sweep_key(seed, sweep_index)
    for mu in range(4):
        for p in (0, 1):
            sites = np.nonzero(par == p)[0]
            A = staples(U, dims, mu, sites)
            U_l = U[sites, mu].copy()
            W = U_l @ A
            for g, (i, j) in enumerate(SUBGROUPS):
                ctr0 = ((sites.astype(np.uint64) * np.uint64(4) + np.uint64(mu)) * np.uint64(3) + np.uint64(g)) \
                    * np.uint64(NDRAW)
                U_l, W = _update_subgroup(U_l, W, i, j, beta, key, ctr0, heatbath)
            U[sites, mu] = U_l
    U[:] = reunitarize(U)
    return U


def plaquette(U, dims):
    """Average Re tr U_P / 3 over all x and mu < nu."""
    c = _coords(dims)
    acc = 0.0
    lex = np.arange(int(np.prod(dims)))
    for mu in range(4):
        xpmu = _shift(dims, c, mu, +1)
        for nu in range(mu + 1, 4):
            xpnu = _shift(dims, c, nu, +1)
            P = U[lex, mu] @ U[xpmu, nu] @ _dag(U[xpnu, mu]) @ _dag(U[lex, nu])
            acc += np.trace(P, axis1=-2, axis2=-1).real.sum()
    return acc / (3.0 * 6 * len(lex))


def action(U, dims, beta):
    return beta * 6 * int(np.prod(dims)) * (1.0 - plaquette(U, dims))


def single_plaquette_expectation(beta, n=256):
    """<Re tr U / 3> for one SU(3) matrix with weight exp(beta/3 Re tr U) dU:
    Weyl's integration formula over the eigenphases (th1, th2, -th1-th2),
    Haar density ~ prod_{i<j} |e^{i th_i} - e^{i th_j}|^2 (periodic grid:
    spectral accuracy)."""
    th = 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(th, th, indexing="ij")
    t3 = -(t1 + t2)
    vdm = (np.abs(np.exp(1j * t1) - np.exp(1j * t2)) ** 2 * np.abs(np.exp(1j * t1) - np.exp(1j * t3)) ** 2
           * np.abs(np.exp(1j * t2) - np.exp(1j * t3)) ** 2)
    re = (np.cos(t1) + np.cos(t2) + np.cos(t3)) / 3.0
    w = vdm * np.exp(beta * re)
    return float(np.sum(w * re) / np.sum(w))
