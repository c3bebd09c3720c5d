"""Oracle pins for the 5D operator, the Neff form and the solve.

Pins (none re-types the oracle's block formula):
* adjointness <phi, D psi> = <D^dag phi, psi>;
* the paper's identity D^(alpha) P = D P A (Sec. 2.3, eq. relation_to_alpha=1);
* gamma_5 R_5 Hermiticity of the Shamir operator (b, c) = (1, 0);
* the 4D solution equals the closed form (1-m) G + 1 = D_eff^-1 with
  D_eff = (1+m)/2 + (1-m)/2 gamma_5 eps_Ls(H) of the Moebius literature
  (free field per momentum, and dense on tiny lattices with random links);
* the 4D solution does not depend on alpha (Sec. 2.3);
* dense LU (numpy.linalg.solve) on tiny lattices;
* the even-odd Schur complement and reconstruction agree with the dense
  block restriction (Sec. 2.3, eq. even-odd_linear_equation).
"""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import freefield as ff

PARAM_SETS = [(1.0, 0.0, 1.0), (1.0, 0.0, 0.5), (1.5, 0.5, 0.6), (1.0, 1.0, 0.4)]


def _inner(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def _setup(dims=(4, 2, 2, 4), Ls=4, b=1.0, c=0.0, alpha=1.0, m=0.05, M0=1.6, eps=0.5, seed=7):
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=b, c=c, alpha=alpha)
    U = dwfgen.random_su3_links(dims, eps, seed)
    return p, U


def _dense(fn, n):
    cols = []
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1
        cols.append(fn(e).reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("b,c,alpha", PARAM_SETS)
def test_adjointness(b, c, alpha):
    p, U = _setup(b=b, c=c, alpha=alpha)
    psi = dwfgen.gaussian_source_5d(p.dims, p.Ls, 1)
    phi = dwfgen.gaussian_source_5d(p.dims, p.Ls, 2)
    lhs = _inner(phi, oracle.dwf_apply(p, U, psi))
    rhs = _inner(oracle.dwf_apply(p, U, phi, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _Pcal(v, Ls, adjoint=False):
    """(P v)_s = P_- v_s + P_+ v_{s+1 mod Ls} (the paper's cyclic projector matrix)."""
    pp = np.array([1, 1, 0, 0.])[None, None, :, None]
    pm = 1 - pp
    if not adjoint:
        return pm * v + pp * np.roll(v, -1, axis=0)
    return pm * v + pp * np.roll(v, 1, axis=0)


@pytest.mark.parametrize("b,c,alpha", PARAM_SETS)
def test_neff_relation(b, c, alpha):
    """D^(alpha) P = D^(1) P A with A = diag(1, alpha, ..., alpha)."""
    p, U = _setup(b=b, c=c, alpha=alpha)
    p1 = p.replace(alpha=1.0)
    v = dwfgen.gaussian_source_5d(p.dims, p.Ls, 3)
    A = np.array([1.0] + [alpha] * (p.Ls - 1))[:, None, None, None]
    lhs = oracle.dwf_apply(p, U, _Pcal(v, p.Ls))
    rhs = oracle.dwf_apply(p1, U, _Pcal(A * v, p.Ls))
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(lhs).max()
    # P^dag P = 1
    assert np.allclose(_Pcal(_Pcal(v, p.Ls), p.Ls, adjoint=True), v)


def test_gamma5_r5_hermiticity_shamir():
    p, U = _setup(b=1.0, c=0.0, alpha=1.0)
    g5 = np.diag(oracle.gamma(4)).real[None, None, :, None]
    psi = dwfgen.gaussian_source_5d(p.dims, p.Ls, 4)
    lhs = g5 * oracle.dwf_apply(p, U, (g5 * psi)[::-1].copy())[::-1]
    rhs = oracle.dwf_apply(p, U, psi, dagger=True)
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("b,c,alpha", PARAM_SETS)
@pytest.mark.parametrize("Ls", [4, 7])
def test_free_field_4d_solution_closed_form(b, c, alpha, Ls):
    dims = (4, 4, 2, 4)
    m, M0 = 0.03, 1.6
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=b, c=c, alpha=alpha)
    U = dwfgen.unit_links(dims)
    moms = ff.momenta(dims)
    u = dwfgen.gaussian_source_4d((1, 1, 1, 1), 11).reshape(4, 3)
    for k in (0, 9, 50):
        b4 = ff.plane_wave_4d(dims, moms[k], u)
        x5, it, tr = oracle.solve(p, U, oracle.source_4d(p, U, b4), tol=1e-12)
        assert it > 0 and tr < 1e-12
        x4 = oracle.project_4d(p, x5)
        G = ff.g_from_dw(ff.dw_of_p(moms[k], M0), Ls, m, b, c)
        want = ff.plane_wave_4d(dims, moms[k], G @ u)
        assert np.abs(x4 - want).max() < 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("b,c", [(1.0, 0.0), (1.5, 0.5), (1.0, 1.0)])
def test_interacting_4d_solution_closed_form_dense(b, c):
    """Random SU(3) links on 2x2x2x4: G from the dense D_W closed form."""
    dims = (2, 2, 2, 4)
    p, U = _setup(dims=dims, Ls=5, b=b, c=c, alpha=0.6, m=0.04)
    n4 = p.V * 12
    # dense D_W from the (already pinned) Wilson operator, spin-major blocks per site
    Dw = _dense(lambda e: oracle.wilson(p, U, e.reshape(p.V, 4, 3)), n4)
    # reorder to (site, colour, spin) so that gamma_5 acts as kron(1, g5) on blocks of 4
    perm = np.array([(x * 4 + s) * 3 + a for x in range(p.V) for a in range(3) for s in range(4)])
    Dw_b = Dw[np.ix_(perm, perm)]
    G = ff.g_from_dw(Dw_b, p.Ls, p.m, b, c)
    b4 = dwfgen.gaussian_source_4d(dims, 12)
    x5, it, tr = oracle.solve(p, U, oracle.source_4d(p, U, b4), tol=1e-13)
    x4 = oracle.project_4d(p, x5)
    want = np.empty(n4, np.complex128)
    want[perm] = G @ b4.reshape(-1)[perm]
    assert np.abs(x4.reshape(-1) - want).max() < 1e-10 * np.abs(want).max()
    assert oracle.residual_4d(p, U, x4, b4) < 1e-11


@pytest.mark.parametrize("b,c", [(1.0, 0.0), (1.5, 0.5)])
def test_4d_solution_alpha_invariance(b, c):
    dims = (4, 2, 2, 4)
    p, U = _setup(dims=dims, Ls=6, b=b, c=c, m=0.02)
    b4 = dwfgen.gaussian_source_4d(dims, 21)
    b5 = oracle.source_4d(p, U, b4)
    x4s, x5s = [], []
    for al in (1.0, 0.7, 0.4):
        pa = p.replace(alpha=al)
        x5, it, tr = oracle.solve(pa, U, b5, tol=1e-13)
        assert tr < 1e-13
        x4s.append(oracle.project_4d(pa, x5))
        x5s.append(x5)
    for k in (1, 2):
        assert np.abs(x4s[k] - x4s[0]).max() < 1e-11 * np.abs(x4s[0]).max()
    # x5 itself changes: x5^(alpha) = T^-1 x5, T = diag_s(P_- + a P_+, a, .., a, P_+ + a P_-)
    al = 0.4
    Tinv = np.full((p.Ls, 4), 1.0 / al)
    Tinv[0, 2:] = 1.0
    Tinv[-1, :2] = 1.0
    assert np.abs(x5s[2] - Tinv[:, None, :, None] * x5s[0]).max() < 1e-10 * np.abs(x5s[0]).max()


def test_dense_lu_solve_tiny():
    dims = (2, 2, 2, 2)
    p, U = _setup(dims=dims, Ls=4, b=1.5, c=0.5, alpha=0.5, m=0.1)
    n = p.Ls * p.V * 12
    D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(p.Ls, p.V, 4, 3)), n)
    b5 = dwfgen.gaussian_source_5d(dims, p.Ls, 5)
    x_lu = np.linalg.solve(D, b5.reshape(-1))
    x5, it, tr = oracle.solve(p, U, b5, tol=1e-13)
    assert np.abs(x5.reshape(-1) - x_lu).max() < 1e-11 * np.abs(x_lu).max()
    # adjoint of the dense matrix is the dense matrix of the adjoint
    Dd = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(p.Ls, p.V, 4, 3), dagger=True), n)
    assert np.abs(Dd - D.conj().T).max() < 1e-13


def test_schur_pieces_against_dense_blocks():
    dims = (2, 2, 2, 4)
    p, U = _setup(dims=dims, Ls=3, b=1.0, c=1.0, alpha=0.7, m=0.08)
    n = p.Ls * p.V * 12
    D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(p.Ls, p.V, 4, 3)), n)
    par, _, le, lo = oracle.site_maps(dims)
    idx = np.arange(n).reshape(p.Ls, p.V, 12)
    ie = idx[:, le].reshape(-1)
    io = idx[:, lo].reshape(-1)
    Dee, Deo = D[np.ix_(ie, ie)], D[np.ix_(ie, io)]
    Doe, Doo = D[np.ix_(io, ie)], D[np.ix_(io, io)]
    # D_ee is site-local and equal to D_oo
    assert np.abs(Dee - Doo).max() < 1e-14
    Dhat = np.eye(len(ie)) - np.linalg.solve(Dee, Deo @ np.linalg.solve(Doo, Doe))
    xe = dwfgen.gaussian_source_5d(dims, p.Ls, 9)[:, : p.Vh].copy()
    got = oracle.dhat(p, U, xe).reshape(-1)
    assert np.abs(got - Dhat @ xe.reshape(-1)).max() < 1e-12
    gotd = oracle.dhat(p, U, xe, dagger=True).reshape(-1)
    assert np.abs(gotd - Dhat.conj().T @ xe.reshape(-1)).max() < 1e-12
    # Schur RHS + reconstruction of the exact even solution solves the full system
    b5 = dwfgen.gaussian_source_5d(dims, p.Ls, 10)
    bt = oracle.schur_rhs(p, U, b5).reshape(-1)
    xe_exact = np.linalg.solve(Dhat, bt)
    x5 = oracle.reconstruct(p, U, xe_exact.reshape(p.Ls, p.Vh, 4, 3), b5)
    assert np.abs(D @ x5.reshape(-1) - b5.reshape(-1)).max() < 1e-12 * np.abs(b5).max()


def test_left_schur_similarity_and_right_schur_alpha_independence():
    """Left Schur operators of different alpha share eigenvalues; the
    right-preconditioned form (Sec. 2.3, eq. another_even-odd_linear_equation)
    is alpha independent."""
    dims = (2, 2, 2, 2)
    res = {}
    for al in (1.0, 0.5):
        p, U = _setup(dims=dims, Ls=4, b=1.5, c=0.5, alpha=al, m=0.05)
        n = p.Ls * p.V * 12
        D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(p.Ls, p.V, 4, 3)), n)
        par, _, le, lo = oracle.site_maps(dims)
        idx = np.arange(n).reshape(p.Ls, p.V, 12)
        ie, io = idx[:, le].reshape(-1), idx[:, lo].reshape(-1)
        Dee, Deo, Doe, Doo = (D[np.ix_(a, b)] for a, b in ((ie, ie), (ie, io), (io, ie), (io, io)))
        left = np.eye(len(ie)) - np.linalg.solve(Dee, Deo @ np.linalg.solve(Doo, Doe))
        right = np.eye(len(ie)) - Deo @ np.linalg.solve(Doo, Doe @ np.linalg.inv(Dee))
        res[al] = (np.linalg.eigvals(left), right, np.linalg.svd(left, compute_uv=False))
    ea, eb = res[1.0][0], res[0.5][0]
    dist = np.abs(ea[:, None] - eb[None, :])
    assert dist.min(axis=1).max() < 1e-9 and dist.min(axis=0).max() < 1e-9
    assert np.abs(res[1.0][1] - res[0.5][1]).max() < 1e-12
    # ... while the singular values (what CGNR sees) do change with alpha
    assert np.abs(res[1.0][2] - res[0.5][2]).max() > 1e-3


def test_freefield_dhat_of_p_matches_oracle():
    dims = (4, 2, 2, 4)
    Ls, M0, m, b, c, al = 4, 1.6, 0.05, 1.5, 0.5, 0.6
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=b, c=c, alpha=al)
    U = dwfgen.unit_links(dims)
    par, _, le, _ = oracle.site_maps(dims)
    u = dwfgen.gaussian_source_5d((1, 1, 1, 1), Ls, 3).reshape(Ls, 4, 3)
    for mom in ff.momenta(dims)[::7]:
        pw = np.stack([ff.plane_wave_4d(dims, mom, u[s]) for s in range(Ls)])
        xe = np.ascontiguousarray(pw[:, le])
        got = oracle.dhat(p, U, xe)
        Dp = ff.dhat_of_p(mom, Ls, M0, m, b, c, al)
        want_u = np.einsum("ij,jc->ic", Dp, u.reshape(Ls * 4, 3)).reshape(Ls, 4, 3)
        want = np.stack([ff.plane_wave_4d(dims, mom, want_u[s]) for s in range(Ls)])[:, le]
        assert np.abs(got - want).max() < 1e-12
