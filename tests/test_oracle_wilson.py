"""Oracle pins for the Wilson kernel D_W(-M0) (Sec. 2.1, eq. Wilson_matrix).

* unit links: plane waves are eigen-directions with the momentum-space
  closed form D_W(p) = -M0 + sum(1 - cos p) + i sum gamma sin p;
* gamma_5-Hermiticity D_W^dag = gamma_5 D_W gamma_5;
* the oracle's adjoint is the adjoint: <phi, D psi> = <D^dag phi, psi>;
* gauge covariance D[U^g] g psi = g D[U] psi.
"""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import freefield as ff


def _p(dims, apbc=1, M0=1.6):
    return oracle.Params(dims=dims, Ls=2, M0=M0, m=0.1, antiperiodic_t=apbc)


@pytest.mark.parametrize("apbc", [0, 1])
def test_free_field_plane_waves(apbc):
    dims = (4, 2, 6, 4)
    p = _p(dims, apbc)
    U = dwfgen.unit_links(dims)
    moms = ff.momenta(dims, antiperiodic_t=bool(apbc))
    u = dwfgen.gaussian_source_4d((1, 1, 1, 1), 5).reshape(4, 3)
    for k in (0, 3, 17, 40, len(moms) - 1):
        psi = ff.plane_wave_4d(dims, moms[k], u)
        got = oracle.wilson(p, U, psi)
        want = ff.plane_wave_4d(dims, moms[k], ff.dw_of_p(moms[k], p.M0) @ u)
        assert np.abs(got - want).max() < 1e-13


def _inner(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def test_gamma5_hermiticity_and_adjoint():
    dims = (4, 4, 2, 4)
    p = _p(dims)
    U = dwfgen.random_su3_links(dims, 0.5, 3)
    g5 = np.diag(oracle.gamma(4)).real
    psi = dwfgen.gaussian_source_4d(dims, 1)
    phi = dwfgen.gaussian_source_4d(dims, 2)
    Dpsi = oracle.wilson(p, U, psi)
    Ddphi = oracle.wilson(p, U, phi, dagger=True)
    assert abs(_inner(phi, Dpsi) - _inner(Ddphi, psi)) < 1e-12 * abs(_inner(phi, Dpsi))
    g5D = g5[None, :, None] * oracle.wilson(p, U, g5[None, :, None] * phi)
    assert np.abs(g5D - Ddphi).max() < 1e-13


def test_gauge_covariance():
    dims = (4, 2, 4, 4)
    p = _p(dims)
    U = dwfgen.random_su3_links(dims, 0.7, 8)
    g = dwfgen.random_su3_links(dims, 1.0, 9)[:, 0]       # one SU(3) matrix per site
    V = U.shape[0]
    nbr = oracle.neighbors(dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[nbr[:, 2 * mu]], -1, -2))
    psi = dwfgen.gaussian_source_4d(dims, 4)
    gpsi = np.einsum("xab,xsb->xsa", g, psi)
    lhs = oracle.wilson(p, Ug, gpsi)
    rhs = np.einsum("xab,xsb->xsa", g, oracle.wilson(p, U, psi))
    assert np.abs(lhs - rhs).max() < 1e-13


def test_parity_mask_restricts_outputs():
    dims = (4, 4, 2, 2)
    p = _p(dims)
    U = dwfgen.random_su3_links(dims, 0.5, 3)
    psi = dwfgen.gaussian_source_4d(dims, 1)
    full = oracle.wilson(p, U, psi)
    par, _, _, _ = oracle.site_maps(dims)
    for mask, keep in ((1, 0), (2, 1)):
        part = oracle.wilson(p, U, psi, parity_mask=mask)
        assert np.array_equal(part[par == keep], full[par == keep])
        assert np.all(part[par != keep] == 0)
