"""Input generators: random SU(3) links and stout smearing (Sec. 2.2, Link smearing)."""
import numpy as np

import dwfgen
import oracle


def test_uniform_and_gaussian_streams():
    u = dwfgen.uniform01(3, 1, 200000)
    assert u.min() > 0 and u.max() <= 1
    assert abs(u.mean() - 0.5) < 5e-3
    g = dwfgen.gaussian(3, 2, 200000)
    assert abs(g.mean()) < 1e-2 and abs(g.var() - 1) < 2e-2
    # pure function of (seed, stream, index)
    assert np.array_equal(dwfgen.gaussian(3, 2, 10), g[:10])
    assert not np.array_equal(dwfgen.gaussian(4, 2, 10), g[:10])


def _is_su3(U):
    UU = U @ np.conj(np.swapaxes(U, -1, -2))
    return np.abs(UU - np.eye(3)).max() < 1e-13 and np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_random_su3():
    U = dwfgen.random_su3_links((4, 4, 2, 2), 0.5, 1)
    assert _is_su3(U)
    U0 = dwfgen.random_su3_links((4, 4, 2, 2), 1e-8, 1)
    assert np.abs(U0 - np.eye(3)).max() < 1e-7


def test_stout_fixed_point_and_rho_zero():
    dims = (4, 2, 2, 4)
    one = dwfgen.unit_links(dims)
    assert np.abs(dwfgen.stout_smear(one, dims, 0.1, 3) - one).max() < 1e-14
    U = dwfgen.random_su3_links(dims, 0.5, 2)
    assert np.abs(dwfgen.stout_smear(U, dims, 0.0, 2) - U).max() < 1e-13


def test_stout_gauge_covariance_unitarity_and_plaquette():
    dims = (4, 4, 2, 4)
    U = dwfgen.random_su3_links(dims, 0.6, 5)
    g = dwfgen.random_su3_links(dims, 1.0, 6)[:, 0]
    nbr = oracle.neighbors(dims)
    def transform(W):
        out = np.empty_like(W)
        for mu in range(4):
            out[:, mu] = g @ W[:, mu] @ np.conj(np.swapaxes(g[nbr[:, 2 * mu]], -1, -2))
        return out
    S = dwfgen.stout_smear(U, dims, 0.1, 3)
    Sg = dwfgen.stout_smear(transform(U), dims, 0.1, 3)
    assert np.abs(Sg - transform(S)).max() < 1e-12
    assert _is_su3(S)
    p0 = dwfgen.plaquette(U, dims)
    p1 = dwfgen.plaquette(dwfgen.stout_smear(U, dims, 0.1, 1), dims)
    p3 = dwfgen.plaquette(S, dims)
    assert p0 < p1 < p3 <= 1.0
    assert abs(dwfgen.plaquette(dwfgen.unit_links(dims), dims) - 1.0) < 1e-15
