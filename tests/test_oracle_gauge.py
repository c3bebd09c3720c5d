"""Pins of the quenched gauge generator oracle (oracle/gauge.py):

* Kennedy-Pendleton's sampler against the exact density
  sqrt(1 - y0^2) exp(alpha y0) (chi-square over 40 bins, 2x10^5 draws);
* over-relaxation leaves every link's local action Re tr(U A) unchanged and
  moves the links; the total action is unchanged;
* heatbath and over-relaxation keep the links in SU(3);
* strong coupling: at beta = 1 the plaquette of the heatbath ensemble equals
  the single-plaquette expectation (Weyl integral; lattice corrections enter
  at order u^5 ~ 1e-6), whose small-beta series beta/18 + beta^2/216 pins the
  integral itself.
"""
import numpy as np
import pytest
from scipy import integrate

import dwfgen
from oracle import gauge as G


@pytest.mark.parametrize("alpha", [0.5, 3.0, 12.0])
def test_kennedy_pendleton_density(alpha):
    key = G.sweep_key(5, 1)
    N = 200000
    y0, ok = G.kp_sample(np.full(N, alpha), key, np.arange(N, dtype=np.uint64) * np.uint64(G.NDRAW))
    assert ok.all()
    bins = np.linspace(-1, 1, 41)
    h, _ = np.histogram(y0, bins)
    f = lambda x: np.sqrt(1 - x * x) * np.exp(alpha * x)
    Z = integrate.quad(f, -1, 1)[0]
    expc = np.array([integrate.quad(f, bins[i], bins[i + 1])[0] for i in range(40)]) / Z * N
    m = expc > 5
    chi2 = np.sum((h[m] - expc[m]) ** 2 / expc[m])
    dof = int(m.sum()) - 1
    assert chi2 < dof + 5 * np.sqrt(2 * dof)


def test_over_relaxation_is_microcanonical():
    dims = (4, 4, 2, 4)
    U = dwfgen.random_su3_links(dims, 0.5, 3)
    par = np.sum(G._coords(dims), axis=1) & 1
    sites = np.nonzero(par == 1)[0]
    A = G.staples(U, dims, 2, sites)
    Ul = U[sites, 2].copy()
    W = Ul @ A
    for g, (i, j) in enumerate(G.SUBGROUPS):
        Ul, W = G._update_subgroup(Ul, W, i, j, 6.0, G.sweep_key(1, 0), np.zeros(len(sites), np.uint64), False)
    before = np.trace(U[sites, 2] @ A, axis1=1, axis2=2).real
    after = np.trace(Ul @ A, axis1=1, axis2=2).real
    assert np.abs(after - before).max() < 1e-12
    assert np.abs(Ul - U[sites, 2]).max() > 0.1
    S0 = G.action(U, dims, 6.0)
    G.sweep(U, dims, 6.0, 1, 0, heatbath=False)
    assert abs(G.action(U, dims, 6.0) - S0) < 1e-10 * S0


def test_sweeps_stay_in_su3():
    dims = (4, 2, 4, 2)
    U = dwfgen.random_su3_links(dims, 1.0, 4)
    for k in range(2):
        G.sweep(U, dims, 5.7, 9, k, heatbath=True)
        G.sweep(U, dims, 5.7, 9, k, heatbath=False)
    eye = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-13


def test_single_plaquette_integral_small_beta_series():
    for b in (0.05, 0.1):
        assert abs(G.single_plaquette_expectation(b) - (b / 18 + b * b / 216)) < 2 * b ** 3 / 100


def test_strong_coupling_plaquette():
    dims, beta = (4, 4, 4, 4), 1.0
    U = dwfgen.random_su3_links(dims, 1.0, 7)
    for k in range(10):
        G.sweep(U, dims, beta, 21, k)
    ps = []
    for k in range(10, 90):
        G.sweep(U, dims, beta, 21, k)
        ps.append(G.plaquette(U, dims))
    ps = np.array(ps)
    blocks = ps.reshape(8, 10).mean(axis=1)
    err = blocks.std(ddof=1) / np.sqrt(len(blocks))
    want = G.single_plaquette_expectation(beta)
    assert abs(ps.mean() - want) < 4 * err + 1e-4, (ps.mean(), want, err)
