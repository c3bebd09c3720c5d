"""Pins of the oracle's two residual checkers, which every GPU solve-parity
test relies on.

* ``true_residual`` (|b5 - D^(alpha) x5| / |b5|): at the dense-LU solution it
  is at rounding level; at x5 = x_LU + delta with delta = D^-1 e (dense LU) it
  equals |e| / |b5| exactly, whatever the operator code does (the expected
  value never applies D).
* ``residual_4d`` (|b4 - D_eff((1-m) x4 + b4)| / |b4|, Sec. 2.3: the 4D
  solution is the same for every alpha): at x4 = G b4 + delta4, with G and
  D_eff the closed forms of the Moebius literature evaluated on the dense
  Wilson matrix, it equals (1-m) |D_eff delta4| / |b4|.
"""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import freefield as ff


def _dense(fn, n):
    cols = []
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1
        cols.append(fn(e).reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("b,c,alpha", [(1.0, 0.0, 0.5), (1.5, 0.5, 1.0)])
def test_true_residual_dense_lu(b, c, alpha):
    dims, Ls = (2, 2, 2, 2), 4
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=0.07, b=b, c=c, alpha=alpha)
    U = dwfgen.random_su3_links(dims, 0.5, 31)
    n = Ls * p.V * 12
    D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(Ls, p.V, 4, 3)), n)
    b5 = 3.0 * dwfgen.gaussian_source_5d(dims, Ls, 32)
    x_lu = np.linalg.solve(D, b5.reshape(-1))
    r0 = oracle.true_residual(p, U, x_lu.reshape(b5.shape), b5)
    assert r0 < 1e-14
    for scale in (1e-6, 1e-2, 1.0):
        e = scale * dwfgen.gaussian_source_5d(dims, Ls, 33).reshape(-1)
        delta = np.linalg.solve(D, e)      # D (x_lu + delta) = b5 + e
        want = np.linalg.norm(e) / np.linalg.norm(b5)
        got = oracle.true_residual(p, U, (x_lu + delta).reshape(b5.shape), b5)
        assert abs(got - want) <= 1e-12 * want + 1e-15


@pytest.mark.parametrize("b,c,alpha", [(1.0, 0.0, 0.6), (1.0, 1.0, 0.4)])
def test_residual_4d_closed_form(b, c, alpha):
    dims, Ls, m = (2, 2, 2, 4), 5, 0.04
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=m, b=b, c=c, alpha=alpha)
    U = dwfgen.random_su3_links(dims, 0.5, 41)
    n4 = p.V * 12
    Dw = _dense(lambda e: oracle.wilson(p, U, e.reshape(p.V, 4, 3)), n4)
    # (site, colour, spin) order: gamma_5 acts on blocks of four
    perm = np.array([(x * 4 + s) * 3 + a for x in range(p.V) for a in range(3) for s in range(4)])
    Dw_b = Dw[np.ix_(perm, perm)]
    Deff = ff.deff_from_dw(Dw_b, Ls, m, b, c)
    G = ff.g_from_dw(Dw_b, Ls, m, b, c)
    b4 = dwfgen.gaussian_source_4d(dims, 42)
    bp = b4.reshape(-1)[perm]
    x4 = np.empty(n4, np.complex128)
    x4[perm] = G @ bp
    assert oracle.residual_4d(p, U, x4.reshape(b4.shape), b4) < 1e-11
    for scale in (1e-4, 1e-1):
        d4 = scale * dwfgen.gaussian_source_4d(dims, 43).reshape(-1)
        want = (1 - m) * np.linalg.norm(Deff @ d4[perm]) / np.linalg.norm(b4)
        got = oracle.residual_4d(p, U, (x4 + d4).reshape(b4.shape), b4)
        assert abs(got - want) <= 1e-9 * want
