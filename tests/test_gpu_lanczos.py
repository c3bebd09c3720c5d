"""Extreme eigenvalues of the normal operator D^dag D^ on the GPU (thick-restart
Lanczos in FP64, Sec. 3.2.1) against two independent references:

* unit links: the spectrum is the union over lattice momenta of the squared
  singular values of the (4 Ls) x (4 Ls) momentum-space Schur matrix, so the
  extremes have a closed form at any lattice size;
* random SU(3) links on a tiny lattice: the dense matrix of the oracle's D^,
  built column by column, and numpy's Hermitian eigensolver.
"""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import freefield as ff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_lanczos_free_field(alpha):
    import paper_2602_14454_amd as dwf
    dims, Ls, M0, m, b, c = (8, 4, 4, 8), 8, 1.6, 0.05, 1.0, 0.0
    lat = dwf.Lattice(dims)
    lat.set_gauge(dwfgen.unit_links(dims))
    op = dwf.Op(lat, Ls, M0, m, b, c, alpha)
    lo, hi, mv, conv = op.lanczos_extremes(basis=48, keep=16, max_restarts=60, tol=1e-10)
    wlo, whi = ff.normal_spectrum_extremes(dims, Ls, M0, m, b, c, alpha)
    assert conv and mv > 0
    assert abs(lo - wlo) < 1e-8 * wlo
    assert abs(hi - whi) < 1e-8 * whi


@pytest.mark.parametrize("case", [((4, 2, 2, 2), 4, 1.6, 0.05, 1.0, 0.0, 0.5),
                                  ((2, 2, 2, 4), 6, 1.8, 0.02, 1.5, 0.5, 1.0)])
def test_lanczos_dense_oracle(case):
    import paper_2602_14454_amd as dwf
    dims, Ls, M0, m, b, c, al = case
    U = dwfgen.random_su3_links(dims, 0.6, 11)
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=b, c=c, alpha=al)
    n = Ls * p.Vh * 12
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((Ls, p.Vh, 4, 3), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        A[:, j] = oracle.dhat(p, U, e).reshape(-1)
        e.reshape(-1)[j] = 0.0
    ev = np.linalg.eigvalsh(A.conj().T @ A)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, M0, m, b, c, al)
    lo, hi, mv, conv = op.lanczos_extremes(basis=64, keep=20, max_restarts=80, tol=1e-11)
    assert conv
    assert abs(lo - ev[0]) < 1e-9 * ev[0]
    assert abs(hi - ev[-1]) < 1e-9 * ev[-1]


def test_lanczos_bad_arguments():
    import paper_2602_14454_amd as dwf
    dims = (2, 2, 2, 2)
    lat = dwf.Lattice(dims)
    lat.set_gauge(dwfgen.unit_links(dims))
    op = dwf.Op(lat, 4, 1.6, 0.05, 1.0, 0.0, 1.0)
    with pytest.raises(dwf.DwfError):
        op.lanczos_extremes(basis=8, keep=7)
