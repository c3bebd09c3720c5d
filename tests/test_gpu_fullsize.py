"""Parity at the benchmark's full size and launch configuration
(16^3x32, Ls = 16, M0 = 1.6, m = 0.01, Neff alpha = 0.5, smeared links, 4D
Gaussian source; defect correction with BF16 inner CG, as bench.py times it):
the FP64 oracle recomputes the true 5D residual of the GPU solution with its
own operator, and the 4D residual of x4 is checked.  Also: every solver path
is deterministic (repeating a solve reproduces the bits)."""
import numpy as np
import pytest

import dwfgen
import oracle

pytestmark = pytest.mark.gpu

C2 = dict(dims=(16, 16, 16, 32), Ls=16, M0=1.6, m=0.01, b=1.0, c=0.0, alpha=0.5)


@pytest.fixture(scope="module")
def c2():
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = C2["dims"], C2["Ls"]
    U = dwfgen.make_links(dims, 0.5, 11, rho=0.1, nsmear=3)
    b4h = dwfgen.gaussian_source_4d(dims, 12)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, C2["M0"], C2["m"], C2["b"], C2["c"], C2["alpha"])
    V = int(np.prod(dims))
    b4 = torch.from_numpy(b4h).to("cuda")
    b5 = torch.empty((Ls, V, 4, 3), dtype=torch.complex128, device="cuda")
    op.source_4d(b5, b4)
    return U, lat, op, b4, b5


def test_bench_configuration_against_oracle(c2):
    import torch
    import paper_2602_14454_amd as dwf
    U, lat, op, b4, b5 = c2
    prm = dwf.default_params(tol=1e-10, check_every=8, algo=dwf.ALGO_DC, inner_prec=dwf.BF16)
    x5 = torch.zeros_like(b5)
    st, info = op.solve(x5, b5, prm)
    assert st == 0 and info.converged and info.true_res5 <= 1e-10
    p = oracle.Params(dims=C2["dims"], Ls=C2["Ls"], M0=C2["M0"], m=C2["m"], b=C2["b"], c=C2["c"], alpha=C2["alpha"])
    r5 = oracle.true_residual(p, U, x5.cpu().numpy(), b5.cpu().numpy())
    assert r5 <= 1.2e-10 and abs(r5 - info.true_res5) <= 0.05 * r5
    x4 = torch.empty((int(np.prod(C2["dims"])), 4, 3), dtype=torch.complex128, device="cuda")
    op.project_4d(x4, x5)
    assert op.residual_4d(x4, b4) <= 1e-10


@pytest.mark.parametrize("algo,prec", [(0, 0), (1, 1), (1, 2), (3, 1)])
def test_solves_are_deterministic(c2, algo, prec):
    import torch
    import paper_2602_14454_amd as dwf
    U, lat, op, b4, b5 = c2
    prm = dwf.default_params(tol=1e-10, check_every=8, algo=algo, inner_prec=prec)
    xs = []
    for _ in range(2):
        x5 = torch.zeros_like(b5)
        st, info = op.solve(x5, b5, prm)
        assert st == 0
        xs.append((x5.cpu().numpy(), info.iters))
    assert xs[0][1] == xs[1][1]
    assert np.array_equal(xs[0][0], xs[1][0])


def test_lanczos_is_deterministic():
    import paper_2602_14454_amd as dwf
    dims = (8, 8, 8, 8)
    U = dwfgen.make_links(dims, 0.5, 3, rho=0.1, nsmear=1)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, 8, 1.6, 0.05, 1.0, 0.0, 0.5)
    a = op.lanczos_extremes(basis=32, keep=12, max_restarts=30, tol=1e-8)
    b = op.lanczos_extremes(basis=32, keep=12, max_restarts=30, tol=1e-8)
    assert a == b
