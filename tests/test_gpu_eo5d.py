"""The split by 5D parity on the GPU (Sec. 2.3: even and odd sites in five
instead of four dimensions), checked by the FP64 CPU oracle.

* D^5 and its adjoint element by element against oracle.eo5.dhat5 (the
  oracle's 5D operator restricted to the 5D-parity subspaces), FP64 to
  1e-13 and FP32 to 1e-5 relative, over Ls = 2, 4, 8, 16, alpha = 1 and 0.5,
  b = 1, 1.5 and s-dependent b_s, on lattices whose Ls * V / 2 sites leave a
  ragged last block;
* solves with schur = 2 (FP64 CGNR, DC with FP32 inner CG, FP32 paper mode)
  reach the oracle's true 5D residual and the 4D-split solution;
* c != 0, odd Ls and BF16 are rejected.
"""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import eo5

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(dims, Ls, M0, m, b=1.0, alpha=1.0, seed=41, nsmear=0):
    import paper_2602_14454_amd as dwf
    U = dwfgen.make_links(dims, 0.5, seed, rho=0.1, nsmear=nsmear)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    bs = tuple(b) if isinstance(b, (list, tuple)) else None
    op = dwf.Op(lat, Ls, M0, m, list(b) if bs else b, [0.0] * Ls if bs else 0.0, alpha)
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=1.0 if bs else b, c=0.0, alpha=alpha, bs=bs)
    return lat, op, p, U


CASES = [
    ((4, 4, 2, 6), 4, 1.0, 1.0),
    ((4, 4, 2, 6), 8, 1.5, 0.5),
    ((4, 2, 2, 4), 2, 1.0, 0.5),
    ((6, 4, 4, 4), 16, 1.0, 0.5),
    ((4, 4, 2, 6), 6, (1.2, 0.9, 1.1, 1.0, 0.8, 1.3), 0.7),
]


@pytest.mark.parametrize("dims,Ls,b,alpha", CASES)
def test_dhat5_matches_oracle(dims, Ls, b, alpha):
    import torch
    import paper_2602_14454_amd as dwf
    lat, op, p, U = _setup(dims, Ls, 1.8, 0.02, b, alpha)
    print(f"[eo5d] dims {dims} Ls {Ls} b {b} alpha {alpha}", flush=True)
    x = dwfgen.gaussian_source_5d(dims, Ls, 42)
    xd = _dev(x)
    e = np.repeat(eo5.even_mask(p)[:, :, None, None], 4, 2).repeat(3, 3)
    for dag in (False, True):
        ref = eo5.dhat5(p, U, x, dagger=dag)
        for prec, tol in ((dwf.F64, 1e-13), (dwf.F32, 1e-5)):
            out = torch.empty_like(xd)
            op.apply_eo5(out, xd, dagger=dag, prec=prec)
            y = out.cpu().numpy()
            assert np.abs(y[~e]).max() == 0.0
            err = np.abs(y - ref).max() / np.abs(ref).max()
            assert err < tol, (dag, prec, err)


def test_dhat5_adjoint_pairing():
    """<y, D^5 x> = <D^5^dag y, x> on the GPU in FP64 (both sides the library's)."""
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 4), 8
    lat, op, p, U = _setup(dims, Ls, 1.6, 0.05, 1.0, 0.6)
    e = torch.from_numpy(np.repeat(eo5.even_mask(p)[:, :, None, None], 4, 2).repeat(3, 3)).cuda()
    x = _dev(dwfgen.gaussian_source_5d(dims, Ls, 43)) * e
    y = _dev(dwfgen.gaussian_source_5d(dims, Ls, 44)) * e
    dx, dy = torch.empty_like(x), torch.empty_like(y)
    op.apply_eo5(dx, x)
    op.apply_eo5(dy, y, dagger=True)
    lhs = torch.vdot(y.flatten(), dx.flatten()).item()
    rhs = torch.vdot(dy.flatten(), x.flatten()).item()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("b,alpha", [(1.0, 1.0), (1.0, 0.5), (1.5, 0.6)])
def test_solve_5d_split_matches_oracle_and_4d_split(b, alpha):
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 6), 8
    lat, op, p, U = _setup(dims, Ls, 1.8, 0.02, b, alpha, nsmear=1)
    b5 = dwfgen.gaussian_source_5d(dims, Ls, 45)
    bd = _dev(b5)
    print(f"[eo5d] solve b {b} alpha {alpha}", flush=True)
    x4d = torch.zeros_like(bd)
    st, i4 = op.solve(x4d, bd, dwf.default_params(tol=1e-11, check_every=1))
    assert st == 0
    for prm in (dwf.default_params(tol=1e-11, check_every=1, schur=2),
                dwf.default_params(tol=1e-11, check_every=4, schur=2, algo=dwf.ALGO_DC, inner_prec=dwf.F32)):
        x5 = torch.zeros_like(bd)
        st, info = op.solve(x5, bd, prm)
        assert st == 0 and info.converged
        xg = x5.cpu().numpy()
        assert oracle.true_residual(p, U, xg, b5) <= 1e-11
        assert abs(info.true_res5 - oracle.true_residual(p, U, xg, b5)) < 1e-13
        ref = x4d.cpu().numpy()
        assert np.abs(xg - ref).max() / np.abs(ref).max() < 1e-8
    pp = dwf.default_params(check_every=1, paper_mode=1, inner_prec=dwf.F32, schur=2)
    xp = torch.zeros_like(bd)
    st, ip = op.solve(xp, bd, pp)
    assert st == 0 and ip.iters > 0 and ip.outer_iters == 1
    assert oracle.true_residual(p, U, xp.cpu().numpy(), b5) < 1e-4


def test_5d_split_rejections():
    import torch
    import paper_2602_14454_amd as dwf
    dims = (4, 4, 2, 2)
    U = dwfgen.make_links(dims, 0.5, 46)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    for Ls, b, c, prec in ((4, 1.5, 0.5, dwf.F64), (5, 1.0, 0.0, dwf.F64), (4, 1.0, 0.0, dwf.BF16)):
        op = dwf.Op(lat, Ls, 1.8, 0.02, b, c, 1.0)
        V = int(np.prod(dims))
        x = torch.zeros((Ls, V, 4, 3), dtype=torch.complex128, device="cuda")
        with pytest.raises(dwf.DwfError):
            op.apply_eo5(torch.empty_like(x), x, prec=prec)
        prm = dwf.default_params(schur=2, algo=dwf.ALGO_DC, inner_prec=prec) if prec == dwf.BF16 else \
            dwf.default_params(schur=2)
        with pytest.raises(dwf.DwfError):
            op.solve(torch.empty_like(x), x, prm)
    op = dwf.Op(lat, 4, 1.8, 0.02, 1.0, 0.0, 1.0)
    x = torch.zeros((4, int(np.prod(dims)), 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dwf.DwfError):
        op.solve(torch.empty_like(x), x, dwf.default_params(schur=2, algo=dwf.ALGO_MIXED))


def test_dhat5_matches_oracle_16c4():
    """D^5 and its adjoint on 16^4, Ls = 8 (1024 blocks of the 5D kernel), smeared links,
    alpha = 0.5, against the oracle's restriction element by element."""
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (16, 16, 16, 16), 8
    lat, op, p, U = _setup(dims, Ls, 1.8, 0.01, 1.0, 0.5, seed=47, nsmear=2)
    print(f"[eo5d] 16^4 Ls {Ls}", flush=True)
    x = dwfgen.gaussian_source_5d(dims, Ls, 48)
    xd = _dev(x)
    for dag in (False, True):
        ref = eo5.dhat5(p, U, x, dagger=dag)
        for prec, tol in ((dwf.F64, 1e-13), (dwf.F32, 1e-5)):
            out = torch.empty_like(xd)
            op.apply_eo5(out, xd, dagger=dag, prec=prec)
            err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
            assert err < tol, (dag, prec, err)
