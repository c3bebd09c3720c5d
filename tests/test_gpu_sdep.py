"""GPU parity of the operator with s-dependent coefficients b_i, c_i
(Sec. 2.2: D_+^(i) = b_i D_W + 1, D_-^(i) = c_i D_W - 1 in row i) against
the FP64 oracle, element by element in FP64 / FP32 / BF16 (1e-13 / 1e-5 /
3e-2 relative max-norm), on lattices with ragged tails: Chiu's optimal
b_i = c_i = omega_i (Zolotarev weights), a Moebius-type set with
b_i - c_i constant and a general s-dependent set; the source with
c_1 != c_Ls; constant arrays against the s-independent entry point (same
bits); and solves checked by the oracle's true 5D and 4D residuals."""
import numpy as np
import pytest

import dwfgen
import oracle

pytestmark = pytest.mark.gpu

TOL = {0: 1e-13, 1: 1e-5, 2: 3e-2}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _coef_sets(Ls):
    w = dwfgen.zolotarev_omega(Ls, 0.1, 6.5)
    bm = 1.1 + 0.1 * np.arange(Ls)
    bg = 1.0 + 0.3 * np.sin(np.arange(Ls))
    cg = 0.2 + 0.25 * np.cos(1.7 * np.arange(Ls))
    return {"chiu": (w, w), "moebius_sdep": (bm, bm - 0.7), "general": (bg, cg)}


CASES = [((4, 4, 6, 4), 6, 1.8, 0.02, 0.6), ((6, 4, 2, 4), 8, 1.6, 0.05, 0.5), ((4, 2, 4, 2), 12, 1.7, 0.01, 1.0)]


def _make(case, which, seed=3):
    import paper_2602_14454_amd as dwf
    dims, Ls, M0, m, al = case
    bs, cs = _coef_sets(Ls)[which]
    U = dwfgen.random_su3_links(dims, 0.5, seed)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, M0, m, list(bs), list(cs), al)
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, alpha=al, bs=tuple(bs), cs=tuple(cs))
    return lat, op, p, U


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("which", ["chiu", "moebius_sdep", "general"])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_sdep_operators(case, which, prec):
    import torch
    import paper_2602_14454_amd as dwf
    lat, op, p, U = _make(case, which)
    psi = dwfgen.gaussian_source_5d(p.dims, p.Ls, 7)
    out = torch.empty((p.Ls, p.V, 4, 3), dtype=torch.complex128, device="cuda")
    for dag in (0, 1):
        op.apply(out, _dev(psi), space=dwf.FULL5D, dagger=dag, prec=prec)
        assert _rel(out.cpu().numpy(), oracle.dwf_apply(p, U, psi, dagger=bool(dag))) < TOL[prec]
    xe = psi[:, : p.Vh].copy()
    oute = torch.empty((p.Ls, p.Vh, 4, 3), dtype=torch.complex128, device="cuda")
    for dag in (0, 1):
        op.apply(oute, _dev(xe), space=dwf.EVEN5D, dagger=dag, prec=prec)
        assert _rel(oute.cpu().numpy(), oracle.dhat(p, U, xe, dagger=bool(dag))) < TOL[prec]
    op.apply_normal(oute, _dev(xe), prec=prec)
    assert _rel(oute.cpu().numpy(), oracle.dhat(p, U, oracle.dhat(p, U, xe), dagger=True)) < TOL[prec]


@pytest.mark.parametrize("which", ["chiu", "general"])
def test_sdep_source(which):
    import torch
    lat, op, p, U = _make(CASES[0], which)
    b4 = dwfgen.gaussian_source_4d(p.dims, 4)
    b5 = torch.empty((p.Ls, p.V, 4, 3), dtype=torch.complex128, device="cuda")
    op.source_4d(b5, _dev(b4))
    assert _rel(b5.cpu().numpy(), oracle.source_4d(p, U, b4)) < 1e-14


def test_constant_arrays_same_bits_as_scalar_entry():
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 2, 6), 8
    U = dwfgen.random_su3_links(dims, 0.5, 9)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    a = dwf.Op(lat, Ls, 1.6, 0.03, 1.5, 0.5, 0.6)
    b = dwf.Op(lat, Ls, 1.6, 0.03, [1.5] * Ls, [0.5] * Ls, 0.6)
    xe = _dev(dwfgen.gaussian_source_5d(dims, Ls, 2)[:, : lat_vh(dims)])
    for prec in (0, 1, 2):
        oa, ob = torch.empty_like(xe), torch.empty_like(xe)
        a.apply_normal(oa, xe, prec=prec)
        b.apply_normal(ob, xe, prec=prec)
        assert torch.equal(oa, ob)


def lat_vh(dims):
    return int(np.prod(dims)) // 2


@pytest.mark.parametrize("which", ["chiu", "moebius_sdep"])
@pytest.mark.parametrize("algo", ["cgnr", "dc_f32"])
def test_sdep_solve_against_oracle(which, algo):
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 6), 8
    lat, op, p, U = _make((dims, Ls, 1.8, 0.02, 0.5), which, seed=5)
    b4 = dwfgen.gaussian_source_4d(dims, 6)
    b5 = torch.empty((Ls, p.V, 4, 3), dtype=torch.complex128, device="cuda")
    op.source_4d(b5, _dev(b4))
    prm = (dwf.default_params(tol=1e-11, check_every=4) if algo == "cgnr" else
           dwf.default_params(tol=1e-11, check_every=4, algo=dwf.ALGO_DC, inner_prec=dwf.F32))
    x5 = torch.zeros_like(b5)
    st, info = op.solve(x5, b5, prm)
    assert st == 0 and info.converged
    assert oracle.true_residual(p, U, x5.cpu().numpy(), b5.cpu().numpy()) <= 1e-11
    x4 = torch.empty((p.V, 4, 3), dtype=torch.complex128, device="cuda")
    op.project_4d(x4, x5)
    x4h = x4.cpu().numpy()
    assert oracle.residual_4d(p, U, x4h, b4) <= 1e-10
    assert op.residual_4d(x4, _dev(b4)) <= 1e-10
