"""Element-wise and solve parity at the full sizes of the workloads.

* 16^3x32, Ls = 16 (M0 = 1.6, m = 0.01, Neff alpha = 0.5, smeared links):
  D^, D^dag, D^dag D^ element by element in FP64, FP32 and BF16 against the
  oracle (padded row stride, 1024-site bricks, the fused stage-2 chain and
  stage-4 epilogues at their real launch sizes).
* A lattice whose spatial volume is above 16^3 (20x20x12x4), where the site
  order uses 4096-site bricks: D^ and D^dag D^ in every precision.
* 24^3x48, Ls = 16 (M0 = 1.8, m = 0.005, Neff alpha = 0.5, smeared links, the
  headline workload): D^ element by element in every precision, and the
  defect-correction solve with FP32 inner CG as the benchmark times it,
  checked by the oracle's true 5D residual; its 4D residual comes from the
  library's dwf_residual_4d (which is compared with the oracle's on small
  lattices in test_gpu_solver.py; the oracle's own needs a full m = 1 solve,
  hours at this size).
* The 12 spin-colour point sources on 16^3x32, Ls = 12 as one batched solve:
  two sampled right-hand sides checked by the oracle's true residual.
* Failure paths of a single solve: a tolerance below the FP64 floor forces the
  stagnation step-up BF16 -> FP32 -> FP64 and ends DWF_NOT_CONVERGED with the
  best iterate; a small maxiter ends DWF_NOT_CONVERGED in FP64 CGNR and in
  paper mode.
Tolerances as in test_gpu_operator.py: 1e-13 / 1e-5 / 3e-2 relative max-norm.
"""
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


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


def _operator(dims, Ls, M0, m, alpha, seed, nsmear=3):
    import paper_2602_14454_amd as dwf
    U = dwfgen.make_links(dims, 0.5, seed, rho=0.1, nsmear=nsmear)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, M0, m, 1.0, 0.0, alpha)
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=1.0, c=0.0, alpha=alpha)
    return U, lat, op, p


def _check_ops(op, p, U, normal=True, dagger=True, seed=8):
    import torch
    import paper_2602_14454_amd as dwf
    xe = dwfgen.gaussian_source_5d(p.dims, p.Ls, seed)[:, : p.Vh].copy()
    want = {"dhat": oracle.dhat(p, U, xe)}
    if dagger:
        want["dhat_dag"] = oracle.dhat(p, U, xe, dagger=True)
    if normal:
        want["normal"] = oracle.dhat(p, U, want["dhat"], dagger=True)
    xd = _dev(xe)
    out = torch.empty_like(xd)
    for prec in (0, 1, 2):
        for name, ref in want.items():
            if name == "normal":
                op.apply_normal(out, xd, prec=prec)
            else:
                op.apply(out, xd, space=dwf.EVEN5D, dagger=int(name == "dhat_dag"), prec=prec)
            err = _rel(out.cpu().numpy(), ref)
            _say(f"{p.dims} Ls={p.Ls} {name} prec {prec}: {err:.2e}")
            assert err < TOL[prec], (name, prec, err)


@pytest.mark.timeout(600)
def test_operators_16c32_ls16_elementwise():
    U, lat, op, p = _operator((16, 16, 16, 32), 16, 1.6, 0.01, 0.5, 11)
    _check_ops(op, p, U)


@pytest.mark.timeout(300)
def test_operators_above_16cubed_spatial_elementwise():
    # spatial volume 4800 > 16^3: the site order cuts it into 20x10x12 bricks
    U, lat, op, p = _operator((20, 20, 12, 4), 16, 1.6, 0.02, 0.5, 5, nsmear=1)
    _check_ops(op, p, U)


@pytest.fixture(scope="module")
def c3():
    import torch
    _say("24^3x48 links (3 stout steps)")
    U, lat, op, p = _operator((24, 24, 24, 48), 16, 1.8, 0.005, 0.5, 21)
    b4h = dwfgen.gaussian_source_4d(p.dims, 22)
    b4 = _dev(b4h)
    b5 = torch.empty((p.Ls, p.V, 4, 3), dtype=torch.complex128, device="cuda")
    op.source_4d(b5, b4)
    return U, lat, op, p, b4, b5


@pytest.mark.timeout(900)
def test_operators_24c48_ls16_dhat_elementwise(c3):
    U, lat, op, p, b4, b5 = c3
    _check_ops(op, p, U, normal=False, dagger=False)


@pytest.mark.timeout(900)
def test_solve_24c48_dc_f32_against_oracle(c3):
    import torch
    import paper_2602_14454_amd as dwf
    U, lat, op, p, b4, b5 = c3
    prm = dwf.default_params(tol=1e-10, check_every=8, algo=dwf.ALGO_DC, inner_prec=dwf.F32)
    x5 = torch.zeros_like(b5)
    st, info = op.solve(x5, b5, prm)
    _say(f"24^3x48 DC-FP32: status {st} iters {info.iters} outer {info.outer_iters} true_res5 {info.true_res5:.2e}")
    assert st == 0 and info.converged and info.true_res5 <= 1e-10
    r5 = oracle.true_residual(p, U, x5.cpu().numpy(), b5.cpu().numpy())
    _say(f"oracle true_res5 {r5:.3e}")
    assert r5 <= 1e-10 and abs(r5 - info.true_res5) <= 0.05 * r5
    x4 = torch.empty((p.V, 4, 3), dtype=torch.complex128, device="cuda")
    op.project_4d(x4, x5)
    r4 = op.residual_4d(x4, b4)
    _say(f"res4 {r4:.3e}")
    assert r4 <= 1e-10


@pytest.mark.timeout(600)
def test_point_source_batch_16c32_ls12_sampled_slots():
    import torch
    import paper_2602_14454_amd as dwf
    U, lat, op, p = _operator((16, 16, 16, 32), 12, 1.6, 0.01, 0.5, 31)
    b4 = torch.stack([torch.from_numpy(dwfgen.point_source_4d(p.dims, s, c)) for s in range(4) for c in range(3)])
    b4 = b4.to("cuda")
    b5 = torch.empty((12, p.Ls, p.V, 4, 3), dtype=torch.complex128, device="cuda")
    for k in range(12):
        op.source_4d(b5[k], b4[k])
    x5 = torch.zeros_like(b5)
    prm = dwf.default_params(algo=dwf.ALGO_DC, inner_prec=dwf.F32, check_every=8, tol=1e-10)
    st, infos = dwf.solve_batch([op], [x5], [b5], [12], prm)
    _say(f"point-source batch: status {st}, iters {[f.iters for f in infos]}")
    assert st == 0 and all(f.converged for f in infos)
    for k in (0, 7):
        r5 = oracle.true_residual(p, U, x5[k].cpu().numpy(), b5[k].cpu().numpy())
        _say(f"slot {k}: library {infos[k].true_res5:.3e} oracle {r5:.3e}")
        assert r5 <= 1e-10 and abs(r5 - infos[k].true_res5) <= 0.05 * r5


def test_stagnation_step_up_and_not_converged():
    """tol = 1e-17 is below what an FP64 residual can show: BF16 defect
    correction stagnates, steps up to FP32, then FP64, and the solve ends
    DWF_NOT_CONVERGED at maxiter with its best iterate (still an accurate
    solution)."""
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 4), 8
    U, lat, op, p = _operator(dims, Ls, 1.6, 0.05, 0.5, 1, nsmear=0)
    b5h = dwfgen.gaussian_source_5d(dims, Ls, 2)
    b5 = _dev(b5h)
    x5 = torch.zeros_like(b5)
    prm = dwf.default_params(tol=1e-17, maxiter=3000, check_every=4, algo=dwf.ALGO_DC, inner_prec=dwf.BF16)
    st, info = op.solve(x5, b5, prm)
    _say(f"step-up: status {st} iters {info.iters} outer {info.outer_iters} fallback {info.fallback_used} "
         f"final prec {info.final_inner_prec} true_res5 {info.true_res5:.2e}")
    assert st == dwf.NOT_CONVERGED and not info.converged
    assert info.fallback_used == 1 and info.final_inner_prec == dwf.F64
    assert oracle.true_residual(p, U, x5.cpu().numpy(), b5h) <= 1e-13


def test_maxiter_not_converged():
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 4), 8
    U, lat, op, p = _operator(dims, Ls, 1.6, 0.05, 0.5, 1, nsmear=0)
    b5 = _dev(dwfgen.gaussian_source_5d(dims, Ls, 2))
    for prm in (dwf.default_params(tol=1e-10, maxiter=5),
                dwf.default_params(tol=1e-10, maxiter=4, algo=dwf.ALGO_DC, inner_prec=dwf.F32),
                dwf.default_params(maxiter=6, paper_mode=1, inner_prec=dwf.F32)):
        x5 = torch.zeros_like(b5)
        st, info = op.solve(x5, b5, prm)
        assert st == dwf.NOT_CONVERGED and not info.converged and info.iters <= prm.maxiter
        assert np.isfinite(x5.cpu().numpy()).all()
