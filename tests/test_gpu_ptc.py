"""GPU kernels of the learned preconditioner against the FP64 oracle
(oracle/ptc.py): forward, loss and weight gradients element by element;
training pairs against the oracle's operator; checkpoint round trip; FGCR
with and without the network, its CGNR fallback, and the gain of training.
Tolerances are FP32 ones: the kernels run in FP32 with FP64 reductions."""
import numpy as np
import pytest

import dwfgen
import oracle
from oracle import ptc as optc

pytestmark = pytest.mark.gpu

CASES = [
    # dims, Ls, hidden
    ((4, 4, 2, 4), 4, 8),
    ((6, 2, 2, 4), 3, 3),     # Vh = 48 (one partial block), odd channel count
    ((4, 4, 4, 6), 5, 2),
]


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _setup(dims, Ls, seed=1):
    import paper_2602_14454_amd as dwf
    U = dwfgen.random_su3_links(dims, 0.6, seed)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, 1.6, 0.05, 1.0, 0.0, 0.5)
    return U, lat, op


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("case", CASES)
def test_forward_matches_oracle(case):
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls, H = case
    U, lat, op = _setup(dims, Ls)
    W1, W2 = optc.random_weights(H, 5)
    M = dwf.PtcModel(H)
    M.set_weights(W1, W2)
    V = int(np.prod(dims))
    r = dwfgen.gaussian_source_5d(dims, Ls, 6)[:, : V // 2].copy()
    out = torch.empty((Ls, V // 2, 4, 3), dtype=torch.complex128, device="cuda")
    M.apply(op, out, _dev(r))
    want, _ = optc.forward(U, dims, W1.astype(np.complex64).astype(np.complex128),
                           W2.astype(np.complex64).astype(np.complex128), r.astype(np.complex64))
    assert _rel(out.cpu().numpy(), want) < 2e-5


def test_identity_weights_pass_through():
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 2, 2), 4
    U, lat, op = _setup(dims, Ls)
    M = dwf.PtcModel(8)
    M.set_weights(*optc.identity_weights(8))
    r = dwfgen.gaussian_source_5d(dims, Ls, 2)[:, :16].copy()
    out = torch.empty((Ls, 16, 4, 3), dtype=torch.complex128, device="cuda")
    M.apply(op, out, _dev(r))
    assert np.array_equal(out.cpu().numpy(), r.astype(np.complex64).astype(np.complex128))


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("kind", [0, 1])
def test_gradient_matches_oracle(case, kind):
    """Both losses; for the residual loss the oracle applies A = D^dag D^ with
    its own operator and r = A e is built from the oracle too."""
    import paper_2602_14454_amd as dwf
    dims, Ls, H = case
    U, lat, op = _setup(dims, Ls, seed=3)
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=0.05, b=1.0, c=0.0, alpha=0.5)

    def A(v):
        return oracle.dhat(p, U, oracle.dhat(p, U, v), dagger=True)
    W1, W2 = optc.random_weights(H, 7)
    W1 = W1.astype(np.complex64).astype(np.complex128)
    W2 = W2.astype(np.complex64).astype(np.complex128)
    M = dwf.PtcModel(H)
    M.set_weights(W1, W2)
    M.set_loss(kind)
    V = int(np.prod(dims))
    e = dwfgen.gaussian_source_5d(dims, Ls, 9)[:, : V // 2].astype(np.complex64).astype(np.complex128)
    if kind == 0:
        r = dwfgen.gaussian_source_5d(dims, Ls, 8)[:, : V // 2].astype(np.complex64).astype(np.complex128)
    else:
        r = A(e).astype(np.complex64).astype(np.complex128)
    loss, (g1, g2) = M.gradient(op, _dev(r), _dev(e))
    L, o1, o2 = optc.gradients(U, dims, W1, W2, r, e, kind=kind, apply_A=A)
    assert abs(loss - L) < 3e-5 * L
    for g, o in ((g1, o1), (g2, o2)):
        err = np.linalg.norm(g - o) / np.linalg.norm(o)
        assert err < 3e-5, err


def test_pairs_and_training():
    """Pairs satisfy r_k = D^dag D^ e_k (oracle operator) and e_0 = x*; a
    short training run lowers the loss; a checkpoint reloads bit for bit and
    a corrupted one is refused."""
    import os
    import tempfile
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 4), 6
    U, lat, op = _setup(dims, Ls, seed=4)
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=0.05, b=1.0, c=0.0, alpha=0.5)
    V = int(np.prod(dims))
    b5 = dwfgen.gaussian_source_5d(dims, Ls, 10)
    pairs = dwf.PtcPairs(op, _dev(b5), [0, 3, 10, 20])
    rk = torch.empty((Ls, V // 2, 4, 3), dtype=torch.complex128, device="cuda")
    ek = torch.empty_like(rk)
    pairs.get(0, rk, ek)
    xstar = oracle.cgnr_even(p, U, oracle.schur_rhs(p, U, b5), 1e-12)[0]
    assert _rel(ek.cpu().numpy(), xstar) < 1e-6
    for k in (0, 2):
        pairs.get(k, rk, ek)
        e = ek.cpu().numpy()
        want = oracle.dhat(p, U, oracle.dhat(p, U, e), dagger=True)
        assert _rel(rk.cpu().numpy(), want) < 1e-5
    M = dwf.PtcModel(8, seed=3, init_scale=0.05)
    before = M.eval([pairs])
    hist = M.train([pairs], 150, lr=2e-3)
    after = M.eval([pairs])
    assert np.all(np.isfinite(hist)) and after < before and M.steps == 150
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "m.ptc")
        M.save(f)
        M2 = dwf.PtcModel.load_file(f)
        assert M2.steps == 150
        for a, b in zip(M.weights(), M2.weights()):
            assert np.array_equal(a, b)
        raw = bytearray(open(f, "rb").read())
        raw[100] ^= 0x40
        open(f, "wb").write(bytes(raw))
        with pytest.raises(dwf.DwfError):
            dwf.PtcModel.load_file(f)


def _fgcr_solve(op, b5, model, restart=8, nan=False):
    import torch
    import paper_2602_14454_amd as dwf
    prm = dwf.default_params(algo=dwf.ALGO_FGCR_LEARNED, tol=1e-10, check_every=4, restart=restart)
    prm.ptc_model = model._h.value if model is not None else None
    x5 = torch.zeros_like(b5)
    st, info = op.solve(x5, b5, prm)
    return st, info, x5


def test_fgcr_converges_and_falls_back():
    import paper_2602_14454_amd as dwf
    dims, Ls = (4, 4, 4, 4), 6
    U, lat, op = _setup(dims, Ls, seed=5)
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=0.05, b=1.0, c=0.0, alpha=0.5)
    b5 = dwfgen.gaussian_source_5d(dims, Ls, 11)
    bd = _dev(b5)
    st, info, x5 = _fgcr_solve(op, bd, None)
    assert st == 0 and info.converged and not info.fallback_used
    assert oracle.true_residual(p, U, x5.cpu().numpy(), b5) <= 1.2e-10
    M = dwf.PtcModel(8, seed=2, init_scale=0.02)
    st, info, x5 = _fgcr_solve(op, bd, M)
    assert st == 0 and info.converged
    assert oracle.true_residual(p, U, x5.cpu().numpy(), b5) <= 1.2e-10
    # NaN weights: the network output is NaN, FGCR fails, CGNR finishes the solve
    W1, W2 = M.weights()
    W1 = W1.copy()
    W1[3, 2, 0, 1, 1] = np.nan
    M.set_weights(W1, W2)
    st, info, x5 = _fgcr_solve(op, bd, M)
    assert st == 0 and info.converged and info.fallback_used
    assert oracle.true_residual(p, U, x5.cpu().numpy(), b5) <= 1.2e-10


def test_training_gains_over_identity():
    """Trained on solver-generated pairs (known-solution systems and CGNR
    trajectories) of other gauge fields, the network cuts the FGCR
    iterations on a held-out field below those without it (M = I) and
    below those of the untrained network."""
    import paper_2602_14454_amd as dwf
    dims, Ls, m = (6, 6, 6, 6), 6, 0.02
    sets, keep = [], []
    for sd in range(3):
        U = dwfgen.make_links(dims, 0.5, 40 + sd, rho=0.1, nsmear=2)
        import paper_2602_14454_amd as dwf
        lat = dwf.Lattice(dims)
        lat.set_gauge(U)
        op = dwf.Op(lat, Ls, 1.6, m, 1.0, 0.0, 0.5)
        sets.append(dwf.PtcPairs(op, None, [0, 1, 2, 4, 8], seed=60 + sd))
        keep.append(lat)
    U = dwfgen.make_links(dims, 0.5, 50, rho=0.1, nsmear=2)
    lat = dwf.Lattice(dims)
    lat.set_gauge(U)
    op = dwf.Op(lat, Ls, 1.6, m, 1.0, 0.0, 0.5)
    b5 = _dev(dwfgen.gaussian_source_5d(dims, Ls, 51))
    _, base, _ = _fgcr_solve(op, b5, None, restart=16)
    M = dwf.PtcModel(8, seed=4, init_scale=0.02)
    _, untrained, _ = _fgcr_solve(op, b5, M, restart=16)
    before = M.eval(sets)
    M.train(sets, 600, lr=2e-3, seed=5)
    assert M.eval(sets) < 0.5 * before
    st, trained, x5 = _fgcr_solve(op, b5, M, restart=16)
    assert st == 0 and trained.converged and not trained.fallback_used
    assert trained.iters <= 0.85 * base.iters, (trained.iters, base.iters)
    assert trained.iters < untrained.iters
