"""Pins of the FP64 oracle of the learned preconditioner (parallel-transport
convolution network): closed forms, invariances and finite differences."""
import numpy as np
import pytest

import dwfgen
from oracle import ptc
from oracle import freefield as ff

DIMS = (4, 2, 2, 4)
LS = 3


def _rand_full(dims, Ls, seed, lead=()):
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    shape = lead + (Ls, V, 4, 3)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_identity_weights_give_identity():
    U = dwfgen.random_su3_links(DIMS, 0.7, 1)
    W1, W2 = ptc.identity_weights(8)
    r = ptc.restrict_even(DIMS, _rand_full(DIMS, LS, 2))
    y, h = ptc.forward(U, DIMS, W1, W2, r)
    assert np.array_equal(y, r)
    assert np.count_nonzero(h[1:]) == 0


@pytest.mark.parametrize("p", range(1, 9))
def test_transport_of_plane_wave_with_unit_links(p):
    """With U = 1, T_{+mu} e^{ik.x} u = e^{i k_mu} e^{ik.x} u and T_{-mu} the
    inverse phase, with antiperiodic momenta in t (closed form)."""
    dims = (4, 6, 2, 4)
    U = dwfgen.unit_links(dims)
    k = ff.momenta(dims)[17]
    u = _rand_full((1, 1, 1, 1), 2, 3).reshape(2, 4, 3)
    psi = np.stack([ff.plane_wave_4d(dims, k, u[s]) for s in range(2)])
    mu = (p - 1) % 4
    phase = np.exp(1j * k[mu]) if p <= 4 else np.exp(-1j * k[mu])
    assert np.allclose(ptc.transport(U, dims, psi, p), phase * psi, atol=1e-13)


@pytest.mark.parametrize("p", range(ptc.NPATH))
def test_transport_adjoint_and_inverse(p):
    """<T_p x, y> = <x, T_reverse(p) y>; for the link paths T_reverse T = 1."""
    U = dwfgen.random_su3_links(DIMS, 0.9, 4)
    x = _rand_full(DIMS, LS, 5, (2,))
    y = _rand_full(DIMS, LS, 6, (2,))
    q = ptc.reverse_path(p)
    lhs = np.vdot(ptc.transport(U, DIMS, x, p), y)
    rhs = np.vdot(x, ptc.transport(U, DIMS, y, q))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    if 1 <= p <= 8 or p == 0:
        assert np.allclose(ptc.transport(U, DIMS, ptc.transport(U, DIMS, x, p), q), x, atol=1e-13)


def test_s_shifts_do_not_wrap():
    U = dwfgen.unit_links(DIMS)
    x = np.zeros((LS, int(np.prod(DIMS)), 4, 3), np.complex128)
    x[0] = 1.0
    assert np.count_nonzero(ptc.transport(U, DIMS, x, 9)) == 0
    y = ptc.transport(U, DIMS, x, 10)
    assert np.array_equal(y[1], x[0]) and np.count_nonzero(y[0]) == 0 and np.count_nonzero(y[2]) == 0


def test_gauge_equivariance():
    """M[U^g](g r) = g M[U](r) for a random SU(3) gauge transformation g."""
    U = dwfgen.random_su3_links(DIMS, 0.8, 7)
    V = int(np.prod(DIMS))
    g = dwfgen.random_su3_links((V, 1, 1, 1), 1.5, 8)[:, 0]          # V random SU(3)
    Lx, Ly, Lz, Lt = DIMS
    lex = np.arange(V)
    xs, ys, zs, ts = lex % Lx, (lex // Lx) % Ly, (lex // (Lx * Ly)) % Lz, lex // (Lx * Ly * Lz)
    Ug = np.empty_like(U)
    for mu in range(4):
        c = [xs, ys, zs, ts]
        c[mu] = (c[mu] + 1) % DIMS[mu]
        fwd = c[0] + Lx * (c[1] + Ly * (c[2] + Lz * c[3]))
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(g[fwd], (0, 2, 1)))
    W1, W2 = ptc.random_weights(8, 9)
    r = _rand_full(DIMS, LS, 10)
    re = ptc.restrict_even(DIMS, r)
    gr = np.einsum("vab,svib->svia", g, r)
    y, _ = ptc.forward(U, DIMS, W1, W2, re)
    yg, _ = ptc.forward(Ug, DIMS, W1, W2, ptc.restrict_even(DIMS, gr))
    gy = np.einsum("vab,svib->svia", g[ptc.parity(DIMS) == 0], y)
    assert np.allclose(yg, gy, atol=1e-12)
    # a wrong link (U instead of U^g) breaks it
    yb, _ = ptc.forward(U, DIMS, W1, W2, ptc.restrict_even(DIMS, gr))
    assert not np.allclose(yb, gy, atol=1e-6)


def test_gradients_match_central_differences():
    """Analytic dL/dW against central finite differences (h = 1e-6, FP64)
    for sampled entries of both layers, real and imaginary parts."""
    U = dwfgen.random_su3_links(DIMS, 0.6, 11)
    W1, W2 = ptc.random_weights(4, 12)
    r = ptc.restrict_even(DIMS, _rand_full(DIMS, LS, 13))
    e = ptc.restrict_even(DIMS, _rand_full(DIMS, LS, 14))
    L, g1, g2 = ptc.gradients(U, DIMS, W1, W2, r, e)
    assert abs(L - ptc.loss(U, DIMS, W1, W2, r, e)) < 1e-14 * L
    rng = np.random.default_rng(15)
    h = 1e-6
    for W, G, which in ((W1, g1, 1), (W2, g2, 2)):
        for _ in range(12):
            idx = tuple(rng.integers(0, n) for n in W.shape)
            for unit in (1.0, 1j):
                Wp, Wm = W.copy(), W.copy()
                Wp[idx] += h * unit
                Wm[idx] -= h * unit
                args = (Wp, W2) if which == 1 else (W1, Wp)
                argm = (Wm, W2) if which == 1 else (W1, Wm)
                fd = (ptc.loss(U, DIMS, *args, r, e) - ptc.loss(U, DIMS, *argm, r, e)) / (2 * h)
                an = G[idx].real if unit == 1.0 else G[idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (which, idx, unit, fd, an)


def test_residual_loss_gradients_match_central_differences():
    """Residual loss |A (M r - e)|^2 / |r|^2 with A = D^dag D^ of the C
    oracle: analytic gradient against central differences, and the loss
    equals |A M r - r|^2 / |r|^2 when r = A e."""
    import oracle
    dims, Ls = (4, 2, 2, 2), 3
    U = dwfgen.random_su3_links(dims, 0.6, 21)
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.6, m=0.1, b=1.0, c=0.0, alpha=0.7)

    def A(v):
        return oracle.dhat(p, U, oracle.dhat(p, U, v), dagger=True)
    W1, W2 = ptc.random_weights(3, 22)
    e = ptc.restrict_even(dims, _rand_full(dims, Ls, 23))
    r = A(e)
    L, g1, g2 = ptc.gradients(U, dims, W1, W2, r, e, kind=1, apply_A=A)
    y, _ = ptc.forward(U, dims, W1, W2, r)
    res = A(y) - r
    assert abs(L - np.vdot(res, res).real / np.vdot(r, r).real) < 1e-12 * L
    rng = np.random.default_rng(24)
    h = 1e-6
    for W, G, which in ((W1, g1, 1), (W2, g2, 2)):
        for _ in range(8):
            idx = tuple(rng.integers(0, n) for n in W.shape)
            for unit in (1.0, 1j):
                Wp, Wm = W.copy(), W.copy()
                Wp[idx] += h * unit
                Wm[idx] -= h * unit
                args = (Wp, W2) if which == 1 else (W1, Wp)
                argm = (Wm, W2) if which == 1 else (W1, Wm)
                fd = (ptc.loss_residual(U, dims, *args, r, e, A) - ptc.loss_residual(U, dims, *argm, r, e, A)) / (2 * h)
                an = G[idx].real if unit == 1.0 else G[idx].imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (which, idx, unit, fd, an)


def test_adam_first_step_is_signed_lr():
    """From m = v = 0 the bias-corrected first Adam step is -lr sign(g)
    (up to eps), per real component."""
    rng = np.random.default_rng(16)
    W = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    G = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    m = np.zeros((2, 3, 4))
    v = np.zeros((2, 3, 4))
    Wn, m, v = ptc.adam(W, G, m, v, 1, lr=1e-3)
    d = Wn - W
    assert np.allclose(d.real, -1e-3 * np.sign(G.real), rtol=1e-6)
    assert np.allclose(d.imag, -1e-3 * np.sign(G.imag), rtol=1e-6)


def test_loss_zero_at_exact_map():
    U = dwfgen.random_su3_links(DIMS, 0.5, 17)
    W1, W2 = ptc.identity_weights(2)
    r = ptc.restrict_even(DIMS, _rand_full(DIMS, LS, 18))
    assert ptc.loss(U, DIMS, W1, W2, r, r) == 0.0
    assert abs(ptc.loss(U, DIMS, W1, W2, r, 2 * r) - 0.25) < 1e-15
