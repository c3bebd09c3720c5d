"""FP64 oracle of the learned preconditioner: a gauge-equivariant
parallel-transport convolution (PTC) network, its loss, analytic gradients
and the Adam update.  Test infrastructure only.

Network (linear, two layers, 1 -> H -> 1 channels):

    out^a(x, s) = sum_b sum_p  W_p^{ab} . T_p[in^b](x, s)

with W_p^{ab} a complex 4x4 matrix acting on spin (identity on colour) and
the 11 paths
    p = 0            identity
    p = 1..4         T_{+mu} psi(x) = U_mu(x) psi(x + mu)        mu = x, y, z, t
    p = 5..8         T_{-mu} psi(x) = U_mu(x - mu)^dag psi(x - mu)
    p = 9, 10        psi(x, s + 1), psi(x, s - 1) (zero outside 0..Ls-1)
The fermion boundary phase (antiperiodic in t) is part of the transport, so
a transport across the t boundary carries a factor -1.  Layer 1 reads an
even-site field (zero on odd sites) and writes the hidden channels on all
sites; layer 2 reads them and the result is kept on even sites.  Under a
gauge transformation psi -> g psi, U_mu(x) -> g(x) U_mu(x) g(x + mu)^dag the
network is equivariant: M[U^g](g r) = g M[U](r).

Fields here are full-lattice arrays [ch][Ls][V][4][3] (complex128), V in
lexicographic order x + Lx (y + Ly (z + Lz t)).  Even-canonical vectors
([Ls][V/2][4][3], eo = lex >> 1 over parity-0 sites) convert with
`embed_even` / `restrict_even`.

Complex weight gradients are returned as dL/dRe W + i dL/dIm W.

Two losses for a pair (r, e) with r = A e (A = D^dag D^, Hermitian):
    kind 0:  |M r - e|^2 / |e|^2
    kind 1:  |A (M r - e)|^2 / |r|^2  (= |A M r - r|^2 / |r|^2)
The caller passes A as a function on even-canonical vectors.
"""
from __future__ import annotations

import numpy as np

NPATH = 11


def _shape5(dims):
    Lx, Ly, Lz, Lt = dims
    return (Lt, Lz, Ly, Lx)   # axis order of a lexicographic site index


def parity(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return ((x + y + z + t) & 1).reshape(-1)


def embed_even(dims, v_even):
    """[Ls][V/2][4][3] even canonical -> [Ls][V][4][3] with zeros on odd sites."""
    par = parity(dims)
    Ls = v_even.shape[0]
    out = np.zeros((Ls, par.size, 4, 3), dtype=np.complex128)
    out[:, par == 0] = v_even
    return out


def restrict_even(dims, v):
    par = parity(dims)
    return np.ascontiguousarray(v[..., par == 0, :, :])


def _links5(U, dims):
    """U [V][4][3][3] -> [4][Lt][Lz][Ly][Lx][3][3] (mu first)."""
    return np.moveaxis(np.asarray(U).reshape(_shape5(dims) + (4, 3, 3)), 4, 0)


def transport(U, dims, psi, p, antiperiodic_t=True):
    """T_p psi for psi [..., Ls, V, 4, 3] (leading axes are channels)."""
    psi = np.asarray(psi)
    if p == 0:
        return psi.copy()
    if p in (9, 10):
        out = np.zeros_like(psi)
        if p == 9:
            out[..., :-1, :, :, :] = psi[..., 1:, :, :, :]
        else:
            out[..., 1:, :, :, :] = psi[..., :-1, :, :, :]
        return out
    lead = psi.shape[:-3]
    Ls = psi.shape[-4]
    f = psi.reshape(lead[:-1] + (Ls,) + _shape5(dims) + (4, 3))
    mu = (p - 1) % 4
    axis = -3 - mu           # x -> -3, y -> -4, z -> -5, t -> -6 (before spin, colour)
    L = _links5(U, dims)[mu]  # [Lt][Lz][Ly][Lx][3][3]
    n = dims[mu]
    if p <= 4:
        # U_mu(x) psi(x + mu)
        sh = np.roll(f, -1, axis=axis)
        if mu == 3 and antiperiodic_t:
            idx = [slice(None)] * sh.ndim
            idx[axis] = n - 1
            sh[tuple(idx)] *= -1.0
        out = np.einsum("tzyxab,...tzyxsb->...tzyxsa", L, sh)
    else:
        # U_mu(x - mu)^dag psi(x - mu)
        sh = np.roll(f, 1, axis=axis)
        Lm = np.roll(L, 1, axis=3 - mu)      # U_mu(x - mu); link axes t,z,y,x = 0..3
        if mu == 3 and antiperiodic_t:
            idx = [slice(None)] * sh.ndim
            idx[axis] = 0
            sh[tuple(idx)] *= -1.0
        out = np.einsum("tzyxba,...tzyxsb->...tzyxsa", Lm.conj(), sh)
    return out.reshape(psi.shape)


def reverse_path(p):
    if p == 0:
        return 0
    if 1 <= p <= 4:
        return p + 4
    if 5 <= p <= 8:
        return p - 4
    return 19 - p   # 9 <-> 10


def layer(U, dims, W, x, antiperiodic_t=True):
    """out^a = sum_b sum_p W[p, a, b] . T_p[x^b];  W [11][A][B][4][4], x [B][Ls][V][4][3]."""
    out = 0
    for p in range(NPATH):
        t = transport(U, dims, x, p, antiperiodic_t)
        out = out + np.einsum("abij,bsvjc->asvic", W[p], t)
    return out


def forward(U, dims, W1, W2, r_even, antiperiodic_t=True):
    """M r on even sites: r_even [Ls][V/2][4][3] -> [Ls][V/2][4][3]; also
    returns the hidden channels (all sites)."""
    r = embed_even(dims, r_even)[None]
    h = layer(U, dims, W1, r, antiperiodic_t)
    y = layer(U, dims, W2, h, antiperiodic_t)[0]
    return restrict_even(dims, y), h


def loss(U, dims, W1, W2, r_even, e_even, antiperiodic_t=True):
    y, _ = forward(U, dims, W1, W2, r_even, antiperiodic_t)
    d = y - e_even
    return float(np.vdot(d, d).real / np.vdot(e_even, e_even).real)


def _layer_backward(U, dims, W, x, g, antiperiodic_t):
    """Given out = layer(W, x) and g = dL/dRe out + i dL/dIm out, return
    (dL/dW, dL/dx) in the same complex convention."""
    A, B = W.shape[1], W.shape[2]
    gW = np.zeros_like(W)
    gx = np.zeros_like(x)
    for p in range(NPATH):
        t = transport(U, dims, x, p, antiperiodic_t)
        # out_i = W_ij t_j  ->  dL/dW_ij = sum g_i conj(t_j)
        gW[p] = np.einsum("asvic,bsvjc->abij", g, t.conj())
        # dL/dt_j = sum_i conj(W_ij) g_i, then the adjoint transport
        gt = np.einsum("abij,asvic->bsvjc", W[p].conj(), g)
        gx = gx + transport(U, dims, gt, reverse_path(p), antiperiodic_t)
    return gW, gx


def loss_residual(U, dims, W1, W2, r_even, e_even, apply_A, antiperiodic_t=True):
    y, _ = forward(U, dims, W1, W2, r_even, antiperiodic_t)
    u = apply_A(y - e_even)
    return float(np.vdot(u, u).real / np.vdot(r_even, r_even).real)


def gradients(U, dims, W1, W2, r_even, e_even, antiperiodic_t=True, kind=0, apply_A=None):
    """(loss, dL/dW1, dL/dW2) by the chain rule through both layers."""
    r = embed_even(dims, r_even)[None]
    h = layer(U, dims, W1, r, antiperiodic_t)
    yfull = layer(U, dims, W2, h, antiperiodic_t)
    y = restrict_even(dims, yfull[0])
    d = y - e_even
    if kind == 0:
        e2 = np.vdot(e_even, e_even).real
        L = float(np.vdot(d, d).real / e2)
        gy = embed_even(dims, 2.0 * d / e2)[None]
    else:
        # L = |A d|^2 / |r|^2, dL/dy = 2 A^dag A d / |r|^2 = 2 A A d / |r|^2
        u = apply_A(d)
        r2 = np.vdot(r_even, r_even).real
        L = float(np.vdot(u, u).real / r2)
        gy = embed_even(dims, 2.0 * apply_A(u) / r2)[None]
    gW2, gh = _layer_backward(U, dims, W2, h, gy, antiperiodic_t)
    gW1, _ = _layer_backward(U, dims, W1, r, gh, antiperiodic_t)
    return L, gW1, gW2


def adam(W, G, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) treating real and imaginary parts as
    independent parameters; step counts from 1.  Returns new (W, m, v)."""
    def split(z):
        return np.stack([z.real, z.imag])
    g = split(G)
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    w = split(W) - lr * mh / (np.sqrt(vh) + eps)
    return w[0] + 1j * w[1], m, v


def identity_weights(hidden):
    """W1, W2 with only the p = 0 path, channel 0 active and identity spin
    weights: M = I on even fields."""
    W1 = np.zeros((NPATH, hidden, 1, 4, 4), dtype=np.complex128)
    W2 = np.zeros((NPATH, 1, hidden, 4, 4), dtype=np.complex128)
    W1[0, 0, 0] = np.eye(4)
    W2[0, 0, 0] = np.eye(4)
    return W1, W2


def random_weights(hidden, seed, scale=0.3):
    rng = np.random.default_rng(seed)

    def c(shape):
        return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)
    return c((NPATH, hidden, 1, 4, 4)), c((NPATH, 1, hidden, 4, 4))
