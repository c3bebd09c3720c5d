"""Even-odd preconditioning in five dimensions (Sec. 2.3: sites can be split
into even and odd in 5D or in 4D; the solver uses the 4D split), checked on
dense matrices built from the oracle's 5D operator on a tiny lattice with
random links, Shamir (b, c) = (1, 0), where the 5D-diagonal blocks are
site- and s-local:

* the 5D split's Schur complement and reconstruction solve the 5D system;
* its D_ee is diagonal in (site, s), so D_ee^-1 is a local operation;
* the condition numbers of the normal operators (the quantity CGNR sees) of
  the 4D-left, 4D-right and 5D-left Schur forms at alpha = 1 and 0.5 are
  printed; the 4D-right one does not depend on alpha.
"""
import numpy as np
import pytest

import dwfgen
import oracle


def _dense(fn, n):
    cols = []
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1
        cols.append(fn(e).reshape(-1))
    return np.array(cols).T


def _schur(D, ie, io, right=False):
    Dee, Deo, Doe, Doo = (D[np.ix_(a, b)] for a, b in ((ie, ie), (ie, io), (io, ie), (io, io)))
    if right:
        return np.eye(len(ie)) - Deo @ np.linalg.solve(Doo, Doe @ np.linalg.inv(Dee))
    return np.eye(len(ie)) - np.linalg.solve(Dee, Deo @ np.linalg.solve(Doo, Doe))


def _kappa(A):
    s = np.linalg.svd(A, compute_uv=False)
    return float((s.max() / s.min()) ** 2)


def test_5d_even_odd_shamir(capsys):
    dims, Ls = (2, 2, 2, 4), 4
    U = dwfgen.random_su3_links(dims, 0.5, 17)
    par4, _, le, lo = oracle.site_maps(dims)
    V = int(np.prod(dims))
    n = Ls * V * 12
    idx = np.arange(n).reshape(Ls, V, 12)
    p5 = (par4[None, :] + np.arange(Ls)[:, None]) & 1          # 5D parity of (s, x)
    i5e = idx[p5 == 0].reshape(-1)
    i5o = idx[p5 == 1].reshape(-1)
    i4e, i4o = idx[:, le].reshape(-1), idx[:, lo].reshape(-1)
    out = {}
    for al in (1.0, 0.5):
        p = oracle.Params(dims=dims, Ls=Ls, M0=1.8, m=0.02, b=1.0, c=0.0, alpha=al)
        D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(Ls, V, 4, 3)), n)
        Dee5 = D[np.ix_(i5e, i5e)]
        assert np.abs(Dee5 - np.diag(np.diag(Dee5))).max() < 1e-14   # 5D-local: diagonal
        S5 = _schur(D, i5e, i5o)
        b5 = dwfgen.gaussian_source_5d(dims, Ls, 18).reshape(-1)
        be, bo = b5[i5e], b5[i5o]
        Dee, Deo, Doe, Doo = (D[np.ix_(a, b)] for a, b in ((i5e, i5e), (i5e, i5o), (i5o, i5e), (i5o, i5o)))
        bt = np.linalg.solve(Dee, be - Deo @ np.linalg.solve(Doo, bo))
        xe = np.linalg.solve(S5, bt)
        xo = np.linalg.solve(Doo, bo - Doe @ xe)
        x = np.empty(n, np.complex128)
        x[i5e], x[i5o] = xe, xo
        assert np.abs(D @ x - b5).max() < 1e-11 * np.abs(b5).max()
        out[al] = {"4d_left": _kappa(_schur(D, i4e, i4o)), "4d_right": _kappa(_schur(D, i4e, i4o, right=True)),
                   "5d_left": _kappa(S5)}
    assert abs(out[1.0]["4d_right"] - out[0.5]["4d_right"]) < 1e-8 * out[1.0]["4d_right"]
    with capsys.disabled():
        print("\n[eo5d] kappa of the normal operator (2^3x4, Ls=4, Shamir, M0=1.8, m=0.02):",
              {a: {k: round(v, 2) for k, v in d.items()} for a, d in out.items()})


def test_dhat5_helper_matches_dense_schur():
    """oracle.eo5.dhat5 (masks on the oracle's operator and a division by the
    5D-diagonal block) against the dense Schur complement of the same split,
    built with dense block solves and pinned above by solving the 5D system;
    the adjoint against the dense conjugate transpose.  Shamir-type c = 0 with
    b = 1.3, s-dependent b_s, Ls = 3 (a wrap-around in s at both ends)."""
    from oracle import eo5
    dims = (2, 2, 2, 4)
    U = dwfgen.random_su3_links(dims, 0.5, 23)
    par4, _, _, _ = oracle.site_maps(dims)
    V = int(np.prod(dims))
    rng = np.random.default_rng(24)
    for Ls, b, bs, al in ((4, 1.3, None, 0.5), (6, 1.0, (1.2, 0.9, 1.1, 1.0, 0.8, 1.3), 0.7), (4, 1.0, None, 1.0),
                          (2, 1.1, None, 0.6)):
        p = oracle.Params(dims=dims, Ls=Ls, M0=1.8, m=0.03, b=b, c=0.0, alpha=al, bs=bs)
        n = Ls * V * 12
        idx = np.arange(n).reshape(Ls, V, 12)
        p5 = (par4[None, :] + np.arange(Ls)[:, None]) & 1
        i5e, i5o = idx[p5 == 0].reshape(-1), idx[p5 == 1].reshape(-1)
        D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(Ls, V, 4, 3)), n)
        S5 = _schur(D, i5e, i5o)
        x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).reshape(Ls, V, 4, 3)
        xe = x.reshape(-1)[i5e]
        for dag, S in ((False, S5), (True, S5.conj().T)):
            y = eo5.dhat5(p, U, x, dagger=dag).reshape(-1)
            ref = S @ xe
            assert np.abs(y[i5e] - ref).max() < 1e-12 * np.abs(ref).max()
            assert np.abs(y[i5o]).max() == 0.0


def test_dhat5_helper_rejects_c_and_odd_ls():
    """c != 0 puts D_W into D_- (D_ee not local); for odd Ls the mass term
    couples slices of one 5D parity: the dense D_ee then has off-diagonal
    entries, and the helper refuses both cases."""
    from oracle import eo5
    p = oracle.Params(dims=(2, 2, 2, 2), Ls=4, M0=1.8, m=0.03, b=1.5, c=0.5, alpha=1.0)
    with pytest.raises(ValueError):
        eo5.diagonal(p)
    dims, Ls = (2, 2, 2, 2), 3
    p = oracle.Params(dims=dims, Ls=Ls, M0=1.8, m=0.03, b=1.0, c=0.0, alpha=1.0)
    with pytest.raises(ValueError):
        eo5.diagonal(p)
    U = dwfgen.random_su3_links(dims, 0.5, 25)
    V = int(np.prod(dims))
    n = Ls * V * 12
    D = _dense(lambda e: oracle.dwf_apply(p, U, e.reshape(Ls, V, 4, 3)), n)
    e = eo5.even_mask(oracle.Params(dims=dims, Ls=Ls, M0=1.8, m=0.03)).repeat(12, axis=1).reshape(-1)
    Dee = D[np.ix_(e, e)]
    assert np.abs(Dee - np.diag(np.diag(Dee))).max() == pytest.approx(0.03)
