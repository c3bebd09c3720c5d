"""Oracle pins: gamma algebra (Sec. 2.1), site maps and neighbours (Sec. 2.3, even-odd)."""
import numpy as np
import pytest

import oracle


def test_clifford_algebra_and_gamma5():
    g = [oracle.gamma(mu) for mu in range(4)]
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2.0 * np.eye(4) * (mu == nu), atol=1e-15)
    g5 = oracle.gamma(4)
    # gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4, Hermitian, squares to 1, anticommutes
    assert np.allclose(g5, g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g5 @ g5, np.eye(4))
    for mu in range(4):
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0)
    # chiral basis: P+ selects spins 0,1 and P- spins 2,3
    assert np.allclose(g5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 4, 8), (8, 6, 2, 4)])
def test_site_maps_bijection(dims):
    V = int(np.prod(dims))
    par, eo, le, lo = oracle.site_maps(dims)
    Lx, Ly, Lz, Lt = dims
    lex = np.arange(V)
    x = lex % Lx
    y = (lex // Lx) % Ly
    z = (lex // (Lx * Ly)) % Lz
    t = lex // (Lx * Ly * Lz)
    assert np.array_equal(par, (x + y + z + t) & 1)
    assert np.array_equal(eo, lex >> 1)
    assert np.array_equal(np.sort(le), np.sort(lex[par == 0]))
    assert np.array_equal(np.sort(lo), np.sort(lex[par == 1]))
    assert np.array_equal(le >> 1, np.arange(V // 2))
    assert np.array_equal(lo >> 1, np.arange(V // 2))


def test_neighbors_formula():
    dims = (4, 6, 2, 8)
    nbr = oracle.neighbors(dims)
    Lx, Ly, Lz, Lt = dims
    V = int(np.prod(dims))
    c = np.stack(np.unravel_index(np.arange(V), (Lt, Lz, Ly, Lx))[::-1], axis=1)
    for mu in range(4):
        for k, d in enumerate((+1, -1)):
            cc = c.copy()
            cc[:, mu] = (cc[:, mu] + d) % dims[mu]
            want = cc[:, 0] + Lx * (cc[:, 1] + Ly * (cc[:, 2] + Lz * cc[:, 3]))
            assert np.array_equal(nbr[:, 2 * mu + k], want)
