"""Even-odd split by 5D parity, written out from its definition -- TEST
INFRASTRUCTURE (only tests/ may import it).

Sec. 2.3: the sites can be divided into even and odd in five dimensions as
well as in four.  With "e" the (s, x) whose (x + y + z + t + s) is even
(s = 0..Ls-1) the Schur operator of eq. even-odd_linear_equation is

    D^5 = 1 - D_ee^-1 D_eo D_oo^-1 D_oe,

where every block is the oracle's 5D operator restricted to the parity
subspaces (masks on input and output).  D_ee and D_oo are then the
site-and-s-diagonal part of the operator: for c = 0 the diagonal of the
oracle's site-local block (the operator with D_W replaced by its
site-diagonal part), for even Ls (the mass term joins s = Ls-1 to s = 0,
which have the same 5D parity when Ls is odd).  No new arithmetic beyond
the oracle's operator, the masks and a division by that diagonal.
"""
from __future__ import annotations

import numpy as np

from . import Params, dwf_apply, local_block, site_maps


def even_mask(p: Params) -> np.ndarray:
    """Boolean (Ls, V): True where (x + y + z + t + s) is even."""
    par4, _, _, _ = site_maps(p.dims)
    return ((par4[None, :] + np.arange(p.Ls)[:, None]) & 1) == 0


def diagonal(p: Params) -> np.ndarray:
    """(Ls, 4) diagonal of D restricted to one site and slice (c = 0: D_ee = D_oo = this)."""
    cs = p.cs if p.cs is not None else [p.c] * p.Ls
    if any(float(c) != 0.0 for c in cs):
        raise ValueError("the 5D-diagonal blocks are local only for c = 0")
    if p.Ls % 2:
        # the mass term couples s = Ls-1 to s = 0: same 5D parity for odd Ls
        raise ValueError("the 5D split needs an even Ls")
    M = local_block(p)
    d = np.diag(M).reshape(p.Ls, 4)
    off = M - np.diag(np.diag(M))
    # within one slice the block is diagonal in spin (the s-couplings are off-slice)
    for s in range(p.Ls):
        assert np.abs(off[4 * s:4 * s + 4, 4 * s:4 * s + 4]).max() == 0.0
    return d


def dhat5(p: Params, U, x5, dagger: bool = False) -> np.ndarray:
    """D^5 x (or D^5^dag x) on the 5D-even entries of a canonical (Ls, V, 4, 3) field;
    the 5D-odd entries of the result are zero."""
    e = even_mask(p)[:, :, None, None]
    o = ~e
    d = diagonal(p)[:, None, :, None]   # broadcast over sites and colour
    x = np.where(e, np.asarray(x5, np.complex128), 0.0)
    if not dagger:
        z = np.where(o, dwf_apply(p, U, x), 0.0) / d          # D_oo^-1 D_oe x
        w = np.where(e, dwf_apply(p, U, z), 0.0) / d          # D_ee^-1 D_eo z
    else:
        # (D_ee^-1 D_eo D_oo^-1 D_oe)^dag = D_oe^dag D_oo^-1 D_eo^dag D_ee^-1 (real diagonal blocks)
        z = np.where(o, dwf_apply(p, U, x / d, dagger=True), 0.0)
        w = np.where(e, dwf_apply(p, U, np.where(o, z / d, 0.0), dagger=True), 0.0)
    return np.where(e, x - w, 0.0)
