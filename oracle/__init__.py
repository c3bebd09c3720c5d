"""FP64 CPU oracle for the domain-wall fermion solve -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.

The arithmetic lives in ``oracle.c`` (plain C99 + OpenMP, FP64), written from
the paper's definitions; this module only loads it with ctypes and marshals
numpy arrays.  ``freefield`` and ``dense`` hold the momentum-space closed
forms and the dense brute-force checks used to pin it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("antiperiodic_t", ctypes.c_int),
                ("Ls", ctypes.c_int), ("M0", ctypes.c_double), ("m", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double), ("alpha", ctypes.c_double),
                ("bs", ctypes.POINTER(ctypes.c_double)), ("cs", ctypes.POINTER(ctypes.c_double))]


@dataclass(frozen=True)
class Params:
    dims: tuple
    Ls: int
    M0: float
    m: float
    b: float = 1.0
    c: float = 0.0
    alpha: float = 1.0
    antiperiodic_t: int = 1
    bs: tuple = None   # s-dependent b_i (Ls values) or None: b for every s
    cs: tuple = None   # s-dependent c_i (Ls values) or None: c for every s

    @property
    def V(self) -> int:
        return int(np.prod(self.dims))

    @property
    def Vh(self) -> int:
        return self.V // 2

    def replace(self, **kw) -> "Params":
        d = dict(self.__dict__)
        d.update(kw)
        return Params(**d)

    def _c(self) -> _Params:
        p = _Params()
        for i in range(4):
            p.dims[i] = int(self.dims[i])
        p.antiperiodic_t = int(self.antiperiodic_t)
        p.Ls = int(self.Ls)
        p.M0, p.m, p.b, p.c, p.alpha = (float(self.M0), float(self.m), float(self.b),
                                        float(self.c), float(self.alpha))
        keep = []
        for name in ("bs", "cs"):
            v = getattr(self, name)
            if v is None:
                setattr(p, name, None)
                continue
            arr = (ctypes.c_double * int(self.Ls))(*[float(x) for x in v])
            if len(v) != int(self.Ls):
                raise ValueError(f"{name} needs Ls entries")
            keep.append(arr)
            setattr(p, name, ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)))
        p._keep = keep   # the arrays live as long as the struct
        return p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Params)
    vp = ctypes.c_void_p
    sig = {
        "or_volume": (ctypes.c_long, [vp]),
        "or_gamma": (None, [ctypes.c_int, vp]),
        "or_site_maps": (None, [vp, vp, vp, vp, vp]),
        "or_neighbors": (None, [vp, vp]),
        "or_wilson": (None, [P, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "or_dwf_apply": (None, [P, vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "or_local_block": (None, [P, vp]),
        "or_invert_dense": (ctypes.c_int, [ctypes.c_int, vp, vp]),
        "or_dhat": (None, [P, vp, vp, vp, ctypes.c_int]),
        "or_schur_rhs": (None, [P, vp, vp, vp]),
        "or_reconstruct": (None, [P, vp, vp, vp, vp]),
        "or_cgnr_even": (ctypes.c_int, [P, vp, vp, vp, ctypes.c_double, ctypes.c_int]),
        "or_solve": (ctypes.c_int, [P, vp, vp, vp, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double)]),
        "or_source_4d": (None, [P, vp, vp, vp]),
        "or_project_4d": (None, [P, vp, vp]),
        "or_residual_4d": (ctypes.c_double, [P, vp, vp, vp, ctypes.c_double]),
        "or_true_residual": (ctypes.c_double, [P, vp, vp, vp]),
        "or_num_threads": (ctypes.c_int, []),
        "or_set_num_threads": (None, [ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads used by later oracle calls (for CPU-baseline timing)."""
    _load().or_set_num_threads(int(n))


def gamma(mu: int) -> np.ndarray:
    """gamma_1..gamma_4 for mu = 0..3, gamma_5 for mu = 4 (chiral basis)."""
    out = np.zeros((4, 4), dtype=np.complex128)
    _load().or_gamma(mu, _ptr(out))
    return out


def site_maps(dims):
    dims_c = np.ascontiguousarray(dims, dtype=np.int32)
    V = int(np.prod(dims))
    par = np.zeros(V, np.int32)
    eo = np.zeros(V, np.int32)
    le = np.zeros(V // 2, np.int32)
    lo = np.zeros(V // 2, np.int32)
    _load().or_site_maps(_ptr(dims_c), _ptr(par), _ptr(eo), _ptr(le), _ptr(lo))
    return par, eo, le, lo


def neighbors(dims) -> np.ndarray:
    dims_c = np.ascontiguousarray(dims, dtype=np.int32)
    V = int(np.prod(dims))
    nbr = np.zeros((V, 8), np.int32)
    _load().or_neighbors(_ptr(dims_c), _ptr(nbr))
    return nbr


def wilson(p: Params, U, psi4, dagger=False, parity_mask=3) -> np.ndarray:
    U = _c128(U)
    x = _c128(psi4)
    out = np.empty_like(x)
    pc = p._c()
    _load().or_wilson(ctypes.byref(pc), _ptr(U), _ptr(x), _ptr(out), int(dagger), int(parity_mask))
    return out


def dwf_apply(p: Params, U, psi5, dagger=False, parity_mask=3) -> np.ndarray:
    """D^(alpha) psi5 (or its adjoint), full 5D canonical layout."""
    U = _c128(U)
    x = _c128(psi5)
    out = np.empty_like(x)
    pc = p._c()
    _load().or_dwf_apply(ctypes.byref(pc), _ptr(U), _ptr(x), _ptr(out), int(dagger), int(parity_mask))
    return out


def local_block(p: Params) -> np.ndarray:
    n = 4 * p.Ls
    out = np.zeros((n, n), np.complex128)
    pc = p._c()
    _load().or_local_block(ctypes.byref(pc), _ptr(out))
    return out


def invert_dense(A) -> np.ndarray:
    A = _c128(A)
    out = np.empty_like(A)
    rc = _load().or_invert_dense(A.shape[0], _ptr(A), _ptr(out))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return out


def dhat(p: Params, U, x_e, dagger=False) -> np.ndarray:
    U = _c128(U)
    x = _c128(x_e)
    out = np.empty_like(x)
    pc = p._c()
    _load().or_dhat(ctypes.byref(pc), _ptr(U), _ptr(x), _ptr(out), int(dagger))
    return out


def schur_rhs(p: Params, U, b5) -> np.ndarray:
    U = _c128(U)
    b = _c128(b5)
    out = np.empty((p.Ls, p.Vh, 4, 3), np.complex128)
    pc = p._c()
    _load().or_schur_rhs(ctypes.byref(pc), _ptr(U), _ptr(b), _ptr(out))
    return out


def reconstruct(p: Params, U, x_e, b5) -> np.ndarray:
    U = _c128(U)
    xe = _c128(x_e)
    b = _c128(b5)
    out = np.empty_like(b)
    pc = p._c()
    _load().or_reconstruct(ctypes.byref(pc), _ptr(U), _ptr(xe), _ptr(b), _ptr(out))
    return out


def cgnr_even(p: Params, U, bt_e, tol: float, maxiter: int = 100000):
    U = _c128(U)
    b = _c128(bt_e)
    x = np.empty_like(b)
    pc = p._c()
    it = _load().or_cgnr_even(ctypes.byref(pc), _ptr(U), _ptr(b), _ptr(x), float(tol), int(maxiter))
    return x, it


def solve(p: Params, U, b5, tol: float = 1e-13, maxiter: int = 100000):
    """x5 = D^(alpha)^-1 b5 in FP64; returns (x5, iterations, true relative residual)."""
    U = _c128(U)
    b = _c128(b5)
    x = np.empty_like(b)
    tr = ctypes.c_double(0.0)
    pc = p._c()
    it = _load().or_solve(ctypes.byref(pc), _ptr(U), _ptr(b), _ptr(x), float(tol), int(maxiter),
                          ctypes.byref(tr))
    return x, it, tr.value


def source_4d(p: Params, U, b4) -> np.ndarray:
    U = _c128(U)
    b = _c128(b4)
    out = np.empty((p.Ls,) + b.shape, np.complex128)
    pc = p._c()
    _load().or_source_4d(ctypes.byref(pc), _ptr(U), _ptr(b), _ptr(out))
    return out


def project_4d(p: Params, x5) -> np.ndarray:
    x = _c128(x5)
    out = np.empty(x.shape[1:], np.complex128)
    pc = p._c()
    _load().or_project_4d(ctypes.byref(pc), _ptr(x), _ptr(out))
    return out


def residual_4d(p: Params, U, x4, b4, tol_inner: float = 1e-13) -> float:
    U = _c128(U)
    x = _c128(x4)
    b = _c128(b4)
    pc = p._c()
    return _load().or_residual_4d(ctypes.byref(pc), _ptr(U), _ptr(x), _ptr(b), float(tol_inner))


def true_residual(p: Params, U, x5, b5) -> float:
    U = _c128(U)
    x = _c128(x5)
    b = _c128(b5)
    pc = p._c()
    return _load().or_true_residual(ctypes.byref(pc), _ptr(U), _ptr(x), _ptr(b))


def to_even(p: Params, v5) -> np.ndarray:
    """Gather the parity-0 sites of a full 5D vector into the even layout."""
    par, _, le, _ = site_maps(p.dims)
    return np.ascontiguousarray(np.asarray(v5)[:, le])


def to_odd(p: Params, v5) -> np.ndarray:
    _, _, _, lo = site_maps(p.dims)
    return np.ascontiguousarray(np.asarray(v5)[:, lo])
