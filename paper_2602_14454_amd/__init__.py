"""Python binding of libdwf, the MI355X domain-wall fermion solver.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libdwf.so`` (built by ``paper_2602_14454_amd.build``).  PyTorch
is used for device memory and streams; vectors are complex128 CUDA/HIP
tensors in the canonical layouts documented in ``include/dwf.h``.

There is no CPU fallback: importing the binding without the built library,
or calling it without a HIP device, raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

__all__ = [
    "load", "DwfError", "SolveParams", "SolveInfo", "Lattice", "Op",
    "F64", "F32", "BF16", "FULL5D", "EVEN5D", "ALGO_CGNR", "ALGO_DC", "ALGO_FGCR_LEARNED", "ALGO_MIXED",
    "solve_batch", "autotune_batch", "tune_cache_put", "tune_cache_get", "tune_cache_reload",
    "PtcModel", "PtcPairs", "gauge_sweeps", "gauge_plaquette",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# DWF_LIB selects another build of the same library (kernel-variant tuning).
LIB_PATH = os.environ.get("DWF_LIB") or os.path.join(_HERE, "libdwf.so")

F64, F32, BF16 = 0, 1, 2
FULL5D, EVEN5D = 0, 1
ALGO_CGNR, ALGO_DC, ALGO_FGCR_LEARNED, ALGO_MIXED = 0, 1, 2, 3
OK, NOT_CONVERGED = 0, 1


class DwfError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status} ({msg})")
        self.status = status


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("algo", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("check_every", ctypes.c_int), ("paper_mode", ctypes.c_int),
                ("ptc_model", ctypes.c_void_p), ("restart", ctypes.c_int),
                ("autotune", ctypes.c_int), ("use_graph", ctypes.c_int), ("schur", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("fallback_used", ctypes.c_int),
                ("converged", ctypes.c_int), ("true_res5", ctypes.c_double), ("seconds", ctypes.c_double),
                ("final_rel_res_even", ctypes.c_double), ("final_inner_prec", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# name -> (restype, argtypes)
_vp, _ip, _d, _i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_double, ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "dwf_solve_params_default": (None, [ctypes.POINTER(SolveParams)]),
    "dwf_lattice_create": (_i, [_ip, _i, ctypes.POINTER(_vp)]),
    "dwf_lattice_destroy": (None, [_vp]),
    "dwf_lattice_set_gauge": (_i, [_vp, _vp, _i, _vp]),
    "dwf_lattice_maps": (_i, [_vp, _vp, _vp]),
    "dwf_op_create": (_i, [_vp, _i, _d, _d, _d, _d, _d, ctypes.POINTER(_vp)]),
    "dwf_op_create_sdep": (_i, [_vp, _i, _d, _d, _dp, _dp, _d, ctypes.POINTER(_vp)]),
    "dwf_op_destroy": (None, [_vp]),
    "dwf_apply": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "dwf_apply_normal": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dwf_apply_eo5": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "dwf_source_4d": (_i, [_vp, _vp, _vp, _vp]),
    "dwf_cg_residual_update": (_i, [_vp, _i, _vp, _vp, _dp, _dp, _vp]),
    "dwf_apply_normal_noalloc": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dwf_project_4d": (_i, [_vp, _vp, _vp, _vp]),
    "dwf_solve": (_i, [_vp, _vp, _vp, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo), _vp]),
    "dwf_true_residual": (_i, [_vp, _vp, _vp, _dp, _vp]),
    "dwf_bench_hop": (_i, [_vp, _i, _i, _dp, _dp, _vp]),
    "dwf_residual_4d": (_i, [_vp, _vp, _vp, _d, _dp, _vp]),
    "dwf_lanczos_extremes": (_i, [_vp, _i, _i, _i, _d, _dp, _dp, _ip, _ip, _vp]),
    "dwf_solve_batch": (_i, [_i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _ip,
                             ctypes.POINTER(SolveParams), ctypes.POINTER(SolveInfo), _vp]),
    "dwf_autotune_batch": (_i, [_i, ctypes.POINTER(_vp), _ip, _i, _i, _ip, _ip, _dp, _vp]),
    "dwf_tune_cache_put": (_i, [ctypes.c_char_p, _i, _i, _d]),
    "dwf_tune_cache_get": (_i, [ctypes.c_char_p, _ip, _ip, _dp]),
    "dwf_tune_cache_reload": (_i, []),
    "dwf_ptc_create": (_i, [_i, ctypes.c_ulonglong, _d, ctypes.POINTER(_vp)]),
    "dwf_ptc_destroy": (None, [_vp]),
    "dwf_ptc_info": (_i, [_vp, _ip, _ip, _ip]),
    "dwf_ptc_set_loss": (_i, [_vp, _i]),
    "dwf_ptc_get_weights": (_i, [_vp, _vp]),
    "dwf_ptc_set_weights": (_i, [_vp, _vp]),
    "dwf_ptc_apply": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "dwf_ptc_gradient": (_i, [_vp, _vp, _vp, _vp, _dp, _vp, _vp]),
    "dwf_ptc_pairs_create": (_i, [_vp, _vp, ctypes.c_ulonglong, _i, _ip, ctypes.POINTER(_vp), _vp]),
    "dwf_ptc_pairs_get": (_i, [_vp, _i, _vp, _vp, _vp]),
    "dwf_ptc_pairs_destroy": (None, [_vp]),
    "dwf_ptc_train": (_i, [_vp, _i, ctypes.POINTER(_vp), _i, _d, ctypes.c_ulonglong, _dp, _vp]),
    "dwf_ptc_eval": (_i, [_vp, _i, ctypes.POINTER(_vp), _dp, _vp]),
    "dwf_ptc_save": (_i, [_vp, ctypes.c_char_p]),
    "dwf_ptc_load": (_i, [ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "dwf_bench_copy": (_i, [ctypes.c_size_t, _i, _dp, _vp]),
    "dwf_gauge_sweeps": (_i, [_ip, _vp, _d, _i, _i, ctypes.c_ulonglong, ctypes.c_longlong, _vp]),
    "dwf_gauge_plaquette": (_i, [_ip, _vp, _dp, _vp]),
    "dwf_ptc_bench_apply": (_i, [_vp, _vp, _i, _dp, _vp]),
    "dwf_status_string": (ctypes.c_char_p, [_i]),
    "dwf_last_error": (ctypes.c_char_p, []),
}


def _hip_runtimes_mapped() -> set:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def load():
    """Load libdwf.so (raises if it has not been built).

    torch is imported first so that libdwf binds to torch's HIP runtime; a
    process with two HIP runtimes mapped is refused.
    """
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run `python -m paper_2602_14454_amd.build`")
    import torch  # noqa: F401  (loads torch's libamdhip64 before libdwf)
    lib = ctypes.CDLL(LIB_PATH)
    rts = _hip_runtimes_mapped()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes mapped in this process: {sorted(rts)}")
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status < 0:
        lib = load()
        raise DwfError(status, where, lib.dwf_last_error().decode())
    return status


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def solve_batch(ops, x5s, b5s, nrhs, params=None, stream=None):
    """dwf_solve_batch: ops[i] with nrhs[i] right-hand sides stored back to
    back in x5s[i] / b5s[i].  Returns (status, [SolveInfo per slot])."""
    n = len(ops)
    if not (len(x5s) == len(b5s) == len(nrhs) == n):
        raise ValueError("ops, x5s, b5s and nrhs must have the same length")
    arr_ops = (ctypes.c_void_p * n)(*[o._h.value for o in ops])
    arr_x = (ctypes.c_void_p * n)(*[_dev_ptr(x) for x in x5s])
    arr_b = (ctypes.c_void_p * n)(*[_dev_ptr(b) for b in b5s])
    arr_n = (ctypes.c_int * n)(*[int(k) for k in nrhs])
    infos = (SolveInfo * sum(int(k) for k in nrhs))()
    p = params if params is not None else default_params(algo=ALGO_DC, check_every=8)
    st = _check(load().dwf_solve_batch(n, arr_ops, arr_x, arr_b, arr_n, ctypes.byref(p), infos,
                                       _stream(stream)), "dwf_solve_batch")
    return st, list(infos)


def autotune_batch(ops, nrhs, prec=None, force=False, stream=None):
    """(rhs_per_block, order, ms) chosen by the tile autotuner."""
    n = len(ops)
    arr_ops = (ctypes.c_void_p * n)(*[o._h.value for o in ops])
    arr_n = (ctypes.c_int * n)(*[int(k) for k in nrhs])
    a, b, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(load().dwf_autotune_batch(n, arr_ops, arr_n, int(F32 if prec is None else prec), int(bool(force)),
                                     ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms), _stream(stream)),
           "dwf_autotune_batch")
    return a.value, b.value, ms.value


class PtcModel:
    """dwf_ptc: the learned gauge-equivariant preconditioner."""

    def __init__(self, hidden: int = 8, seed: int = 1, init_scale: float = 0.05, _handle=None):
        lib = load()
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib.dwf_ptc_create(int(hidden), int(seed), float(init_scale), ctypes.byref(h)), "dwf_ptc_create")
            _handle = h
        self._h = _handle
        hid, nw, st = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.dwf_ptc_info(self._h, ctypes.byref(hid), ctypes.byref(nw), ctypes.byref(st)), "dwf_ptc_info")
        self.hidden, self.nweights = hid.value, nw.value

    def set_loss(self, kind: int) -> None:
        """0: |M r - e|^2/|e|^2 (error loss); 1: |A M r - r|^2/|r|^2 (residual loss)."""
        _check(load().dwf_ptc_set_loss(self._h, int(kind)), "dwf_ptc_set_loss")

    @classmethod
    def load_file(cls, path: str) -> "PtcModel":
        h = ctypes.c_void_p()
        _check(load().dwf_ptc_load(path.encode(), ctypes.byref(h)), "dwf_ptc_load")
        return cls(_handle=h)

    def save(self, path: str) -> None:
        _check(load().dwf_ptc_save(self._h, path.encode()), "dwf_ptc_save")

    @property
    def steps(self) -> int:
        st = ctypes.c_int()
        _check(load().dwf_ptc_info(self._h, None, None, ctypes.byref(st)), "dwf_ptc_info")
        return st.value

    def weights(self):
        """(W1 [11][H][1][4][4], W2 [11][1][H][4][4]) as complex64 numpy arrays."""
        import numpy as np
        w = np.empty(self.nweights, dtype=np.complex64)
        _check(load().dwf_ptc_get_weights(self._h, w.ctypes.data_as(ctypes.c_void_p)), "dwf_ptc_get_weights")
        half = self.nweights // 2
        return w[:half].reshape(11, self.hidden, 1, 4, 4), w[half:].reshape(11, 1, self.hidden, 4, 4)

    def set_weights(self, W1, W2) -> None:
        import numpy as np
        w = np.ascontiguousarray(np.concatenate([np.asarray(W1).reshape(-1), np.asarray(W2).reshape(-1)])
                                 .astype(np.complex64))
        if w.size != self.nweights:
            raise ValueError("weight count mismatch")
        _check(load().dwf_ptc_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p)), "dwf_ptc_set_weights")

    def apply(self, op, out_e, in_e, stream=None) -> None:
        _check(load().dwf_ptc_apply(self._h, op._h, _dev_ptr(out_e), _dev_ptr(in_e), _stream(stream)),
               "dwf_ptc_apply")

    def bench_apply(self, op, nrep=20, stream=None) -> float:
        """Mean time (ms) of one network application on op's lattice (HIP events)."""
        ms = ctypes.c_double()
        _check(load().dwf_ptc_bench_apply(self._h, op._h, int(nrep), ctypes.byref(ms), _stream(stream)),
               "dwf_ptc_bench_apply")
        return ms.value

    def gradient(self, op, r_e, e_e, stream=None):
        """(loss, (G1, G2)) with G = dL/dRe W + i dL/dIm W (complex64)."""
        import numpy as np
        g = np.empty(self.nweights, dtype=np.complex64)
        loss = ctypes.c_double()
        _check(load().dwf_ptc_gradient(self._h, op._h, _dev_ptr(r_e), _dev_ptr(e_e), ctypes.byref(loss),
                                       g.ctypes.data_as(ctypes.c_void_p), _stream(stream)), "dwf_ptc_gradient")
        half = self.nweights // 2
        return loss.value, (g[:half].reshape(11, self.hidden, 1, 4, 4), g[half:].reshape(11, 1, self.hidden, 4, 4))

    def train(self, pair_sets, steps: int, lr: float = 1e-3, seed: int = 7, stream=None):
        import numpy as np
        arr = (ctypes.c_void_p * len(pair_sets))(*[p._h.value for p in pair_sets])
        hist = np.zeros(max(int(steps), 1), dtype=np.float64)
        _check(load().dwf_ptc_train(self._h, len(pair_sets), arr, int(steps), float(lr), int(seed),
                                    hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)),
               "dwf_ptc_train")
        return hist[: int(steps)]

    def eval(self, pair_sets, stream=None) -> float:
        arr = (ctypes.c_void_p * len(pair_sets))(*[p._h.value for p in pair_sets])
        v = ctypes.c_double()
        _check(load().dwf_ptc_eval(self._h, len(pair_sets), arr, ctypes.byref(v), _stream(stream)), "dwf_ptc_eval")
        return v.value

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dwf_ptc_destroy(self._h)
                self._h = None
        except Exception:
            pass


class PtcPairs:
    """dwf_ptc_pairs: training pairs (r_k, e_k) of one operator, kept on the device."""

    def __init__(self, op, b5, snap_iters, seed: int = 0, stream=None):
        """b5: 5D source (device tensor), or None for a system with a seeded random solution."""
        arr = (ctypes.c_int * len(snap_iters))(*[int(k) for k in snap_iters])
        h = ctypes.c_void_p()
        src = _dev_ptr(b5) if b5 is not None else None
        _check(load().dwf_ptc_pairs_create(op._h, src, int(seed), len(snap_iters), arr, ctypes.byref(h),
                                           _stream(stream)), "dwf_ptc_pairs_create")
        self._h = h
        self.op = op          # keeps the operator (and its lattice) alive
        self.count = len(snap_iters)

    def get(self, k, r_out, e_out, stream=None):
        _check(load().dwf_ptc_pairs_get(self._h, int(k), _dev_ptr(r_out), _dev_ptr(e_out), _stream(stream)),
               "dwf_ptc_pairs_get")

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.dwf_ptc_pairs_destroy(self._h)
                self._h = None
        except Exception:
            pass


def tune_cache_put(key: str, nrb: int, order: int, ms: float) -> None:
    _check(load().dwf_tune_cache_put(key.encode(), int(nrb), int(order), float(ms)), "dwf_tune_cache_put")


def tune_cache_get(key: str):
    """(nrb, order, ms) or None."""
    a, b, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    st = _check(load().dwf_tune_cache_get(key.encode(), ctypes.byref(a), ctypes.byref(b), ctypes.byref(ms)),
                "dwf_tune_cache_get")
    return None if st != 0 else (a.value, b.value, ms.value)


def tune_cache_reload() -> None:
    _check(load().dwf_tune_cache_reload(), "dwf_tune_cache_reload")


def default_params(**kw) -> SolveParams:
    p = SolveParams()
    load().dwf_solve_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k == "inner_prec" and isinstance(v, str):
            v = {"f64": F64, "f32": F32, "bf16": BF16}[v]
        setattr(p, k, v)
    return p


class Lattice:
    """dwf_lattice: geometry, neighbour tables and device gauge copies."""

    def __init__(self, dims, antiperiodic_t: bool = True):
        lib = load()
        self.dims = tuple(int(d) for d in dims)
        arr = (ctypes.c_int * 4)(*self.dims)
        h = ctypes.c_void_p()
        _check(lib.dwf_lattice_create(arr, int(bool(antiperiodic_t)), ctypes.byref(h)), "dwf_lattice_create")
        self._h = h
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.Vh = self.V // 2

    def set_gauge(self, U, stream=None):
        """U: complex128 tensor (device) or numpy array (host), canonical [V][4][3][3]."""
        lib = load()
        import numpy as np
        if isinstance(U, np.ndarray):
            U = np.ascontiguousarray(U, dtype=np.complex128)
            _check(lib.dwf_lattice_set_gauge(self._h, U.ctypes.data_as(ctypes.c_void_p), 0, None),
                   "dwf_lattice_set_gauge")
        else:
            _check(lib.dwf_lattice_set_gauge(self._h, _dev_ptr(U), 1, _stream(stream)), "dwf_lattice_set_gauge")

    def maps(self):
        import numpy as np
        lex = np.zeros((2, self.Vh), np.int32)
        nbr = np.zeros((2, 8, self.Vh), np.int32)
        _check(load().dwf_lattice_maps(self._h, lex.ctypes.data_as(ctypes.c_void_p),
                                       nbr.ctypes.data_as(ctypes.c_void_p)), "dwf_lattice_maps")
        return lex, nbr

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dwf_lattice_destroy(self._h)
            self._h = None


@dataclass
class OpParams:
    Ls: int
    M0: float
    m: float
    b: float = 1.0
    c: float = 0.0
    alpha: float = 1.0


class Op:
    """dwf_op: D^(alpha) on a lattice (the lattice must outlive the op)."""

    def __init__(self, lattice: Lattice, Ls, M0, m, b=1.0, c=0.0, alpha=1.0):
        """b, c: numbers (s-independent) or sequences of Ls numbers (b_s, c_s, s = 0..Ls-1)."""
        lib = load()
        self.lattice = lattice
        self.params = OpParams(Ls, M0, m, b, c, alpha)
        h = ctypes.c_void_p()
        if isinstance(b, (int, float)) and isinstance(c, (int, float)):
            _check(lib.dwf_op_create(lattice._h, int(Ls), float(M0), float(m), float(b), float(c), float(alpha),
                                     ctypes.byref(h)), "dwf_op_create")
        else:
            bs = [float(v) for v in (b if not isinstance(b, (int, float)) else [b] * int(Ls))]
            cs = [float(v) for v in (c if not isinstance(c, (int, float)) else [c] * int(Ls))]
            if len(bs) != int(Ls) or len(cs) != int(Ls):
                raise ValueError("b and c need Ls entries")
            arr_b, arr_c = (ctypes.c_double * int(Ls))(*bs), (ctypes.c_double * int(Ls))(*cs)
            _check(lib.dwf_op_create_sdep(lattice._h, int(Ls), float(M0), float(m), arr_b, arr_c, float(alpha),
                                          ctypes.byref(h)), "dwf_op_create_sdep")
        self._h = h
        self.Ls = int(Ls)

    def apply(self, out, inp, space=FULL5D, dagger=False, prec=F64, stream=None):
        _check(load().dwf_apply(self._h, int(space), int(bool(dagger)), int(prec), _dev_ptr(out), _dev_ptr(inp),
                                _stream(stream)), "dwf_apply")
        return out

    def apply_normal(self, out, inp, prec=F64, stream=None):
        _check(load().dwf_apply_normal(self._h, int(prec), _dev_ptr(out), _dev_ptr(inp), _stream(stream)),
               "dwf_apply_normal")
        return out

    def apply_eo5(self, out5, in5, dagger=False, prec=F64, stream=None):
        """Schur operator of the split by 5D parity (or its adjoint) on the 5D-even entries of canonical 5D fields."""
        _check(load().dwf_apply_eo5(self._h, int(prec), int(bool(dagger)), _dev_ptr(out5), _dev_ptr(in5),
                                    _stream(stream)), "dwf_apply_eo5")
        return out5

    def apply_normal_noalloc(self, out, inp, prec=F64, stream=None):
        """D^dag D^ with the library's static scratch (no device allocation, no synchronisation)."""
        _check(load().dwf_apply_normal_noalloc(self._h, int(prec), _dev_ptr(out), _dev_ptr(inp), _stream(stream)),
               "dwf_apply_normal_noalloc")

    def cg_residual_update(self, r, p, prec=F64, stream=None):
        """r <- r - alpha D^dag D^ p with alpha = |r|^2 / |D^ p|^2; returns (alpha, |r_new|^2)."""
        a, rr = ctypes.c_double(), ctypes.c_double()
        _check(load().dwf_cg_residual_update(self._h, int(prec), _dev_ptr(r), _dev_ptr(p), ctypes.byref(a),
                                             ctypes.byref(rr), _stream(stream)), "dwf_cg_residual_update")
        return a.value, rr.value

    def source_4d(self, b5, b4, stream=None):
        _check(load().dwf_source_4d(self._h, _dev_ptr(b5), _dev_ptr(b4), _stream(stream)), "dwf_source_4d")
        return b5

    def project_4d(self, x4, x5, stream=None):
        _check(load().dwf_project_4d(self._h, _dev_ptr(x4), _dev_ptr(x5), _stream(stream)), "dwf_project_4d")
        return x4

    def solve(self, x5, b5, params: SolveParams | None = None, stream=None) -> tuple[int, SolveInfo]:
        info = SolveInfo()
        p = params if params is not None else default_params()
        st = _check(load().dwf_solve(self._h, _dev_ptr(x5), _dev_ptr(b5), ctypes.byref(p), ctypes.byref(info),
                                     _stream(stream)), "dwf_solve")
        return st, info

    def true_residual(self, x5, b5, stream=None) -> float:
        r = ctypes.c_double()
        _check(load().dwf_true_residual(self._h, _dev_ptr(x5), _dev_ptr(b5), ctypes.byref(r), _stream(stream)),
               "dwf_true_residual")
        return r.value

    def residual_4d(self, x4, b4, tol_inner=1e-13, stream=None) -> float:
        r = ctypes.c_double()
        st = load().dwf_residual_4d(self._h, _dev_ptr(x4), _dev_ptr(b4), float(tol_inner), ctypes.byref(r),
                                    _stream(stream))
        _check(st, "dwf_residual_4d")
        if st != 0:   # the inner m = 1 solve stopped short: the value is not a residual bound
            raise DwfError(st, "dwf_residual_4d", load().dwf_last_error().decode())
        return r.value

    def lanczos_extremes(self, basis=64, keep=24, max_restarts=50, tol=1e-10, stream=None):
        """(lambda_min, lambda_max, matvecs, converged) of D^dag D^."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        mv, cv = ctypes.c_int(), ctypes.c_int()
        _check(load().dwf_lanczos_extremes(self._h, int(basis), int(keep), int(max_restarts), float(tol),
                                           ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(mv), ctypes.byref(cv),
                                           _stream(stream)), "dwf_lanczos_extremes")
        return lo.value, hi.value, mv.value, bool(cv.value)

    def bench_hop(self, prec=F32, nrep=50, stream=None):
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(load().dwf_bench_hop(self._h, int(prec), int(nrep), ctypes.byref(ms), ctypes.byref(by),
                                    _stream(stream)), "dwf_bench_hop")
        return ms.value, by.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.dwf_op_destroy(self._h)
            self._h = None


def gauge_sweeps(U, dims, beta, nsweeps=1, n_or=0, seed=1, sweep0=0, stream=None):
    """dwf_gauge_sweeps on a canonical complex128 device tensor U (V, 4, 3, 3), in place."""
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    _check(load().dwf_gauge_sweeps(d, _dev_ptr(U), float(beta), int(nsweeps), int(n_or), int(seed), int(sweep0),
                                   _stream(stream)), "dwf_gauge_sweeps")
    return U


def gauge_plaquette(U, dims, stream=None) -> float:
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    v = ctypes.c_double()
    _check(load().dwf_gauge_plaquette(d, _dev_ptr(U), ctypes.byref(v), _stream(stream)), "dwf_gauge_plaquette")
    return v.value


def bench_copy(nbytes: int, nrep: int = 20, stream=None) -> float:
    """Mean time (ms) of a plain device copy of nbytes (counter calibration)."""
    ms = ctypes.c_double()
    _check(load().dwf_bench_copy(int(nbytes), int(nrep), ctypes.byref(ms), _stream(stream)), "dwf_bench_copy")
    return ms.value
