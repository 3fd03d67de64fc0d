"""ctypes binding of libtpl (include/tpl.h).  Argument marshalling only.

Functions keep the C names (``tpl_create``, ``tpl_step``, ...); the ``Tpl``
class owns one context and turns negative return codes into ``TplError``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "libtpl.so")

TPL_OK, TPL_EINVAL, TPL_ENOMEM, TPL_EHIP, TPL_ESTATE, TPL_EUNSTABLE, TPL_EREJECTED = (
    0, -1, -2, -3, -4, -5, -6)
TPL_FP64, TPL_FP32, TPL_BF16 = 0, 1, 2
TPL_SOLVENT, TPL_POLYMER = 0, 1
TPL_NFIELDS = 10
FIELD_NAMES = ["rho", "Ux", "Uy", "rhoP", "Cxx", "Cxy", "Cyy", "tau_xx", "tau_xy", "tau_yy"]
DIAG_NAMES = ["step", "mass_S", "mass_P", "mom_x", "mom_y", "amplitude", "enstrophy",
              "qrms", "min_psi"]
_CODES = {TPL_EINVAL: "EINVAL", TPL_ENOMEM: "ENOMEM", TPL_EHIP: "EHIP", TPL_ESTATE: "ESTATE",
          TPL_EUNSTABLE: "EUNSTABLE", TPL_EREJECTED: "EREJECTED"}


class TplError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class tpl_forcing(C.Structure):
    _fields_ = [("periods", C.c_int), ("u0", C.c_double)]


class tpl_diag(C.Structure):
    _fields_ = [(n, C.c_double) for n in DIAG_NAMES]


class tpl_instance(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("periods", C.c_int), ("Re", C.c_double),
                ("Wi", C.c_double), ("beta", C.c_double), ("u0", C.c_double),
                ("seed", C.c_uint64), ("perturbation", C.c_double)]

INSTANCE_KEYS = ("nx", "ny", "periods", "Re", "Wi", "beta", "u0", "seed", "perturbation")


_lib = None


def lib_path() -> str:
    return _LIB


def lib():
    """Load libtpl.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise ImportError(f"{_LIB} not built: run python -c 'import __graft_entry__ as g; g.build()'")
    L = C.CDLL(_LIB)
    vp, dp, cp = C.c_void_p, C.POINTER(C.c_double), C.c_char_p
    fp = C.POINTER(C.c_float)
    sig = {
        "tpl_create": (vp, [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, tpl_forcing]),
        "tpl_set_param": (C.c_int, [vp, cp, C.c_double]),
        "tpl_query": (C.c_int, [vp, cp, dp]),
        "tpl_set_stream": (C.c_int, [vp, vp]),
        "tpl_adopt_buffers": (C.c_int, [vp, C.POINTER(vp), C.POINTER(C.c_size_t), C.c_int]),
        "tpl_init": (C.c_int, [vp, C.c_uint64, C.c_double]),
        "tpl_step": (C.c_int, [vp, C.c_int64]),
        "tpl_moments": (C.c_int, [vp, dp, C.c_size_t]),
        "tpl_moments_device": (C.c_int, [vp, vp, C.c_size_t]),
        "tpl_perturbation_amplitude": (C.c_double, [vp]),
        "tpl_diagnostics": (C.c_int, [vp, C.POINTER(tpl_diag)]),
        "tpl_diagnostics_noalloc": (C.c_int, [vp, C.POINTER(tpl_diag)]),
        "tpl_get_state": (C.c_int, [vp, dp, dp, dp, dp]),
        "tpl_set_state": (C.c_int, [vp, dp, dp, dp, dp]),
        "tpl_get_window": (C.c_int, [vp, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp]),
        "tpl_get_populations": (C.c_int, [vp, C.c_int, vp, C.c_size_t]),
        "tpl_set_populations": (C.c_int, [vp, C.c_int, vp, C.c_size_t]),
        "tpl_save": (C.c_int, [vp, cp]),
        "tpl_load": (C.c_int, [vp, cp]),
        "tpl_destroy": (None, [vp]),
        "tpl_last_error": (cp, []),
        "tpl_batch_create": (vp, [C.POINTER(tpl_instance), C.c_int, C.c_int]),
        "tpl_batch_set_param": (C.c_int, [vp, cp, C.c_double]),
        "tpl_batch_query": (C.c_int, [vp, cp, dp]),
        "tpl_batch_set_stream": (C.c_int, [vp, vp]),
        "tpl_batch_init": (C.c_int, [vp]),
        "tpl_batch_step": (C.c_int, [vp, C.c_int64]),
        "tpl_batch_amplitudes": (C.c_int, [vp, dp, C.c_int]),
        "tpl_batch_status": (C.c_int, [vp, C.POINTER(C.c_int), C.c_int]),
        "tpl_batch_instance": (vp, [vp, C.c_int]),
        "tpl_batch_destroy": (None, [vp]),
        "tpl_mlp_create": (vp, [C.c_int, C.c_int, C.c_int, C.c_uint64]),
        "tpl_mlp_set_stream": (C.c_int, [vp, vp]),
        "tpl_mlp_query": (C.c_int, [vp, cp, dp]),
        "tpl_mlp_get_params": (C.c_int, [vp, fp, C.c_size_t]),
        "tpl_mlp_set_params": (C.c_int, [vp, fp, C.c_size_t]),
        "tpl_mlp_set_norm": (C.c_int, [vp, fp, fp, fp, fp]),
        "tpl_mlp_forward": (C.c_int, [vp, vp, vp, C.c_int64]),
        "tpl_mlp_grads": (C.c_int, [vp, vp, vp, C.c_int64, fp, fp]),
        "tpl_mlp_train_step": (C.c_int, [vp, vp, vp, C.c_int64, C.c_float, fp]),
        "tpl_mlp_destroy": (None, [vp]),
        "tpl_restrict": (C.c_int, [vp, vp]),
        "tpl_features": (C.c_int, [vp, vp, C.c_size_t]),
        "tpl_targets": (C.c_int, [vp, vp, vp, C.c_size_t]),
        "tpl_set_source": (C.c_int, [vp, dp, C.c_size_t]),
        "tpl_get_source": (C.c_int, [vp, dp, C.c_size_t]),
        "tpl_attach_mlp": (C.c_int, [vp, vp, C.c_double]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def tpl_last_error() -> str:
    return lib().tpl_last_error().decode()


def _check(rc):
    if rc != TPL_OK:
        raise TplError(rc, tpl_last_error())


def _dptr(a):
    if a is None:
        return None
    if not (a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]):
        raise TypeError("expected a C-contiguous float64 array")
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Tpl:
    """One lattice context (tpl_create ... tpl_destroy)."""

    def __init__(self, nx, ny, Re, Wi, beta, periods=1, u0=0.05, **params):
        L = lib()
        h = L.tpl_create(int(nx), int(ny), float(Re), float(Wi), float(beta),
                         tpl_forcing(int(periods), float(u0)))
        if not h:
            raise TplError(TPL_EINVAL, tpl_last_error())
        self._h = C.c_void_p(h)
        self.nx, self.ny = int(nx), int(ny)
        for k, v in params.items():
            self.set_param(k, v)

    @classmethod
    def _borrow(cls, handle, nx, ny, owner):
        """A view of a context owned by someone else (a batch instance)."""
        t = cls.__new__(cls)
        t._h, t.nx, t.ny, t._owner = C.c_void_p(handle), int(nx), int(ny), owner
        return t

    def close(self):
        if getattr(self, "_h", None) is not None:
            if getattr(self, "_owner", None) is None:
                lib().tpl_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- configuration -----------------------------------------------------------------
    def set_param(self, key, value):
        _check(lib().tpl_set_param(self._h, key.encode(), float(value)))

    def query(self, key) -> float:
        out = C.c_double()
        _check(lib().tpl_query(self._h, key.encode(), C.byref(out)))
        return out.value

    @property
    def nqd(self) -> int:
        return int(self.query("nqd"))

    def set_stream(self, stream_ptr: int):
        _check(lib().tpl_set_stream(self._h, C.c_void_p(stream_ptr)))

    def adopt_buffers(self, ptrs, sizes):
        arr = (C.c_void_p * len(ptrs))(*[C.c_void_p(p) for p in ptrs])
        sz = (C.c_size_t * len(sizes))(*sizes)
        _check(lib().tpl_adopt_buffers(self._h, arr, sz, len(ptrs)))

    # -- time stepping -----------------------------------------------------------------
    def init(self, seed=0, perturbation=0.0):
        _check(lib().tpl_init(self._h, C.c_uint64(seed), float(perturbation)))

    def step(self, n=1):
        _check(lib().tpl_step(self._h, int(n)))

    # -- outputs -----------------------------------------------------------------------
    def moments(self) -> np.ndarray:
        out = np.zeros((TPL_NFIELDS, self.ny, self.nx))
        _check(lib().tpl_moments(self._h, _dptr(out), out.size))
        return out

    def moments_device(self, dptr: int, length: int):
        _check(lib().tpl_moments_device(self._h, C.c_void_p(dptr), int(length)))

    def amplitude(self) -> float:
        v = lib().tpl_perturbation_amplitude(self._h)
        if v != v:
            raise TplError(TPL_EHIP, tpl_last_error())
        return v

    def diagnostics(self) -> dict:
        d = tpl_diag()
        _check(lib().tpl_diagnostics(self._h, C.byref(d)))
        return {n: getattr(d, n) for n in DIAG_NAMES}

    def diagnostics_noalloc(self) -> dict:
        """tpl_diagnostics_noalloc: the same values, computed in the
        library's static working memory (no device allocation)."""
        d = tpl_diag()
        _check(lib().tpl_diagnostics_noalloc(self._h, C.byref(d)))
        return {n: getattr(d, n) for n in DIAG_NAMES}

    def get_state(self, populations=True):
        """XS, XP, psi, U as FP64 arrays; populations=False skips XS and XP
        (those need the plain population order that in-place streaming holds
        after an even number of steps)."""
        nqd = self.nqd
        psi = np.zeros((nqd, self.ny, self.nx)); U = np.zeros((2, self.ny, self.nx))
        if not populations:
            _check(lib().tpl_get_state(self._h, None, None, _dptr(psi), _dptr(U)))
            return dict(psi=psi, U=U)
        XS = np.zeros((9, self.ny, self.nx)); XP = np.zeros((25, nqd, self.ny, self.nx))
        _check(lib().tpl_get_state(self._h, _dptr(XS), _dptr(XP), _dptr(psi), _dptr(U)))
        return dict(XS=XS, XP=XP, psi=psi, U=U)

    def set_state(self, XS=None, XP=None, psi=None, U=None):
        nqd = self.nqd
        shapes = dict(XS=(9, self.ny, self.nx), XP=(25, nqd, self.ny, self.nx),
                      psi=(nqd, self.ny, self.nx), U=(2, self.ny, self.nx))
        arrs = {}
        for k, a in dict(XS=XS, XP=XP, psi=psi, U=U).items():
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != shapes[k]:
                    raise ValueError(f"{k}: shape {a.shape} != {shapes[k]}")
            arrs[k] = a
        _check(lib().tpl_set_state(self._h, *[_dptr(arrs[k]) for k in ("XS", "XP", "psi", "U")]))

    def get_window(self, x0, y0, w, h):
        nqd = self.nqd
        XS = np.zeros((9, h, w)); XP = np.zeros((25, nqd, h, w))
        psi = np.zeros((nqd, h, w)); U = np.zeros((2, h, w))
        _check(lib().tpl_get_window(self._h, int(x0), int(y0), int(w), int(h), _dptr(XS),
                                    _dptr(XP), _dptr(psi), _dptr(U)))
        return dict(XS=XS, XP=XP, psi=psi, U=U)

    # -- learned correction ------------------------------------------------------------
    def restrict_from(self, fine: "Tpl"):
        """This (coarse) state := restriction of the fine context's state."""
        _check(lib().tpl_restrict(fine._h, self._h))

    def features_device(self, dptr: int, length: int):
        _check(lib().tpl_features(self._h, C.c_void_p(dptr), int(length)))

    def targets_device(self, obs_ref_dptr: int, dptr: int, length: int):
        _check(lib().tpl_targets(self._h, C.c_void_p(obs_ref_dptr), C.c_void_p(dptr), int(length)))

    def set_source(self, F=None):
        if F is None:
            _check(lib().tpl_set_source(self._h, None, 0))
            return
        F = np.ascontiguousarray(F, dtype=np.float64)
        if F.shape != (2, self.ny, self.nx):
            raise ValueError(f"source shape {F.shape} != {(2, self.ny, self.nx)}")
        _check(lib().tpl_set_source(self._h, _dptr(F), F.size))

    def get_source(self) -> np.ndarray:
        F = np.zeros((2, self.ny, self.nx))
        _check(lib().tpl_get_source(self._h, _dptr(F), F.size))
        return F

    def attach(self, mlp, drift_bound=0.0):
        _check(lib().tpl_attach_mlp(self._h, None if mlp is None else mlp._h, float(drift_bound)))
        self._mlp = mlp  # keep the network alive while attached

    def save(self, path):
        _check(lib().tpl_save(self._h, os.fspath(path).encode()))

    def load(self, path):
        _check(lib().tpl_load(self._h, os.fspath(path).encode()))


class Batch:
    """Many instances advanced together (tpl_batch_create ... tpl_batch_destroy).

    instances: sequence of dicts with the tpl_instance fields (nx, ny, Re,
    Wi, beta; periods 1, u0 0.05, seed 0, perturbation 0 by default)."""

    def __init__(self, instances, precision=TPL_FP64, **params):
        L = lib()
        n = len(instances)
        arr = (tpl_instance * n)()
        for i, d in enumerate(instances):
            full = {**dict(periods=1, u0=0.05, seed=0, perturbation=0.0), **d}
            for k in INSTANCE_KEYS:
                setattr(arr[i], k, full[k])
        h = L.tpl_batch_create(arr, n, int(precision))
        if not h:
            raise TplError(TPL_EINVAL, tpl_last_error())
        self._h = C.c_void_p(h)
        self.n = n
        self.sizes = [(int(d["nx"]), int(d["ny"])) for d in instances]
        for k, v in params.items():
            self.set_param(k, v)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().tpl_batch_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_param(self, key, value):
        _check(lib().tpl_batch_set_param(self._h, key.encode(), float(value)))

    def query(self, key) -> float:
        out = C.c_double()
        _check(lib().tpl_batch_query(self._h, key.encode(), C.byref(out)))
        return out.value

    def set_stream(self, stream_ptr: int):
        _check(lib().tpl_batch_set_stream(self._h, C.c_void_p(stream_ptr)))

    def init(self):
        _check(lib().tpl_batch_init(self._h))

    def step(self, n=1):
        _check(lib().tpl_batch_step(self._h, int(n)))

    def amplitudes(self) -> np.ndarray:
        out = np.zeros(self.n)
        _check(lib().tpl_batch_amplitudes(self._h, _dptr(out), self.n))
        return out

    def status(self) -> np.ndarray:
        out = (C.c_int * self.n)()
        _check(lib().tpl_batch_status(self._h, out, self.n))
        return np.array(out[:], dtype=np.int32)

    def instance(self, i) -> Tpl:
        h = lib().tpl_batch_instance(self._h, int(i))
        if not h:
            raise TplError(TPL_EINVAL, tpl_last_error())
        nx, ny = self.sizes[i]
        return Tpl._borrow(h, nx, ny, self)


def _fptr(a):
    if not (a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]):
        raise TypeError("expected a C-contiguous float32 array")
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Mlp:
    """Correction network (tpl_mlp_create ... tpl_mlp_destroy).  Inputs and
    targets of forward/grads/train_step are device pointers (FP32, e.g. from
    torch tensors)."""

    def __init__(self, n_in=54, hidden=64, n_out=5, seed=0):
        h = lib().tpl_mlp_create(int(n_in), int(hidden), int(n_out), C.c_uint64(seed))
        if not h:
            raise TplError(TPL_EINVAL, tpl_last_error())
        self._h = C.c_void_p(h)
        self.n_in, self.hidden, self.n_out = int(n_in), int(hidden), int(n_out)
        self.nparams = int(self.query("nparams"))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().tpl_mlp_destroy(self._h)
            self._h = None

    __del__ = close

    def query(self, key) -> float:
        out = C.c_double()
        _check(lib().tpl_mlp_query(self._h, key.encode(), C.byref(out)))
        return out.value

    def set_stream(self, stream_ptr: int):
        _check(lib().tpl_mlp_set_stream(self._h, C.c_void_p(stream_ptr)))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.nparams, dtype=np.float32)
        _check(lib().tpl_mlp_get_params(self._h, _fptr(out), out.size))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        _check(lib().tpl_mlp_set_params(self._h, _fptr(theta), theta.size))

    def set_norm(self, in_mean, in_std, out_mean, out_std):
        a = [np.ascontiguousarray(v, dtype=np.float32) for v in (in_mean, in_std, out_mean, out_std)]
        _check(lib().tpl_mlp_set_norm(self._h, *[_fptr(v) for v in a]))

    def forward(self, X_dptr: int, Y_dptr: int, n: int):
        _check(lib().tpl_mlp_forward(self._h, C.c_void_p(X_dptr), C.c_void_p(Y_dptr), int(n)))

    def grads(self, X_dptr: int, T_dptr: int, n: int):
        dW = np.zeros(self.nparams, dtype=np.float32)
        loss = C.c_float()
        _check(lib().tpl_mlp_grads(self._h, C.c_void_p(X_dptr), C.c_void_p(T_dptr), int(n),
                                   _fptr(dW), C.byref(loss)))
        return dW, loss.value

    def train_step(self, X_dptr: int, T_dptr: int, n: int, lr: float = 1e-3) -> float:
        loss = C.c_float()
        _check(lib().tpl_mlp_train_step(self._h, C.c_void_p(X_dptr), C.c_void_p(T_dptr), int(n),
                                        C.c_float(lr), C.byref(loss)))
        return loss.value
