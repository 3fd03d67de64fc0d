"""ctypes marshalling for the C oracle (test infrastructure only).

No arithmetic of the method is done here: every number comes from
``tpl_oracle.c``.  Arrays use the canonical layouts of ``tpl_oracle.h``:
XS[9][ny][nx], XP[25][nqd][ny][nx], psi[nqd][ny][nx], U[2][ny][nx].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpl_oracle.c")
_LIB = os.path.join(_HERE, "libtpl_oracle.so")


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over lattice rows, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nq", C.c_int), ("periods", C.c_int),
                ("Re", C.c_double), ("Wi", C.c_double), ("beta", C.c_double),
                ("u0", C.c_double), ("phi", C.c_double), ("spring", C.c_int),
                ("b", C.c_double), ("tau_drag", C.c_double), ("tau_ratio_p", C.c_double),
                ("force_scale", C.c_double), ("lambda_set", C.c_double),
                ("ny_param", C.c_int), ("y_offset", C.c_int), ("x_offset", C.c_int),
                ("nx_param", C.c_int), ("drift_cap", C.c_double), ("drift_relax", C.c_double),
                ("qe_model", C.c_int), ("gradients", C.c_int), ("spring_shift", C.c_int)]


_DERIVED = ["kf", "l", "nu", "nuS", "lambda", "G", "tau1S", "tau2S", "tau1P", "tau2P",
            "R", "sigma", "DQ", "F0", "kappa", "meq", "rhoS0", "rhoP0", "Sc"]


class _Derived(C.Structure):
    _fields_ = [(n, C.c_double) for n in _DERIVED]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        ip = P(C.c_int)
        lib.orc_new.restype = C.c_void_p
        lib.orc_new.argtypes = [P(_Config), C.c_char_p]
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_nqd.restype = C.c_int
        lib.orc_nqd.argtypes = [C.c_void_p]
        lib.orc_get_derived.argtypes = [C.c_void_p, P(_Derived)]
        lib.orc_get_tables.argtypes = [C.c_void_p, ip, dp, ip, dp, dp, dp, ip, ip, dp]
        lib.orc_rest.argtypes = [C.c_void_p]
        lib.orc_base_state.argtypes = [C.c_void_p, C.c_long]
        lib.orc_analytic_state.restype = C.c_int
        lib.orc_analytic_state.argtypes = [C.c_void_p]
        lib.orc_default_prerun.restype = C.c_long
        lib.orc_default_prerun.argtypes = [C.c_void_p]
        lib.orc_perturb.argtypes = [C.c_void_p, C.c_uint64, C.c_double, C.c_int]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_step_count.restype = C.c_long
        lib.orc_step_count.argtypes = [C.c_void_p]
        lib.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        lib.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp]
        lib.orc_observables.argtypes = [C.c_void_p, dp]
        lib.orc_set_source.argtypes = [C.c_void_p, dp]
        lib.orc_set_source.restype = None
        lib.orc_amplitude.restype = C.c_double
        lib.orc_amplitude.argtypes = [C.c_void_p]
        lib.orc_diagnostics.argtypes = [C.c_void_p, dp]
        lib.orc_solvent_eq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        lib.orc_polymer_eq.argtypes = [C.c_void_p, C.c_double, dp, dp, dp]
        lib.orc_solvent_qe2.argtypes = [C.c_double, dp, dp, dp]
        lib.orc_polymer_qe2.argtypes = [C.c_void_p, C.c_double, dp, dp, dp]
        lib.orc_collide_node.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_spring_terms.argtypes = [C.c_void_p, C.c_int, C.c_int, dp]
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_max_threads.restype = C.c_int
        lib.orc_max_threads.argtypes = []
        lib.orc_splitmix64_next.restype = C.c_uint64
        lib.orc_splitmix64_next.argtypes = [P(C.c_uint64)]
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's row loops (OpenMP)."""
    _L().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_L().orc_max_threads())


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def splitmix64_next(state: int):
    st = C.c_uint64(state)
    z = _L().orc_splitmix64_next(C.byref(st))
    return int(st.value), int(z)


DEFAULTS = dict(nq=16, periods=1, Re=20.0, Wi=0.5, beta=0.8, u0=0.05, phi=0.01,
                spring=0, b=25.0, tau_drag=0.0, tau_ratio_p=1.0, force_scale=1.0,
                lambda_set=0.0, ny_param=0, y_offset=0, x_offset=0, nx_param=0, drift_cap=0.2,
                drift_relax=1.0, qe_model=1, gradients=0, spring_shift=0)

DIAG_NAMES = ["step", "mass_S", "mass_P", "mom_x", "mom_y", "amplitude",
              "enstrophy", "qrms", "min_psi"]


class OracleSim:
    """One oracle lattice.  Keyword arguments override ``DEFAULTS``."""

    def __init__(self, nx: int, ny: int, **kw):
        cfg = dict(DEFAULTS)
        unknown = set(kw) - set(cfg)
        if unknown:
            raise KeyError(f"unknown oracle options {sorted(unknown)}")
        cfg.update(kw)
        self.cfg = dict(cfg, nx=nx, ny=ny)
        c = _Config(**{k: self.cfg[k] for k, _ in _Config._fields_})
        err = C.create_string_buffer(256)
        h = _L().orc_new(C.byref(c), err)
        if not h:
            raise ValueError(err.value.decode())
        self._h = C.c_void_p(h)
        self.nx, self.ny = nx, ny
        self.nqd = _L().orc_nqd(self._h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # -- parameters and tables -------------------------------------------------
    def derived(self) -> dict:
        d = _Derived()
        _L().orc_get_derived(self._h, C.byref(d))
        return {n: getattr(d, n) for n in _DERIVED}

    def tables(self) -> dict:
        nqd = self.nqd
        cS = np.zeros(18, np.int32); wS = np.zeros(9); cP = np.zeros(100, np.int32)
        wP = np.zeros(25); Q = np.zeros(2 * nqd); Fh = np.zeros(2 * nqd)
        nbr = np.zeros(25 * nqd, np.int32); ks = np.zeros(25, np.int32); peq = np.zeros(nqd)
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))  # noqa: E731
        _L().orc_get_tables(self._h, ip(cS), _ptr(wS), ip(cP), _ptr(wP), _ptr(Q), _ptr(Fh),
                            ip(nbr), ip(ks), _ptr(peq))
        return dict(cS=cS.reshape(9, 2), wS=wS, cP=cP.reshape(25, 4), wP=wP,
                    Q=Q.reshape(nqd, 2), Fhat=Fh.reshape(nqd, 2),
                    nbrQ=nbr.reshape(25, nqd), kstar=ks, peq=peq)

    # -- initial states --------------------------------------------------------
    def rest(self):
        _L().orc_rest(self._h)

    def base_state(self, npre: int = -1):
        _L().orc_base_state(self._h, int(npre))

    def analytic_state(self):
        """Hookean laminar Kolmogorov state in closed form (model 1, Wi > 0)."""
        if _L().orc_analytic_state(self._h) != 0:
            raise ValueError("the analytic state needs Hookean springs, qe_model 1 and Wi > 0")

    def default_prerun(self) -> int:
        return int(_L().orc_default_prerun(self._h))

    def perturb(self, seed: int, amp: float, multimode: bool):
        _L().orc_perturb(self._h, C.c_uint64(seed), float(amp), int(bool(multimode)))

    # -- time stepping ---------------------------------------------------------
    def step(self, n: int = 1):
        _L().orc_step(self._h, int(n))

    @property
    def step_count(self) -> int:
        return int(_L().orc_step_count(self._h))

    # -- state exchange --------------------------------------------------------
    def get_state(self):
        N = self.nx * self.ny
        XS = np.zeros((9, self.ny, self.nx)); XP = np.zeros((25, self.nqd, self.ny, self.nx))
        psi = np.zeros((self.nqd, self.ny, self.nx)); U = np.zeros((2, self.ny, self.nx))
        assert XS.size == 9 * N
        _L().orc_get_state(self._h, _ptr(XS), _ptr(XP), _ptr(psi), _ptr(U))
        return dict(XS=XS, XP=XP, psi=psi, U=U)

    def set_state(self, XS=None, XP=None, psi=None, U=None):
        def chk(a, shape):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            assert a.shape == shape, (a.shape, shape)
            return a
        XS = chk(XS, (9, self.ny, self.nx)); XP = chk(XP, (25, self.nqd, self.ny, self.nx))
        psi = chk(psi, (self.nqd, self.ny, self.nx)); U = chk(U, (2, self.ny, self.nx))
        _L().orc_set_state(self._h, _ptr(XS), _ptr(XP), _ptr(psi), _ptr(U))

    # -- observables -----------------------------------------------------------
    def observables(self) -> np.ndarray:
        out = np.zeros((10, self.ny, self.nx))
        _L().orc_observables(self._h, _ptr(out))
        return out

    def spring_terms(self, x: int, y: int) -> np.ndarray:
        """Spring terms [nqd][2] of J^r_eq at node (x, y) from the recorded psi."""
        out = np.zeros((self.nqd, 2))
        _L().orc_spring_terms(self._h, int(x), int(y), _ptr(out))
        return out

    def set_source(self, F=None):
        """Extra body force F[2][ny][nx] added in every later step (None: off)."""
        if F is None:
            _L().orc_set_source(self._h, None)
            return
        F = np.ascontiguousarray(F, dtype=np.float64)
        assert F.shape == (2, self.ny, self.nx), F.shape
        _L().orc_set_source(self._h, _ptr(F))

    def amplitude(self) -> float:
        return float(_L().orc_amplitude(self._h))

    def diagnostics(self) -> dict:
        out = np.zeros(9)
        _L().orc_diagnostics(self._h, _ptr(out))
        return dict(zip(DIAG_NAMES, out.tolist()))

    # -- single-node pieces (pins) ----------------------------------------------
    @staticmethod
    def solvent_eq(rho, ux, uy):
        out = np.zeros(9)
        _L().orc_solvent_eq(float(rho), float(ux), float(uy), _ptr(out))
        return out

    def polymer_eq(self, psi, Jr, JQ):
        out = np.zeros(25)
        Jr = np.ascontiguousarray(Jr, dtype=np.float64); JQ = np.ascontiguousarray(JQ, dtype=np.float64)
        _L().orc_polymer_eq(self._h, float(psi), _ptr(Jr), _ptr(JQ), _ptr(out))
        return out

    @staticmethod
    def solvent_qe2(rho, J, P):
        """Stress-model quasi-equilibrium on D2Q9, P = (xx, xy, yy)."""
        out = np.zeros(9)
        J = np.ascontiguousarray(J, dtype=np.float64); P = np.ascontiguousarray(P, dtype=np.float64)
        _L().orc_solvent_qe2(float(rho), _ptr(J), _ptr(P), _ptr(out))
        return out

    def polymer_qe2(self, psi, J, P):
        """Stress-model quasi-equilibrium on D4Q25, J[4], P = upper triangle
        of the 4 x 4 second moment, row-major."""
        out = np.zeros(25)
        J = np.ascontiguousarray(J, dtype=np.float64); P = np.ascontiguousarray(P, dtype=np.float64)
        _L().orc_polymer_qe2(self._h, float(psi), _ptr(J), _ptr(P), _ptr(out))
        return out

    def collide_node(self, gS, gP, K, sq, Fb):
        gS = np.ascontiguousarray(gS, dtype=np.float64)
        gP = np.ascontiguousarray(gP, dtype=np.float64)
        assert gP.shape == (self.nqd, 25)
        K = np.ascontiguousarray(K, dtype=np.float64).reshape(4)
        sq = np.ascontiguousarray(sq, dtype=np.float64).reshape(self.nqd, 2)
        Fb = np.ascontiguousarray(Fb, dtype=np.float64).reshape(2)
        oS = np.zeros(9); oP = np.zeros((self.nqd, 25)); U = np.zeros(2)
        _L().orc_collide_node(self._h, _ptr(gS), _ptr(gP), _ptr(K), _ptr(sq), _ptr(Fb),
                              _ptr(oS), _ptr(oP), _ptr(U))
        return oS, oP, U
