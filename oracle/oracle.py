"""ctypes shim over the FP64 CPU oracle (``lbddf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product package.

Parameters come as the plain dictionaries of
``paper_1109_6672_amd.workloads`` (an input description only); everything the
model derives from them (relaxation rates, equilibria, boundary values) is
computed inside the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbddf_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

_KIND = {"periodic": 0, "wall": 1, "adiabatic": 2, "inlet": 3, "outlet": 4}
_ENERGY = {"total": 0, "internal": 1}
_VISC = {"const_tau": 0, "const_mu": 1, "power": 2, "sutherland": 3}
_COLL = {"mrt": 0, "bgk": 1}
_RHOX = {"pressure": 0, "density": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over grid rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("energy", C.c_int32), ("heating", C.c_int32), ("correction", C.c_int32), ("coupled", C.c_int32),
        ("collision", C.c_int32), ("visc", C.c_int32), ("rho_extrap", C.c_int32), ("pad_", C.c_int32),
        ("side_kind", C.c_int32 * 4),
        ("rho0", C.c_double), ("T0", C.c_double), ("R", C.c_double), ("b", C.c_double), ("Pr", C.c_double),
        ("tau_f", C.c_double), ("s_e", C.c_double), ("s_zeta", C.c_double), ("s_q", C.c_double),
        ("tau_rho", C.c_double), ("tau_j", C.c_double),
        ("mu_ref", C.c_double), ("T_ref", C.c_double), ("visc_n", C.c_double), ("suth_S", C.c_double),
        ("g", C.c_double),
        ("side_ux", C.c_double * 4), ("side_uy", C.c_double * 4), ("side_T", C.c_double * 4),
        ("side_amp", C.c_double * 4), ("side_period", C.c_double * 4),
    ]


_lib = None
_D = C.POINTER(C.c_double)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        lib = C.CDLL(LIB)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(_Params)]
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_init.argtypes = [C.c_void_p, _D, _D, _D, _D]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_stream_only.argtypes = [C.c_void_p, C.c_long]
        lib.orc_time.restype = C.c_long
        lib.orc_time.argtypes = [C.c_void_p]
        lib.orc_macros.argtypes = [C.c_void_p, _D, _D, _D, _D]
        lib.orc_pops.argtypes = [C.c_void_p, _D]
        lib.orc_set_pops.argtypes = [C.c_void_p, _D]
        lib.orc_diag.argtypes = [C.c_void_p, _D]
        lib.orc_residual.restype = C.c_double
        lib.orc_residual.argtypes = [C.c_void_p, C.c_int]
        lib.orc_lattice.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int), _D]
        lib.orc_matrices.argtypes = [_D, _D]
        for name in ("orc_node_feq", "orc_node_heq", "orc_node_meq"):
            getattr(lib, name).argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, _D]
        lib.orc_node_correction.argtypes = [C.c_double, C.c_double, _D]
        lib.orc_node_forcing.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, _D, _D]
        lib.orc_node_moments.argtypes = [C.c_void_p, _D, _D]
        lib.orc_node_collide.argtypes = [C.c_void_p, _D, C.c_double, C.c_double, _D]
        lib.orc_node_transport.argtypes = [C.c_void_p, C.c_double, C.c_double, _D]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _check_sides(p: dict):
    kinds = [s["kind"] for s in p["sides"]]
    for a, b in ((0, 1), (2, 3)):
        if (kinds[a] == "periodic") != (kinds[b] == "periodic"):
            raise ValueError("both sides of an axis must be periodic or both bounded")
    if "inlet" in kinds[1:] or "outlet" in (kinds[0], kinds[2], kinds[3]):
        raise ValueError("inlet only at x-, outlet only at x+")
    if ("inlet" in kinds or "outlet" in kinds) and kinds[2] != "periodic":
        raise ValueError("inlet/outlet need a periodic y axis")
    if kinds[0] != "periodic" and p["nx"] < 3 or kinds[2] != "periodic" and p["ny"] < 3:
        raise ValueError("a bounded axis needs at least 3 nodes")
    if ("adiabatic" in kinds[:2] and p["nx"] < 4) or ("adiabatic" in kinds[2:] and p["ny"] < 4):
        raise ValueError("an axis with an adiabatic wall needs at least 4 nodes")


def _make(p: dict) -> _Params:
    _check_sides(p)
    s = _Params()
    s.nx, s.ny = int(p["nx"]), int(p["ny"])
    s.energy = _ENERGY[p["energy"]]
    s.heating = int(bool(p["heating"]))
    s.correction = int(bool(p["correction"]))
    s.coupled = int(bool(p["coupled"]))
    s.collision = _COLL[p["collision"]]
    s.visc = _VISC[p["visc"]]
    s.rho_extrap = _RHOX[p["rho_extrap"]]
    for name in ("rho0", "T0", "R", "b", "Pr", "tau_f", "s_e", "s_zeta", "s_q", "tau_rho", "tau_j",
                 "mu_ref", "T_ref", "visc_n", "suth_S", "g"):
        setattr(s, name, float(p[name]))
    for k, sd in enumerate(p["sides"]):
        s.side_kind[k] = _KIND[sd["kind"]]
        s.side_ux[k] = sd["ux"]
        s.side_uy[k] = sd["uy"]
        s.side_T[k] = sd["T"]
        s.side_amp[k] = sd["amp"]
        s.side_period[k] = sd["period"]
    return s


class Oracle:
    """One grid of the FP64 reference solver."""

    def __init__(self, params: dict):
        self.lib = _load()
        self.p = dict(params)
        self._s = _make(self.p)
        self.nx, self.ny = self._s.nx, self._s.ny
        self.h = self.lib.orc_create(C.byref(self._s))
        if not self.h:
            raise ValueError("orc_create rejected the parameters")

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ------------------------------------------------------------
    def init(self, rho=None, ux=None, uy=None, T=None):
        arrs = []
        for a in (rho, ux, uy, T):
            arrs.append(None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
        ptrs = [None if a is None else _ptr(a) for a in arrs]
        self.lib.orc_init(self.h, *ptrs)
        return self

    def step(self, n: int = 1):
        self.lib.orc_step(self.h, int(n))
        return self

    def stream_only(self, n: int = 1):
        self.lib.orc_stream_only(self.h, int(n))
        return self

    @property
    def time(self) -> int:
        return int(self.lib.orc_time(self.h))

    def macros(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        self.lib.orc_macros(self.h, *[_ptr(a) for a in out])
        return tuple(out)

    def pops(self) -> np.ndarray:
        out = np.empty((18, self.ny, self.nx))
        self.lib.orc_pops(self.h, _ptr(out))
        return out

    def set_pops(self, pops: np.ndarray):
        a = np.ascontiguousarray(pops, dtype=np.float64)
        assert a.shape == (18, self.ny, self.nx)
        self.lib.orc_set_pops(self.h, _ptr(a))

    def diag(self) -> dict:
        out = np.zeros(5)
        self.lib.orc_diag(self.h, _ptr(out))
        return dict(mass=out[0], energy=out[1], jx=out[2], jy=out[3], bad=int(out[4]))

    def residual(self, update: bool = True) -> float:
        return float(self.lib.orc_residual(self.h, int(update)))

    # -- single-node functions ---------------------------------------------
    def feq(self, rho, ux, uy, T):
        o = np.empty(9)
        self.lib.orc_node_feq(self.h, rho, ux, uy, T, _ptr(o))
        return o

    def heq(self, rho, ux, uy, T):
        o = np.empty(9)
        self.lib.orc_node_heq(self.h, rho, ux, uy, T, _ptr(o))
        return o

    def meq(self, rho, ux, uy, T):
        o = np.empty(9)
        self.lib.orc_node_meq(self.h, rho, ux, uy, T, _ptr(o))
        return o

    def forcing(self, ux, uy, ax, ay):
        Fv, Fh = np.empty(9), np.empty(9)
        self.lib.orc_node_forcing(self.h, ux, uy, ax, ay, _ptr(Fv), _ptr(Fh))
        return Fv, Fh

    def node_moments(self, pops18):
        a = np.ascontiguousarray(pops18, dtype=np.float64)
        o = np.empty(4)
        self.lib.orc_node_moments(self.h, _ptr(a), _ptr(o))
        return o

    def node_collide(self, pops18, phix=0.0, phiy=0.0):
        a = np.ascontiguousarray(pops18, dtype=np.float64)
        o = np.empty(18)
        self.lib.orc_node_collide(self.h, _ptr(a), phix, phiy, _ptr(o))
        return o

    def transport(self, rho, T):
        o = np.empty(12)
        self.lib.orc_node_transport(self.h, rho, T, _ptr(o))
        return dict(tau_f=o[0], s=o[1:10].copy(), omega_h=o[10], inv_tau_hf=o[11])


def set_threads(n: int):
    """Threads of the oracle's OpenMP passes from now on (the CPU baseline)."""
    _load().orc_set_threads(int(n))


def threads() -> int:
    return int(_load().orc_threads())


def correction(phix, phiy):
    o = np.empty(9)
    _load().orc_node_correction(phix, phiy, _ptr(o))
    return o


def lattice():
    ex = (C.c_int * 9)()
    ey = (C.c_int * 9)()
    w = np.empty(9)
    _load().orc_lattice(ex, ey, _ptr(w))
    return np.array(ex[:]), np.array(ey[:]), w


def matrices():
    M, Mi = np.empty((9, 9)), np.empty((9, 9))
    _load().orc_matrices(_ptr(M), _ptr(Mi))
    return M, Mi
