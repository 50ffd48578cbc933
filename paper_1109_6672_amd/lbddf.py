"""Thin ctypes binding of ``liblbddf.so`` (declared in ``include/lbddf.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
the library.  PyTorch provides the device buffer and the stream.  There is no
CPU fallback: importing works without a GPU, but creating a solver needs the
built library and a visible GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbddf.so")  # FP32 arithmetic
# the same ABI with the step's arithmetic in FP64 (storage formats unchanged)
LIB_PATH_FP64 = os.path.join(HERE, "liblbddf_fp64.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_EUNSTABLE, LB_EBUSY = 0, -1, -2, -3, -4, -5
_STORAGE = {"f32": 0, "f16": 1, "bf16": 2}
_ENERGY = {"total": 0, "internal": 1}
_VISC = {"const_tau": 0, "const_mu": 1, "power": 2, "sutherland": 3}
_KIND = {"periodic": 0, "wall": 1, "adiabatic": 2, "inlet": 3, "outlet": 4}
_COLL = {"mrt": 0, "bgk": 1}
_RHOX = {"pressure": 0, "density": 1}


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbddf status {status}: {msg}")
        self.status = status


class lb_side(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("ux", C.c_double), ("uy", C.c_double),
                ("T", C.c_double), ("amp", C.c_double), ("period", C.c_double)]


class lb_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("storage", C.c_int32), ("energy", C.c_int32),
        ("heating", C.c_int32), ("correction", C.c_int32), ("coupled", C.c_int32), ("collision", C.c_int32),
        ("visc", C.c_int32), ("rho_extrap", C.c_int32),
        ("rho0", C.c_double), ("T0", C.c_double), ("R", C.c_double), ("b", C.c_double), ("Pr", C.c_double),
        ("tau_f", C.c_double), ("s_e", C.c_double), ("s_zeta", C.c_double), ("s_q", C.c_double),
        ("tau_rho", C.c_double), ("tau_j", C.c_double), ("mu_ref", C.c_double), ("T_ref", C.c_double),
        ("visc_n", C.c_double), ("suth_S", C.c_double), ("g", C.c_double),
        ("side", lb_side * 4),
    ]


_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
# symbol -> (restype, argtypes)
_SIGS = {
    "lb_validate": (C.c_int, [C.POINTER(lb_params)]),
    "lb_state_bytes": (C.c_size_t, [C.POINTER(lb_params)]),
    "lb_create": (C.c_int, [C.POINTER(lb_params), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lb_init": (C.c_int, [C.c_void_p, _D, _D, _D, _D]),
    "lb_step": (C.c_int, [C.c_void_p, C.c_long]),
    "lb_time": (C.c_long, [C.c_void_p]),
    "lb_macros": (C.c_int, [C.c_void_p, _D, _D, _D, _D]),
    "lb_macros_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lb_populations": (C.c_int, [C.c_void_p, _D]),
    "lb_diag": (C.c_int, [C.c_void_p, _D]),
    "lb_diag_noalloc": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lb_residual": (C.c_int, [C.c_void_p, C.c_int, _D]),
    "lb_checkpoint_bytes": (C.c_size_t, [C.c_void_p]),
    "lb_save": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lb_load": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lb_set_strip_rows": (C.c_int, [C.c_void_p, C.c_int]),
    "lb_set_graph_steps": (C.c_int, [C.c_void_p, C.c_int]),
    "lb_strip_rows": (C.c_int, [C.c_void_p]),
    "lb_stream": (C.c_void_p, [C.c_void_p]),
    "lb_copy_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "lb_destroy": (None, [C.c_void_p]),
    "lb_last_error": (C.c_char_p, []),
    "lbs_pool_overhead": (C.c_size_t, []),
    "lbs_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbs_submit": (C.c_int, [C.c_void_p, C.POINTER(lb_params), _D, _D, _D, _D, C.c_double, C.c_long,
                             C.POINTER(C.c_long)]),
    "lbs_advance": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "lbs_poll": (C.c_int, [C.c_void_p, C.c_long, C.POINTER(C.c_int), C.POINTER(C.c_long), _D, _D]),
    "lbs_result": (C.c_int, [C.c_void_p, C.c_long, _D, _D, _D, _D]),
    "lbs_release": (C.c_int, [C.c_void_p, C.c_long]),
    "lbs_stats": (C.c_int, [C.c_void_p, _D]),
    "lbs_destroy": (None, [C.c_void_p]),
}

LBS_STATES = {0: "queued", 1: "running", 2: "converged", 3: "plateau", 4: "step_cap", 5: "unstable"}


_libs = {}


def load(arith: str = "f32"):
    """Loads the in-tree library for the arithmetic ("f32", or "f64":
    liblbddf_fp64.so); raises if it has not been built."""
    path = {"f32": LIB_PATH, "f64": LIB_PATH_FP64}[arith]
    lib = _libs.get(path)
    if lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname as the system
        # one.  Importing torch first makes the library bind to that runtime,
        # so device pointers and streams from torch are valid in both; loaded
        # the other way round the process would hold two runtimes.
        import torch  # noqa: F401
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _libs[path] = lib
    return lib


def _check_in(lib, status):
    _check(status, lib)


def _check(status, lib=None):
    """Raises on a failed call; the message comes from the library that
    failed (each keeps its own last error)."""
    if status != LB_OK:
        raise LBError(status, (lib or load()).lb_last_error().decode())


def make_params(p: dict) -> lb_params:
    s = lb_params()
    s.nx, s.ny = int(p["nx"]), int(p["ny"])
    s.storage = _STORAGE[p.get("storage", "f32")]
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
        s.side[k].kind = _KIND[sd["kind"]]
        s.side[k].ux, s.side[k].uy, s.side[k].T = sd["ux"], sd["uy"], sd["T"]
        s.side[k].amp, s.side[k].period = sd["amp"], sd["period"]
    return s


def state_bytes(p: dict) -> int:
    s = make_params(p)
    n = load().lb_state_bytes(C.byref(s))
    if n == 0:
        raise LBError(LB_EINVAL, load().lb_last_error().decode())
    return int(n)


def validate(p: dict) -> None:
    _check(load().lb_validate(C.byref(make_params(p))))


def copy_probe(src, dst, stream=None) -> None:
    """lb_copy_probe: the library's STREAM-like copy of the device tensor src
    into dst (same byte size, 16-byte aligned), asynchronously on the given
    torch stream (default: the current one); the practical memory ceiling
    that the step's bandwidth is read against."""
    import torch

    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("copy_probe: src and dst differ in size")
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().lb_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                C.c_void_p(st.cuda_stream)))


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_D)


class Solver:
    """One grid on one GPU: device state in a torch buffer, kernels in liblbddf
    (arith="f64": liblbddf_fp64.so, the step's arithmetic in FP64)."""

    def __init__(self, params: dict, device: int = 0, stream=None, arith: str = "f32"):
        import torch

        self.lib = load(arith)
        self.arith = arith
        self.p = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self._s = make_params(self.p)
        nbytes = self.lib.lb_state_bytes(C.byref(self._s))
        if nbytes == 0:
            raise LBError(LB_EINVAL, self.lib.lb_last_error().decode())
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check_in(self.lib, self.lib.lb_create(C.byref(self._s), C.c_void_p(self.buf.data_ptr()), C.c_size_t(nbytes),
                                      C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _field(self, a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        assert a.size == self.nx * self.ny
        return a

    def init(self, rho=None, ux=None, uy=None, T=None):
        arrs = [self._field(a) for a in (rho, ux, uy, T)]
        _check_in(self.lib, self.lib.lb_init(self.h, *[_dptr(a) for a in arrs]))
        return self

    def step(self, n: int = 1):
        _check_in(self.lib, self.lib.lb_step(self.h, int(n)))
        return self

    @property
    def time(self) -> int:
        return int(self.lib.lb_time(self.h))

    def macros(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        _check_in(self.lib, self.lib.lb_macros(self.h, *[_dptr(a) for a in out]))
        return tuple(out)

    def macros_device(self):
        import torch

        out = [torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device) for _ in range(4)]
        _check_in(self.lib, self.lib.lb_macros_device(self.h, *[C.c_void_p(t.data_ptr()) for t in out]))
        return tuple(out)

    def populations(self) -> np.ndarray:
        out = np.empty((18, self.ny, self.nx))
        _check_in(self.lib, self.lib.lb_populations(self.h, _dptr(out)))
        return out

    def diag(self, check: bool = True) -> dict:
        out = np.zeros(6)
        st = self.lib.lb_diag(self.h, _dptr(out))
        if check and st != LB_OK:
            _check(st, self.lib)
        return dict(mass=out[0], energy=out[1], jx=out[2], jy=out[3], bad=int(out[4]), time=int(out[5]),
                    status=int(st))

    def diag_noalloc(self, out):
        """lb_diag_noalloc into a float64 torch tensor of 6 on the device
        (asynchronous on the solver's stream)."""
        _check_in(self.lib, self.lib.lb_diag_noalloc(self.h, C.c_void_p(out.data_ptr())))
        return out

    def residual(self, update: bool = True) -> float:
        r = np.zeros(1)
        _check_in(self.lib, self.lib.lb_residual(self.h, int(update), _dptr(r)))
        return float(r[0])

    def save(self) -> bytes:
        n = self.lib.lb_checkpoint_bytes(self.h)
        buf = C.create_string_buffer(int(n))
        _check_in(self.lib, self.lib.lb_save(self.h, buf))
        return buf.raw

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check_in(self.lib, self.lib.lb_load(self.h, buf))
        return self

    def set_strip_rows(self, rows: int):
        _check_in(self.lib, self.lib.lb_set_strip_rows(self.h, int(rows)))

    def set_graph_steps(self, k: int):
        """Launches per captured graph of step() (even, 0 = host launches)."""
        _check_in(self.lib, self.lib.lb_set_graph_steps(self.h, int(k)))

    @property
    def strip_rows(self) -> int:
        return int(self.lib.lb_strip_rows(self.h))


class Server:
    """Continuous-batching server over one device pool (the lbs_* calls)."""

    def __init__(self, pool_bytes: int, storage: str = "f32", k_steps: int = 100, device: int = 0, stream=None,
                 arith: str = "f32"):
        import torch

        self.lib = load(arith)
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check_in(self.lib, self.lib.lbs_create(C.c_void_p(self.pool.data_ptr()), C.c_size_t(int(pool_bytes)),
                                       _STORAGE[storage], int(k_steps), C.c_void_p(self.stream.cuda_stream),
                                       C.byref(h)))
        self.h = h
        self.storage = storage
        self.k = int(k_steps)
        self.shapes = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, params: dict, fields=None, tol: float = 1e-8, max_steps: int = 10 ** 6) -> int:
        p = dict(params, storage=self.storage)
        s = make_params(p)
        n = int(p["nx"]) * int(p["ny"])
        arrs = [None] * 4 if fields is None else [
            None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in fields]
        for a in arrs:
            assert a is None or a.size == n
        rid = C.c_long()
        _check_in(self.lib, self.lib.lbs_submit(self.h, C.byref(s), *[_dptr(a) for a in arrs], float(tol), int(max_steps),
                                   C.byref(rid)))
        self.shapes[rid.value] = (int(p["ny"]), int(p["nx"]))
        return rid.value

    def advance(self):
        r, q = C.c_int(), C.c_int()
        _check_in(self.lib, self.lib.lbs_advance(self.h, C.byref(r), C.byref(q)))
        return r.value, q.value

    def poll(self, rid: int) -> dict:
        st, steps, res, t = C.c_int(), C.c_long(), np.zeros(1), np.zeros(3)
        _check_in(self.lib, self.lib.lbs_poll(self.h, int(rid), C.byref(st), C.byref(steps), _dptr(res), _dptr(t)))
        return dict(state=LBS_STATES[st.value], steps=steps.value, residual=float(res[0]), t_submit=t[0],
                    t_admit=t[1], t_done=t[2])

    def result(self, rid: int):
        ny, nx = self.shapes[rid]
        out = [np.empty((ny, nx)) for _ in range(4)]
        _check_in(self.lib, self.lib.lbs_result(self.h, int(rid), *[_dptr(a) for a in out]))
        return tuple(out)

    def release(self, rid: int):
        _check_in(self.lib, self.lib.lbs_release(self.h, int(rid)))
        self.shapes.pop(rid, None)

    def stats(self) -> dict:
        o = np.zeros(6)
        _check_in(self.lib, self.lib.lbs_stats(self.h, _dptr(o)))
        return dict(batches=int(o[0]), node_updates=o[1], busy_s=o[2], finished=int(o[3]), free_bytes=int(o[4]),
                    queued=int(o[5]))
