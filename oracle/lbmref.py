"""ctypes binding of the FP64 CPU oracle (liblbmref.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  This module imports nothing from the
GPU package; a run configuration is a plain dict (see
``paper_2211_03160_amd.workloads`` for the recipes) that this module turns
into the oracle's own parameter struct.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LBMREF_LIB points the binding at another build (the planted-mistake tests
# load deliberately broken copies of the oracle through it)
LIB_PATH = os.environ.get("LBMREF_LIB") or os.path.join(HERE, "liblbmref.so")

BC = {"periodic": 0, "adiabatic": 1, "dirichlet": 2}
DERIVED = ["nu", "alpha", "gbeta", "tau_f", "tau_g", "s_nu", "s_e", "s_eps",
           "s_q", "s_pi", "s_m", "q_j", "q_e", "q_nu", "a_t", "omega",
           "cs2_t", "t0", "H"]


class Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3),
                ("storage", C.c_int32), ("bc", C.c_int32 * 6),
                ("reserved", C.c_int32), ("t_wall", C.c_double * 6),
                ("ra", C.c_double), ("pr", C.c_double), ("u_ff", C.c_double),
                ("t_hot", C.c_double), ("t_cold", C.c_double),
                ("nu", C.c_double), ("alpha", C.c_double),
                ("gbeta", C.c_double), ("a_t", C.c_double),
                ("s_e", C.c_double), ("s_eps", C.c_double),
                ("s_q", C.c_double), ("s_pi", C.c_double),
                ("s_m", C.c_double), ("q_e", C.c_double),
                ("q_nu", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_int64), ("mass", C.c_double),
                ("energy", C.c_double), ("umax", C.c_double),
                ("nu_vol", C.c_double), ("re", C.c_double),
                ("nonfinite", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: build it with "
                               f"`python {os.path.join(HERE, 'build.py')}`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.lbmref_create.argtypes = [C.POINTER(Params), C.POINTER(P)]
        L.lbmref_destroy.argtypes = [P]
        L.lbmref_destroy.restype = None
        L.lbmref_last_error.argtypes = [P]
        L.lbmref_last_error.restype = C.c_char_p
        L.lbmref_init.argtypes = [P, C.c_uint64, C.c_double]
        L.lbmref_init_fields.argtypes = [P, dp, dp, dp]
        L.lbmref_step.argtypes = [P, C.c_int64]
        L.lbmref_fields.argtypes = [P, dp, dp, dp]
        L.lbmref_nusselt.argtypes = [P, dp, dp]
        L.lbmref_diagnostics.argtypes = [P, C.POINTER(Diag)]
        L.lbmref_time.argtypes = [P]
        L.lbmref_time.restype = C.c_int64
        L.lbmref_wall_flux.argtypes = [P, dp, dp]
        L.lbmref_get_populations.argtypes = [P, dp, dp]
        L.lbmref_set_populations.argtypes = [P, dp, dp]
        L.lbmref_derived.argtypes = [P, dp]
        L.lbmref_derive.argtypes = [C.POINTER(Params), dp]
        L.lbmref_lattice.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int),
                                     dp, dp, dp, dp]
        L.lbmref_splitmix64.argtypes = [C.c_uint64]
        L.lbmref_splitmix64.restype = C.c_uint64
        L.lbmref_threads.restype = C.c_int
        L.lbmref_set_threads.argtypes = [C.c_int]
        L.lbmref_set_threads.restype = None
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    nan = math.nan
    p = Params()
    p.dim = int(cfg["dim"])
    n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
    for a in range(3):
        p.n[a] = int(n[a])
    for k, b in enumerate(cfg["bc"]):
        p.bc[k] = BC[b] if isinstance(b, str) else int(b)
    tw = cfg.get("t_wall", (0.0,) * 6)
    for k in range(6):
        p.t_wall[k] = float(tw[k])
    for name in ("ra", "pr", "u_ff", "t_hot", "t_cold"):
        setattr(p, name, float(cfg.get(name, nan)))
    for name in ("nu", "alpha", "gbeta", "a_t", "s_e", "s_eps", "s_q",
                 "s_pi", "s_m", "q_e", "q_nu"):
        v = cfg.get(name)
        setattr(p, name, nan if v is None else float(v))
    return p


class Oracle:
    """One cavity advanced by the FP64 CPU oracle."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.dim = int(cfg["dim"])
        n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.qf, self.qg = (9, 5) if self.dim == 2 else (19, 7)
        self._p = make_params(cfg)
        h = C.c_void_p()
        st = lib().lbmref_create(C.byref(self._p), C.byref(h))
        if st != 0:
            raise OracleError(st, lib().lbmref_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().lbmref_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != 0:
            raise OracleError(st, lib().lbmref_last_error(self._h).decode())

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (ny, nx) if self.dim == 2 else (nz, ny, nx)

    def init(self, seed: int, amp: float):
        self._check(lib().lbmref_init(self._h, C.c_uint64(seed), amp))

    def init_fields(self, rho, u, T):
        rho = None if rho is None else np.ascontiguousarray(rho, np.float64).ravel()
        u = np.ascontiguousarray(u, np.float64).reshape(self.dim, self.N)
        T = np.ascontiguousarray(T, np.float64).ravel()
        self._check(lib().lbmref_init_fields(self._h, _dp(rho), _dp(u), _dp(T)))

    def step(self, n: int = 1):
        self._check(lib().lbmref_step(self._h, int(n)))

    @property
    def t(self) -> int:
        return int(lib().lbmref_time(self._h))

    def fields(self, check: bool = True):
        rho = np.empty(self.N)
        u = np.empty(self.dim * self.N)
        T = np.empty(self.N)
        st = lib().lbmref_fields(self._h, _dp(rho), _dp(u), _dp(T))
        if check:
            self._check(st)
        return (rho.reshape(self.shape), u.reshape((self.dim,) + self.shape),
                T.reshape(self.shape))

    def nusselt(self):
        a, b = C.c_double(), C.c_double()
        self._check(lib().lbmref_nusselt(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def diagnostics(self, check: bool = True) -> dict:
        d = Diag()
        st = lib().lbmref_diagnostics(self._h, C.byref(d))
        if check:
            self._check(st)
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def wall_flux(self):
        last = np.empty(6)
        prev = np.empty(6)
        self._check(lib().lbmref_wall_flux(self._h, _dp(last), _dp(prev)))
        return last, prev

    def populations(self):
        f = np.empty(self.qf * self.N)
        g = np.empty(self.qg * self.N)
        self._check(lib().lbmref_get_populations(self._h, _dp(f), _dp(g)))
        return f.reshape(self.qf, self.N), g.reshape(self.qg, self.N)

    def set_populations(self, f, g):
        f = np.ascontiguousarray(f, np.float64).ravel()
        g = np.ascontiguousarray(g, np.float64).ravel()
        self._check(lib().lbmref_set_populations(self._h, _dp(f), _dp(g)))

    def derived(self) -> dict:
        out = np.empty(len(DERIVED))
        self._check(lib().lbmref_derived(self._h, _dp(out)))
        return dict(zip(DERIVED, out.tolist()))


def derive(cfg: dict) -> dict:
    """The oracle's own parameter mapping for a run configuration (no state
    is created)."""
    p = make_params(cfg)
    out = np.empty(len(DERIVED))
    st = lib().lbmref_derive(C.byref(p), _dp(out))
    if st != 0:
        raise OracleError(st, lib().lbmref_last_error(None).decode())
    return dict(zip(DERIVED, out.tolist()))


def lattice(dim: int, thermal: bool):
    """The oracle's lattice tables: (e[q,3], w[q], M[q,q], Minv[q,q])."""
    q = C.c_int()
    L = lib()
    st = L.lbmref_lattice(dim, int(thermal), C.byref(q), None, None, None, None)
    if st != 0:
        raise OracleError(st, "bad lattice request")
    q = q.value
    e = np.empty(q * 3)
    w = np.empty(q)
    M = np.empty(q * q)
    Mi = np.empty(q * q)
    L.lbmref_lattice(dim, int(thermal), None, _dp(e), _dp(w), _dp(M), _dp(Mi))
    return e.reshape(q, 3).astype(int), w, M.reshape(q, q), Mi.reshape(q, q)


def splitmix64(x: int) -> int:
    return int(lib().lbmref_splitmix64(C.c_uint64(x)))


def threads() -> int:
    return int(lib().lbmref_threads())


def set_threads(n: int):
    lib().lbmref_set_threads(int(n))
