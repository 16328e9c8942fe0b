"""ctypes binding of the gfx950 thermal LBM library (include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``liblbm.so``.  PyTorch provides the device workspace (a uint8 tensor the
library carves up) and the stream the kernels are launched on.  There is no
fallback: if the library is missing, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB as LIB_PATH

STORAGE = {"fp32": 0, "fp64": 1, "fp16": 2, "bf16": 3, "mixed": 4}
BC = {"periodic": 0, "adiabatic": 1, "dirichlet": 2}
DERIVED = ["nu", "alpha", "gbeta", "tau_f", "tau_g", "s_nu", "s_e", "s_eps",
           "s_q", "s_pi", "s_m", "q_j", "q_e", "q_nu", "a_t", "omega",
           "cs2_t", "t0", "H"]
STATUS = {0: "LBM_OK", -1: "LBM_E_INVALID", -2: "LBM_E_DEVICE",
          -3: "LBM_E_UNSTABLE", -4: "LBM_E_STATE", -5: "LBM_E_UNSUPPORTED"}

# every entry point declared in include/lbm.h
EXPORTS = ["lbm_derive", "lbm_workspace_bytes", "lbm_bytes_per_update",
           "lbm_create", "lbm_init", "lbm_init_fields", "lbm_step",
           "lbm_set_steps_per_launch", "lbm_get_steps_per_launch",
           "lbm_set_debug_poison", "lbm_get_debug_poison",
           "lbm_fields", "lbm_nusselt", "lbm_wall_flux", "lbm_diagnostics",
           "lbm_state_bytes", "lbm_export_state", "lbm_import_state",
           "lbm_time", "lbm_destroy", "lbm_last_error", "lbm_lattice",
           "lbm_version", "lbm_batch_workspace_bytes", "lbm_batch_create",
           "lbm_batch_init", "lbm_batch_init_fields", "lbm_batch_step",
           "lbm_batch_cavity", "lbm_batch_nusselt", "lbm_batch_unstable",
           "lbm_batch_tune", "lbm_batch_set_config", "lbm_batch_get_config",
           "lbm_batch_set_steps_per_launch", "lbm_batch_get_steps_per_launch",
           "lbm_batch_time", "lbm_batch_destroy", "lbm_batch_last_error",
           "lbm_probe_bandwidth", "lbm_diagnostics_async"]
DIAG_VALUES = 7  # LBM_DIAG_VALUES: t, mass, energy, umax, nu_vol, re, nonfinite


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


class BatchConfig(C.Structure):
    _fields_ = [("block", C.c_int32), ("grid_per_cu", C.c_int32),
                ("graph_steps", C.c_int32), ("reserved", C.c_int32),
                ("stream_rows", C.c_int32), ("stream_waves", C.c_int32)]

    def as_dict(self):
        return {"block": self.block, "grid_per_cu": self.grid_per_cu,
                "graph_steps": self.graph_steps, "stream_rows": self.stream_rows,
                "stream_waves": self.stream_waves}


BATCH_TUNE_MAX = 80  # LBM_BATCH_TUNE_MAX


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load liblbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        P, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.c_size_t
        pp = C.POINTER(Params)
        L.lbm_derive.argtypes = [pp, dp]
        L.lbm_workspace_bytes.argtypes = [pp]
        L.lbm_workspace_bytes.restype = sz
        L.lbm_bytes_per_update.argtypes = [pp]
        L.lbm_bytes_per_update.restype = C.c_double
        L.lbm_create.argtypes = [pp, P, sz, P, C.POINTER(P)]
        L.lbm_init.argtypes = [P, C.c_uint64, C.c_double]
        L.lbm_init_fields.argtypes = [P, dp, dp, dp]
        L.lbm_step.argtypes = [P, C.c_int64]
        L.lbm_set_steps_per_launch.argtypes = [P, C.c_int32]
        L.lbm_get_steps_per_launch.argtypes = [P]
        L.lbm_get_steps_per_launch.restype = C.c_int32
        L.lbm_set_debug_poison.argtypes = [P, C.c_int32]
        L.lbm_get_debug_poison.argtypes = [P]
        L.lbm_get_debug_poison.restype = C.c_int32
        L.lbm_fields.argtypes = [P, P, P, P]
        L.lbm_nusselt.argtypes = [P, dp, dp]
        L.lbm_wall_flux.argtypes = [P, dp, dp]
        L.lbm_diagnostics.argtypes = [P, C.POINTER(Diag)]
        L.lbm_state_bytes.argtypes = [P]
        L.lbm_state_bytes.restype = sz
        L.lbm_export_state.argtypes = [P, P, sz]
        L.lbm_import_state.argtypes = [P, P, sz]
        L.lbm_time.argtypes = [P]
        L.lbm_time.restype = C.c_int64
        L.lbm_destroy.argtypes = [P]
        L.lbm_destroy.restype = None
        L.lbm_last_error.argtypes = [P]
        L.lbm_last_error.restype = C.c_char_p
        ip = C.POINTER(C.c_int32)
        L.lbm_lattice.argtypes = [C.c_int32, C.c_int32, ip, ip, ip, dp]
        L.lbm_version.restype = C.c_char_p
        bp = C.POINTER(BatchConfig)
        L.lbm_batch_workspace_bytes.argtypes = [pp, C.c_int32]
        L.lbm_batch_workspace_bytes.restype = sz
        L.lbm_batch_create.argtypes = [pp, C.c_int32, P, sz, P, C.POINTER(P)]
        L.lbm_batch_init.argtypes = [P, C.POINTER(C.c_uint64), dp]
        L.lbm_batch_init_fields.argtypes = [P, C.c_int32, dp, dp, dp]
        L.lbm_batch_step.argtypes = [P, C.c_int64]
        L.lbm_batch_cavity.argtypes = [P, C.c_int32, C.POINTER(P)]
        L.lbm_batch_nusselt.argtypes = [P, dp, dp]
        L.lbm_batch_unstable.argtypes = [P, C.POINTER(C.c_int32)]
        L.lbm_batch_tune.argtypes = [P, C.c_int32, bp, dp, C.POINTER(C.c_int32)]
        L.lbm_batch_set_config.argtypes = [P, bp]
        L.lbm_batch_get_config.argtypes = [P, bp]
        L.lbm_batch_set_steps_per_launch.argtypes = [P, C.c_int32]
        L.lbm_batch_get_steps_per_launch.argtypes = [P]
        L.lbm_batch_get_steps_per_launch.restype = C.c_int32
        L.lbm_batch_time.argtypes = [P]
        L.lbm_batch_time.restype = C.c_int64
        L.lbm_batch_destroy.argtypes = [P]
        L.lbm_batch_destroy.restype = None
        L.lbm_batch_last_error.argtypes = [P]
        L.lbm_batch_last_error.restype = C.c_char_p
        L.lbm_probe_bandwidth.argtypes = [C.c_int32, P, P, sz, C.c_int32, C.c_int32, P]
        L.lbm_probe_bandwidth.restype = C.c_int32
        L.lbm_diagnostics_async.argtypes = [P, P]
        L.lbm_diagnostics_async.restype = C.c_int32
        for name in ("lbm_batch_create", "lbm_batch_init", "lbm_batch_init_fields",
                     "lbm_batch_step", "lbm_batch_cavity", "lbm_batch_nusselt",
                     "lbm_batch_unstable", "lbm_batch_tune", "lbm_batch_set_config",
                     "lbm_batch_get_config", "lbm_batch_set_steps_per_launch"):
            getattr(L, name).restype = C.c_int32
        for name in ("lbm_derive", "lbm_create", "lbm_init", "lbm_init_fields",
                     "lbm_step", "lbm_set_steps_per_launch", "lbm_set_debug_poison", "lbm_fields",
                     "lbm_nusselt", "lbm_wall_flux",
                     "lbm_diagnostics", "lbm_export_state", "lbm_import_state",
                     "lbm_lattice"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


PROBE_KINDS = {"copy": 0, "read": 1, "write": 2}


def probe_bandwidth(kind: str, src, dst, nbytes: int, per_thread: int, nontemporal: bool, stream):
    """One launch of the HBM bandwidth probe on `stream` (src and dst are
    device tensors; src may be None for kind "write")."""
    st = lib().lbm_probe_bandwidth(PROBE_KINDS[kind], None if src is None else src.data_ptr(),
                                   dst.data_ptr(), int(nbytes), int(per_thread), int(bool(nontemporal)),
                                   stream.cuda_stream)
    if st != 0:
        raise LBMError(st, "lbm_probe_bandwidth rejected its arguments or failed to launch")


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    """lbm_params from a run configuration dict (see workloads)."""
    nan = math.nan
    p = Params()
    p.dim = int(cfg["dim"])
    n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
    for a in range(3):
        p.n[a] = int(n[a])
    st = cfg.get("storage", "fp32")
    p.storage = STORAGE[st] if isinstance(st, str) else int(st)
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


def _raise(status, ctx=None):
    if status != 0:
        raise LBMError(status, lib().lbm_last_error(ctx).decode())


def derive(cfg: dict) -> dict:
    out = np.empty(len(DERIVED))
    _raise(lib().lbm_derive(C.byref(make_params(cfg)), _dp(out)))
    return dict(zip(DERIVED, out.tolist()))


def workspace_bytes(cfg: dict) -> int:
    nbytes = lib().lbm_workspace_bytes(C.byref(make_params(cfg)))
    if nbytes == 0:
        raise LBMError(-1, lib().lbm_last_error(None).decode())
    return int(nbytes)


def bytes_per_update(cfg: dict) -> float:
    return float(lib().lbm_bytes_per_update(C.byref(make_params(cfg))))


def lattice(dim: int, thermal: bool):
    """Kernel tables: (e[q,3], M[q,q], w[q])."""
    q = C.c_int32()
    L = lib()
    _raise(L.lbm_lattice(dim, int(thermal), C.byref(q), None, None, None))
    q = q.value
    e = np.empty(3 * q, np.int32)
    M = np.empty(q * q, np.int32)
    w = np.empty(q)
    ip = C.POINTER(C.c_int32)
    _raise(L.lbm_lattice(dim, int(thermal), None, e.ctypes.data_as(ip),
                         M.ctypes.data_as(ip), _dp(w)))
    return e.reshape(q, 3), M.reshape(q, q), w


class Cavity:
    """One thermal cavity advanced by the fused HIP step on cuda:0.

    The device workspace is a torch uint8 tensor owned by this object; the
    kernels run on ``stream`` (default: torch's current stream).
    """

    def __init__(self, cfg: dict, stream=None):
        import torch
        self.cfg = dict(cfg)
        self.dim = int(cfg["dim"])
        n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self._p = make_params(cfg)
        nbytes = workspace_bytes(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _raise(lib().lbm_create(C.byref(self._p), C.c_void_p(self.workspace.data_ptr()),
                                nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._destroy = lib().lbm_destroy  # kept for close() at interpreter exit

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (ny, nx) if self.dim == 2 else (nz, ny, nx)

    def _check(self, st):
        _raise(st, self._h)

    def init(self, seed: int, amp: float):
        self._check(lib().lbm_init(self._h, C.c_uint64(seed), float(amp)))

    def init_fields(self, rho, u, T):
        rho = None if rho is None else np.ascontiguousarray(rho, np.float64).ravel()
        u = np.ascontiguousarray(u, np.float64).reshape(self.dim, self.N)
        T = np.ascontiguousarray(T, np.float64).ravel()
        self._check(lib().lbm_init_fields(self._h, _dp(rho), _dp(u), _dp(T)))

    def step(self, n: int = 1):
        self._check(lib().lbm_step(self._h, int(n)))

    @property
    def steps_per_launch(self) -> int:
        """Steps per kernel launch of step(): 1 .. 5 in 2D, 1 or 2 in 3D; a
        cavity starts with the fastest count for its storage mode."""
        return int(lib().lbm_get_steps_per_launch(self._h))

    @steps_per_launch.setter
    def steps_per_launch(self, k: int):
        self._check(lib().lbm_set_steps_per_launch(self._h, int(k)))

    @property
    def debug_poison(self) -> bool:
        """Debug mode: the buffer each launch writes is filled with NaN
        first, so a population left unwritten shows as non-finite."""
        return bool(lib().lbm_get_debug_poison(self._h))

    @debug_poison.setter
    def debug_poison(self, on: bool):
        self._check(lib().lbm_set_debug_poison(self._h, 1 if on else 0))

    @property
    def t(self) -> int:
        return int(lib().lbm_time(self._h))

    def fields(self, check: bool = True):
        """(rho, u, T) as FP64 numpy arrays shaped like the grid."""
        rho = np.empty(self.N)
        u = np.empty(self.dim * self.N)
        T = np.empty(self.N)
        st = lib().lbm_fields(self._h, rho.ctypes.data, u.ctypes.data, T.ctypes.data)
        if check:
            self._check(st)
        return (rho.reshape(self.shape), u.reshape((self.dim,) + self.shape),
                T.reshape(self.shape))

    def fields_device(self, check: bool = True):
        """(rho, u, T) as FP64 torch tensors on the device."""
        import torch
        rho = torch.empty(self.N, dtype=torch.float64, device="cuda")
        u = torch.empty(self.dim * self.N, dtype=torch.float64, device="cuda")
        T = torch.empty(self.N, dtype=torch.float64, device="cuda")
        st = lib().lbm_fields(self._h, rho.data_ptr(), u.data_ptr(), T.data_ptr())
        if check:
            self._check(st)
        return rho, u, T

    def nusselt(self):
        a, b = C.c_double(), C.c_double()
        self._check(lib().lbm_nusselt(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def wall_flux(self):
        last = np.empty(6)
        prev = np.empty(6)
        self._check(lib().lbm_wall_flux(self._h, _dp(last), _dp(prev)))
        return last, prev

    def diagnostics(self, check: bool = True) -> dict:
        d = Diag()
        st = lib().lbm_diagnostics(self._h, C.byref(d))
        if check:
            self._check(st)
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def export_state(self) -> bytes:
        nbytes = int(lib().lbm_state_bytes(self._h))
        buf = C.create_string_buffer(nbytes)
        self._check(lib().lbm_export_state(self._h, C.cast(buf, C.c_void_p), nbytes))
        return buf.raw

    def import_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        self._check(lib().lbm_import_state(self._h, C.cast(buf, C.c_void_p), len(state)))

    def derived(self) -> dict:
        return derive(self.cfg)

    def bytes_per_update(self) -> float:
        """Algorithmic HBM bytes per lattice update at the current number
        of steps per launch."""
        return bytes_per_update(self.cfg) / self.steps_per_launch


class _View(Cavity):
    """A cavity owned by a Batch (no workspace of its own)."""

    def __init__(self, batch, k, handle, cfg):
        self.cfg = dict(cfg)
        self.dim = int(cfg["dim"])
        n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
        self.n = tuple(int(v) for v in n)
        self.N = self.n[0] * self.n[1] * self.n[2]
        self.stream = batch.stream
        self._batch = batch  # keeps the workspace alive
        self._h = handle

    def close(self):
        self._h = None  # owned by the batch


class Batch:
    """Many cavities advanced by one launch per step (lbm_batch_*).

    Runs on its own torch stream (default priority) so that hipGraph capture
    is available.
    """

    def __init__(self, cfgs, stream=None):
        import torch
        self.cfgs = [dict(c) for c in cfgs]
        self.count = len(cfgs)
        arr = (Params * self.count)(*[make_params(c) for c in cfgs])
        self._arr = arr
        nbytes = lib().lbm_batch_workspace_bytes(arr, self.count)
        if nbytes == 0:
            raise LBMError(-1, lib().lbm_batch_last_error(None).decode())
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        h = C.c_void_p()
        st = lib().lbm_batch_create(arr, self.count, C.c_void_p(self.workspace.data_ptr()),
                                    int(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise LBMError(st, lib().lbm_batch_last_error(None).decode())
        self._h = h
        self._destroy = lib().lbm_batch_destroy  # kept for close() at interpreter exit
        self.nodes = [int(np.prod(list(c["n"]) + [1] * (3 - len(c["n"])))) for c in cfgs]

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, st):
        if st != 0:
            raise LBMError(st, lib().lbm_batch_last_error(self._h).decode())

    def init(self, seeds, amps):
        s = (C.c_uint64 * self.count)(*[int(v) for v in seeds])
        a = np.ascontiguousarray(amps, np.float64)
        self._check(lib().lbm_batch_init(self._h, s, _dp(a)))

    def init_fields(self, k, rho, u, T):
        n = self.nodes[k]
        dim = int(self.cfgs[k]["dim"])
        rho = None if rho is None else np.ascontiguousarray(rho, np.float64).ravel()
        u = np.ascontiguousarray(u, np.float64).reshape(dim, n)
        T = np.ascontiguousarray(T, np.float64).ravel()
        self._check(lib().lbm_batch_init_fields(self._h, k, _dp(rho), _dp(u), _dp(T)))

    def step(self, n: int = 1):
        self._check(lib().lbm_batch_step(self._h, int(n)))

    @property
    def t(self) -> int:
        return int(lib().lbm_batch_time(self._h))

    @property
    def steps_per_launch(self) -> int:
        """Steps per launch of step(): 1, or 2..5 (streaming, 2D)."""
        return int(lib().lbm_batch_get_steps_per_launch(self._h))

    @steps_per_launch.setter
    def steps_per_launch(self, k: int):
        self._check(lib().lbm_batch_set_steps_per_launch(self._h, int(k)))

    def cavity(self, k: int) -> Cavity:
        h = C.c_void_p()
        self._check(lib().lbm_batch_cavity(self._h, int(k), C.byref(h)))
        return _View(self, k, h, self.cfgs[k])

    def nusselt(self):
        hot = np.empty(self.count)
        cold = np.empty(self.count)
        self._check(lib().lbm_batch_nusselt(self._h, _dp(hot), _dp(cold)))
        return hot, cold

    def unstable(self):
        f = (C.c_int32 * self.count)()
        self._check(lib().lbm_batch_unstable(self._h, f))
        return np.array(f[:], dtype=bool)

    def config(self) -> dict:
        c = BatchConfig()
        self._check(lib().lbm_batch_get_config(self._h, C.byref(c)))
        return c.as_dict()

    def set_config(self, block=256, grid_per_cu=0, graph_steps=0, stream_rows=0, stream_waves=0):
        c = BatchConfig(int(block), int(grid_per_cu), int(graph_steps), 0, int(stream_rows), int(stream_waves))
        self._check(lib().lbm_batch_set_config(self._h, C.byref(c)))

    def tune(self, steps: int = 5):
        """Autotune (lbm_batch_tune): returns the chosen configuration (its
        steps per launch is self.steps_per_launch afterwards) and the
        per-step timings of every candidate, in ms."""
        best = BatchConfig()
        ms = np.zeros(BATCH_TUNE_MAX)
        n = C.c_int32()
        self._check(lib().lbm_batch_tune(self._h, int(steps), C.byref(best), _dp(ms), C.byref(n)))
        return best.as_dict(), ms[: n.value].tolist()
