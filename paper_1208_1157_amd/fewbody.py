"""ctypes binding of libfewbody.so (include/fewbody.h).

Argument marshalling only: every step of the integration runs in the HIP
library.  PyTorch provides device memory (the ensemble workspace and the
input tensors) and the stream (torch's current stream).  Importing this
module fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfewbody.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1208_1157_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_BUDGET, E_STATE, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
ACTIVE, DONE, ENCOUNTER, EJECTED, NONFINITE, STALLED_DT, MAXSTEPS = range(7)
STOP_ENCOUNTER, STOP_EJECT = 1, 2
MAP_AUTO, MAP_SPL, MAP_BPL = 0, 1, 2
SCHED_PLAIN, SCHED_PERSISTENT = 0, 1
MAX_BODIES = 16


class FbOpts(ctypes.Structure):
    _fields_ = [("adaptive", ctypes.c_int32), ("eta", ctypes.c_double),
                ("stop_rules", ctypes.c_int32), ("r_eject", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("schedule", ctypes.c_int32),
                ("steps_per_quantum", ctypes.c_int32), ("compact", ctypes.c_int32)]


_p = ctypes.c_void_p
_i32, _i64, _d, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "fb_opts_default": (None, [ctypes.POINTER(FbOpts)]),
    "fb_workspace_bytes": (_sz, [_i32, _p]),
    "fb_ensemble_create": (ctypes.c_int, [_i32, _p, _p, _p, _p, _p, _p, ctypes.POINTER(_p)]),
    "fb_ensemble_create_device": (ctypes.c_int, [_i32, _p, _p, _p, _p, _p, _p, _sz, _p,
                                                 ctypes.POINTER(_p)]),
    "fb_integrate_steps": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbOpts)]),
    "fb_integrate": (ctypes.c_int, [_p, _d, _d, ctypes.POINTER(FbOpts)]),
    "fb_synchronize": (ctypes.c_int, [_p]),
    "fb_get_state": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    "fb_get_hermite_state": (ctypes.c_int, [_p, _p, _p, _p]),
    "fb_diagnostics": (ctypes.c_int, [_p, _p, _p]),
    "fb_ensemble_shape": (ctypes.c_int, [_p, _p, _p]),
    "fb_ensemble_destroy": (ctypes.c_int, [_p]),
    "fb_set_plan": (ctypes.c_int, [_i32, _i32, _i32, _i32]),
    "fb_get_plan": (ctypes.c_int, [_i32, _p, _p, _p]),
    "fb_profile_enable": (ctypes.c_int, [_i32]),
    "fb_profile_read": (ctypes.c_int, [_p, _p]),
    "fb_last_error": (ctypes.c_char_p, []),
    "fb_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class FewbodyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fewbody error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != OK:
        raise FewbodyError(rc, _lib.fb_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())


def lib():
    return _lib


def version() -> str:
    return _lib.fb_version().decode()


@dataclass
class Opts:
    """Integration options (fb_opts)."""
    adaptive: bool = False
    eta: float = 0.01
    stop_rules: int = 0
    r_eject: float = 100.0
    max_steps: int = 0
    schedule: int = SCHED_PLAIN
    steps_per_quantum: int = 0
    compact: bool = False

    def c(self) -> FbOpts:
        return FbOpts(int(self.adaptive), float(self.eta), int(self.stop_rules), float(self.r_eject),
                      int(self.max_steps), int(self.schedule), int(self.steps_per_quantum),
                      int(self.compact))


def set_plan(n, mapping, waves_per_group, groups_per_cu=0):
    _check(_lib.fb_set_plan(int(n), int(mapping), int(waves_per_group), int(groups_per_cu)))


def get_plan(n):
    m, w, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.fb_get_plan(int(n), ctypes.byref(m), ctypes.byref(w), ctypes.byref(g)))
    return m.value, w.value, g.value


def profile_enable(on=True):
    _check(_lib.fb_profile_enable(1 if on else 0))


def profile_read():
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.fb_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def workspace_bytes(n_body) -> int:
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    return int(_lib.fb_workspace_bytes(int(nb.shape[0]), _ptr(nb)))


class Ensemble:
    """A device-resident ensemble of independent few-body systems.

    ``n_body`` [n_sys] bodies per system; ``mass`` [N], ``pos``/``vel`` [N, 3]
    body-major (body b of system s at row off[s] + b).  Inputs may be numpy
    arrays (uploaded through torch) or float64 CUDA tensors.  With
    ``host=True`` the host-pointer entry point is used and the library
    allocates the device state itself.
    """

    def __init__(self, n_body, mass, pos, vel, t0=None, stream=None, host=False):
        import torch
        self._torch = torch
        self.n_body = np.ascontiguousarray(n_body, dtype=np.int32)
        self.n_sys = int(self.n_body.shape[0])
        self.n_bodies = int(self.n_body.sum())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._handle = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if host:
            m = np.ascontiguousarray(mass, dtype=np.float64)
            x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
            v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
            t = None if t0 is None else np.ascontiguousarray(t0, dtype=np.float64)
            self._keep = None
            _check(_lib.fb_ensemble_create(self.n_sys, _ptr(self.n_body), _ptr(m), _ptr(x), _ptr(v),
                                           _ptr(t), sp, ctypes.byref(self._handle)))
            return
        dev = torch.device("cuda", torch.cuda.current_device())

        def dtensor(a, shape):
            if a is None:
                return None
            if isinstance(a, torch.Tensor):
                tt = a.to(device=dev, dtype=torch.float64)
            else:
                tt = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
            return tt.reshape(shape).contiguous()

        with torch.cuda.stream(self.stream):
            m = dtensor(mass, (-1,))
            x = dtensor(pos, (-1, 3))
            v = dtensor(vel, (-1, 3))
            t = dtensor(t0, (-1,))
        ws = workspace_bytes(self.n_body)
        if ws == 0 and self.n_sys > 0:
            raise FewbodyError(E_INVAL, "invalid body counts (each must be 2..16)")
        raw = torch.empty(ws + 256, dtype=torch.uint8, device=dev)
        addr = raw.data_ptr()
        aligned = (addr + 255) // 256 * 256
        self._workspace = raw
        self._keep = (m, x, v, t)
        _check(_lib.fb_ensemble_create_device(self.n_sys, _ptr(self.n_body), _ptr(m), _ptr(x), _ptr(v),
                                              _ptr(t), ctypes.c_void_p(aligned), ctypes.c_size_t(ws),
                                              sp, ctypes.byref(self._handle)))
        self._keep = None   # inputs were packed into the workspace

    # -- integration ---------------------------------------------------------
    def integrate_steps(self, n_steps, dt, opts: Opts | None = None):
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate_steps(self._handle, int(n_steps), float(dt), ctypes.byref(o)))

    def integrate(self, t_end, dt=0.0, opts: Opts | None = None):
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate(self._handle, float(t_end), float(dt), ctypes.byref(o)))

    def synchronize(self):
        _check(_lib.fb_synchronize(self._handle))

    # -- read back -----------------------------------------------------------
    def state(self):
        N, S = self.n_bodies, self.n_sys
        pos, vel = np.empty((N, 3)), np.empty((N, 3))
        t = np.empty(S)
        status = np.empty(S, dtype=np.int32)
        steps = np.empty(S, dtype=np.int64)
        _check(_lib.fb_get_state(self._handle, _ptr(pos), _ptr(vel), _ptr(t), _ptr(status), _ptr(steps)))
        return {"pos": pos, "vel": vel, "t": t, "status": status, "steps": steps}

    def hermite_state(self):
        N, S = self.n_bodies, self.n_sys
        acc, jerk, dtn = np.empty((N, 3)), np.empty((N, 3)), np.empty(S)
        _check(_lib.fb_get_hermite_state(self._handle, _ptr(acc), _ptr(jerk), _ptr(dtn)))
        return acc, jerk, dtn

    def diagnostics(self):
        E = np.empty(self.n_sys)
        L = np.empty((self.n_sys, 3))
        _check(_lib.fb_diagnostics(self._handle, _ptr(E), _ptr(L)))
        return E, L

    def close(self):
        if self._handle:
            _check(_lib.fb_ensemble_destroy(self._handle))
            self._handle = ctypes.c_void_p()
            self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def from_gen(ens, **kw) -> Ensemble:
    """Ensemble from a paper_1208_1157_amd.gen.Ensemble."""
    return Ensemble(ens.n_body, ens.mass, ens.pos, ens.vel, **kw)
