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
# torch first: its wheel carries its own HIP runtime (SONAME libamdhip64.so.7,
# which torch's libraries request as libamdhip64.so).  Loading torch before
# this library makes the dynamic loader resolve our libamdhip64.so.7 to that
# same runtime, so the process has exactly one HIP runtime and torch's device
# memory and streams are valid in our calls.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfewbody.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1208_1157_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_BUDGET, E_STATE, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
ACTIVE, DONE, ENCOUNTER, EJECTED, NONFINITE, STALLED_DT, MAXSTEPS, UNBOUND = range(8)
MAX_MVS_BODIES = 8
STOP_ENCOUNTER, STOP_EJECT = 1, 2
MAP_AUTO, MAP_SPL, MAP_BPL = 0, 1, 2
SCHED_PLAIN, SCHED_PERSISTENT = 0, 1
MAX_BODIES = 512         # bodies per system
MAX_SMALL_BODIES = 16    # ... for every integrator and schedule (larger: fixed Hermite steps, plain schedule)


class FbOpts(ctypes.Structure):
    _fields_ = [("adaptive", ctypes.c_int32), ("eta", ctypes.c_double),
                ("stop_rules", ctypes.c_int32), ("r_eject", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("schedule", ctypes.c_int32),
                ("steps_per_quantum", ctypes.c_int32), ("compact", ctypes.c_int32)]


class FbServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_resident", ctypes.c_int32),
                ("steps_per_quantum", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("quantum_tiles", ctypes.c_int32), ("chunk_slots", ctypes.c_int32),
                ("long_steps", ctypes.c_int32), ("idle_spread", ctypes.c_int32)]


class FbServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("resident", ctypes.c_int64), ("quanta", ctypes.c_int64),
                ("system_steps", ctypes.c_double), ("busy_seconds", ctypes.c_double),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("spread_quanta", ctypes.c_int64)]


class FbLogSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("every", ctypes.c_int32), ("max_records", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("los", ctypes.c_double * 3), ("d_buffer", ctypes.c_void_p),
                ("buffer_bytes", ctypes.c_size_t)]


class FbTuneEntry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mapping", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("ms", ctypes.c_double), ("chosen", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = range(5)
POLICY_FAIR, POLICY_SRPT = 0, 1
LOG_STATE, LOG_RV, LOG_ENERGY = 0, 1, 2

_p = ctypes.c_void_p
_i32, _i64, _d, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_SIGS = {
    "fb_opts_default": (None, [ctypes.POINTER(FbOpts)]),
    "fb_workspace_bytes": (_sz, [_i32, _p]),
    "fb_ensemble_create": (ctypes.c_int, [_i32, _p, _p, _p, _p, _p, _p, ctypes.POINTER(_p)]),
    "fb_ensemble_create_device": (ctypes.c_int, [_i32, _p, _p, _p, _p, _p, _p, _sz, _p,
                                                 ctypes.POINTER(_p)]),
    "fb_ensemble_restore": (ctypes.c_int, [_i32, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p,
                                           ctypes.POINTER(_p)]),
    "fb_hermite_steps_workspace_bytes": (_sz, [_i32, _i32]),
    "fb_hermite_steps_device": (ctypes.c_int, [_i32, _i32, _p, _p, _p, _p, _i64, _d, _p, _sz, _p]),
    "fb_hermite_steps_device_noalloc": (ctypes.c_int, [_i32, _i32, _p, _p, _p, _p, _i64, _d, _p]),
    "fb_eval_rsqrt": (ctypes.c_int, [_p, _p, _i64, _p]),
    "fb_integrate_steps": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbOpts)]),
    "fb_integrate_mvs": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbOpts)]),
    "fb_log_bytes": (_sz, [_i32, _p, _i32, _i32]),
    "fb_integrate_steps_logged": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbOpts),
                                                 ctypes.POINTER(FbLogSpec), _p]),
    "fb_integrate_to_times": (ctypes.c_int, [_p, _i32, _p, _d, ctypes.POINTER(FbOpts),
                                             ctypes.POINTER(FbLogSpec), _p]),
    "fb_integrate_rkck_steps": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbOpts)]),
    "fb_integrate_rkck": (ctypes.c_int, [_p, _d, _d, _d, ctypes.POINTER(FbOpts)]),
    "fb_integrate": (ctypes.c_int, [_p, _d, _d, ctypes.POINTER(FbOpts)]),
    "fb_synchronize": (ctypes.c_int, [_p]),
    "fb_get_state": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    "fb_get_hermite_state": (ctypes.c_int, [_p, _p, _p, _p]),
    "fb_diagnostics": (ctypes.c_int, [_p, _p, _p]),
    "fb_ensemble_shape": (ctypes.c_int, [_p, _p, _p]),
    "fb_ensemble_destroy": (ctypes.c_int, [_p]),
    "fb_set_plan": (ctypes.c_int, [_i32, _i32, _i32, _i32]),
    "fb_get_plan": (ctypes.c_int, [_i32, _p, _p, _p]),
    "fb_autotune": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(FbTuneEntry), _i32, ctypes.POINTER(_i32)]),
    "fb_profile_enable": (ctypes.c_int, [_i32]),
    "fb_profile_read": (ctypes.c_int, [_p, _p]),
    "fb_server_opts_default": (None, [ctypes.POINTER(FbServerOpts)]),
    "fb_server_create": (ctypes.c_int, [ctypes.POINTER(FbServerOpts), _p, ctypes.POINTER(_p)]),
    "fb_server_request_bytes": (_sz, [ctypes.POINTER(FbServerOpts), _i32, _p]),
    "fb_fp64_fma_ceiling": (ctypes.c_int, [_p]),
    "fb_lds_rates": (ctypes.c_int, [_p, _p]),
    "fb_server_submit": (ctypes.c_int, [_p, _i32, _p, _p, _p, _p, _d, _d, ctypes.POINTER(_i64)]),
    "fb_server_poll": (ctypes.c_int, [_p, _i64, ctypes.POINTER(_i32)]),
    "fb_server_wait": (ctypes.c_int, [_p, _i64, _d, ctypes.POINTER(_i32)]),
    "fb_server_result": (ctypes.c_int, [_p, _i64, _p, _p, _p, _p, _p, _p]),
    "fb_server_cancel": (ctypes.c_int, [_p, _i64]),
    "fb_server_release": (ctypes.c_int, [_p, _i64]),
    "fb_server_get_stats": (ctypes.c_int, [_p, ctypes.POINTER(FbServerStats)]),
    "fb_server_destroy": (ctypes.c_int, [_p]),
    "fb_monotonic_seconds": (_d, []),
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


def fp64_fma_ceiling() -> float:
    """Achievable FP64 FMA rate of the current device in TFLOP/s (fb_fp64_fma_ceiling)."""
    v = ctypes.c_double()
    _check(_lib.fb_fp64_fma_ceiling(ctypes.byref(v)))
    return v.value


def lds_rates():
    """LDS streaming rates of the current device per CU in GB/s, as
    (16-byte wavefront reads, 16-byte wavefront writes) (fb_lds_rates)."""
    r, w = ctypes.c_double(), ctypes.c_double()
    _check(_lib.fb_lds_rates(ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def profile_read():
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_lib.fb_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def eval_rsqrt(x):
    """The library's device reciprocal square root applied to a float64 CUDA
    tensor (fb_eval_rsqrt); returns a new tensor."""
    import torch
    x = x.contiguous()
    out = torch.empty_like(x)
    _check(_lib.fb_eval_rsqrt(_ptr(x), _ptr(out), int(x.numel()),
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    return out


def hermite_steps_device(n, mass, pos, vel, n_steps, dt, status=None, noalloc=False, workspace=None):
    """n_steps fixed Hermite steps of the systems of n bodies held in float64
    CUDA tensors mass [N], pos/vel [N, 3] (N = n_sys * n), in place, on
    torch's current stream (fb_hermite_steps_device, or with noalloc the
    allocation-free fb_hermite_steps_device_noalloc).  status: optional int32
    CUDA tensor [n_sys] for the systems' FB_SYS_* codes.  workspace: optional
    uint8 CUDA tensor (allocated here when None and noalloc is False)."""
    import torch
    for t_ in (mass, pos, vel):
        if not (isinstance(t_, torch.Tensor) and t_.is_cuda and t_.dtype == torch.float64
                and t_.is_contiguous()):
            raise FewbodyError(E_INVAL, "mass, pos and vel must be contiguous float64 CUDA tensors")
    N = int(mass.numel())
    if n < 2 or N % n or pos.numel() != 3 * N or vel.numel() != 3 * N:
        raise FewbodyError(E_INVAL, "pos/vel must hold 3 values per body and N a multiple of n")
    n_sys = N // n
    if status is not None and not (status.is_cuda and status.dtype == torch.int32
                                   and status.numel() == n_sys):
        raise FewbodyError(E_INVAL, "status must be an int32 CUDA tensor of n_sys entries")
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        _check(_lib.fb_hermite_steps_device_noalloc(n_sys, int(n), _ptr(mass), _ptr(pos), _ptr(vel),
                                                    _ptr(status), int(n_steps), float(dt), sp))
        return
    ws = int(_lib.fb_hermite_steps_workspace_bytes(n_sys, int(n)))
    if ws == 0 and n_sys > 0:
        raise FewbodyError(E_INVAL, "invalid batch shape")
    if workspace is None:
        workspace = torch.empty(ws + 256, dtype=torch.uint8, device=mass.device)
    addr = (workspace.data_ptr() + 255) // 256 * 256
    avail = workspace.numel() - (addr - workspace.data_ptr())
    _check(_lib.fb_hermite_steps_device(n_sys, int(n), _ptr(mass), _ptr(pos), _ptr(vel), _ptr(status),
                                        int(n_steps), float(dt), ctypes.c_void_p(addr),
                                        ctypes.c_size_t(max(avail, 0)), sp))


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

    def __init__(self, n_body, mass, pos, vel, t0=None, stream=None, host=False, checkpoint=None):
        import torch
        self._torch = torch
        self.n_body = np.ascontiguousarray(n_body, dtype=np.int32)
        self.n_sys = int(self.n_body.shape[0])
        self.n_bodies = int(self.n_body.sum())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._handle = ctypes.c_void_p()
        sp = ctypes.c_void_p(self.stream.cuda_stream)
        if checkpoint is not None:
            # fb_ensemble_restore: checkpoint holds acc, jerk, t, dt_next, status, steps
            m = np.ascontiguousarray(mass, dtype=np.float64)
            x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
            v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
            c = {k: checkpoint.get(k) for k in ("acc", "jerk", "t", "dt_next", "status", "steps")}
            arr = {
                "acc": np.ascontiguousarray(c["acc"], dtype=np.float64).reshape(-1, 3),
                "jerk": np.ascontiguousarray(c["jerk"], dtype=np.float64).reshape(-1, 3),
                "t": None if c["t"] is None else np.ascontiguousarray(c["t"], dtype=np.float64),
                "dt_next": None if c["dt_next"] is None else np.ascontiguousarray(c["dt_next"], dtype=np.float64),
                "status": None if c["status"] is None else np.ascontiguousarray(c["status"], dtype=np.int32),
                "steps": None if c["steps"] is None else np.ascontiguousarray(c["steps"], dtype=np.int64),
            }
            self._keep = None
            _check(_lib.fb_ensemble_restore(self.n_sys, _ptr(self.n_body), _ptr(m), _ptr(x), _ptr(v),
                                            _ptr(arr["acc"]), _ptr(arr["jerk"]), _ptr(arr["t"]),
                                            _ptr(arr["dt_next"]), _ptr(arr["status"]), _ptr(arr["steps"]),
                                            sp, ctypes.byref(self._handle)))
            return
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
            raise FewbodyError(E_INVAL, f"invalid body counts (each must be 2..{MAX_BODIES})")
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

    def integrate_steps_logged(self, n_steps, dt, every, kind=LOG_RV, los=(0.0, 0.0, 1.0),
                               opts: Opts | None = None, max_records=None, to_host=True):
        """fb_integrate_steps with a monitor that logs every `every` steps
        into a device buffer (torch-owned); returns the records on the host:
        LOG_RV -> (t, rv) [n_sys, R] each; LOG_ENERGY -> (t, E, L)
        [n_sys, R], [n_sys, R], [n_sys, R, 3]; LOG_STATE -> (t [n_sys, R],
        pos [R, N, 3], vel [R, N, 3]).  With to_host=False the call returns
        at once with (device buffer, records written), the records still in
        HBM in the layout fb_log_bytes describes."""
        if every < 1:
            raise FewbodyError(E_INVAL, "every must be >= 1")
        R = max_records or (1 + n_steps // every + (1 if n_steps % every else 0))
        buf, spec = self._log_buffer(kind, R, los, every)
        o = (opts or Opts()).c()
        n_rec = ctypes.c_int32()
        _check(_lib.fb_integrate_steps_logged(self._handle, int(n_steps), float(dt), ctypes.byref(o),
                                              ctypes.byref(spec), ctypes.byref(n_rec)))
        if not to_host:
            return buf, n_rec.value
        return self._read_log(buf, kind, R, n_rec.value)

    def integrate_to_times(self, t_obs, dt=0.0, kind=LOG_RV, los=(0.0, 0.0, 1.0),
                           opts: Opts | None = None, to_host=True):
        """fb_integrate_to_times: integrate to each time of t_obs in turn and
        record every system there; returns the records as
        integrate_steps_logged does (R = len(t_obs))."""
        t = np.ascontiguousarray(t_obs, dtype=np.float64).reshape(-1)
        R = max(int(t.shape[0]), 1)
        buf, spec = self._log_buffer(kind, R, los, 0)
        o = (opts or Opts()).c()
        n_rec = ctypes.c_int32()
        _check(_lib.fb_integrate_to_times(self._handle, int(t.shape[0]), _ptr(t), float(dt), ctypes.byref(o),
                                          ctypes.byref(spec), ctypes.byref(n_rec)))
        if not to_host:
            return buf, n_rec.value
        return self._read_log(buf, kind, R, n_rec.value)

    def _log_buffer(self, kind, R, los, every):
        torch = self._torch
        nb = self.n_body
        nbytes = int(_lib.fb_log_bytes(int(nb.shape[0]), _ptr(nb), int(kind), int(R)))
        if nbytes == 0 and self.n_sys > 0:
            raise FewbodyError(E_INVAL, "invalid log kind or record count")
        with torch.cuda.stream(self.stream):
            buf = torch.empty(max(nbytes, 8), dtype=torch.uint8,
                              device=torch.device("cuda", torch.cuda.current_device()))
        spec = FbLogSpec(int(kind), int(every), int(R), 0, (ctypes.c_double * 3)(*los),
                         ctypes.c_void_p(buf.data_ptr()), nbytes)
        return buf, spec

    def _read_log(self, buf, kind, R, k):
        self.synchronize()
        nb = self.n_body
        S = int(nb.shape[0])
        host = buf.cpu().numpy().view(np.float64)
        if kind == LOG_RV:
            a = host[:S * R * 2].reshape(S, R, 2)[:, :k]
            return a[..., 0], a[..., 1]
        if kind == LOG_ENERGY:
            a = host[:S * R * 5].reshape(S, R, 5)[:, :k]
            return a[..., 0], a[..., 1], a[..., 2:5]
        off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
        N = int(off[-1])
        t = np.empty((S, k))
        pos = np.empty((k, N, 3))
        vel = np.empty((k, N, 3))
        for o_ in range(S):
            n = int(nb[o_])
            base = R * (o_ + 6 * int(off[o_]))
            blk = host[base:base + R * (1 + 6 * n)].reshape(R, 1 + 6 * n)[:k]
            t[o_] = blk[:, 0]
            pos[:, off[o_]:off[o_ + 1]] = blk[:, 1:1 + 3 * n].reshape(k, n, 3)
            vel[:, off[o_]:off[o_ + 1]] = blk[:, 1 + 3 * n:].reshape(k, n, 3)
        return t, pos, vel

    def integrate_mvs(self, n_steps, dt, opts: Opts | None = None):
        """n_steps fixed steps of the mixed-variable symplectic integrator
        (fb_integrate_mvs; systems of at most MAX_MVS_BODIES bodies)."""
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate_mvs(self._handle, int(n_steps), float(dt), ctypes.byref(o)))

    def integrate_rkck_steps(self, n_steps, dt, opts: Opts | None = None):
        """n_steps fixed Runge-Kutta Cash-Karp steps (fb_integrate_rkck_steps)."""
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate_rkck_steps(self._handle, int(n_steps), float(dt), ctypes.byref(o)))

    def integrate_rkck(self, t_end, dt, eps, opts: Opts | None = None):
        """Adaptive Runge-Kutta Cash-Karp to t_end, first trial step dt,
        tolerance eps (fb_integrate_rkck)."""
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate_rkck(self._handle, float(t_end), float(dt), float(eps), ctypes.byref(o)))

    def integrate(self, t_end, dt=0.0, opts: Opts | None = None):
        o = (opts or Opts()).c()
        _check(_lib.fb_integrate(self._handle, float(t_end), float(dt), ctypes.byref(o)))

    def synchronize(self):
        _check(_lib.fb_synchronize(self._handle))

    def autotune(self, steps, dt):
        """Time the candidate plans on this ensemble and install the fastest
        (state restored afterwards).  Returns every timed candidate."""
        buf = (FbTuneEntry * 512)()
        n = ctypes.c_int32()
        _check(_lib.fb_autotune(self._handle, int(steps), float(dt), buf, 512, ctypes.byref(n)))
        return [{k: getattr(buf[i], k) for k, _ in FbTuneEntry._fields_ if k != "pad"}
                for i in range(min(n.value, 512))]

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

    def checkpoint(self):
        """Everything fb_ensemble_restore needs to continue this ensemble
        bitwise: masses are the caller's; returns dict(pos, vel, acc, jerk,
        t, dt_next, status, steps)."""
        st = self.state()
        acc, jerk, dtn = self.hermite_state()
        return {"pos": st["pos"], "vel": st["vel"], "acc": acc, "jerk": jerk, "t": st["t"],
                "dt_next": dtn, "status": st["status"], "steps": st["steps"]}

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


def monotonic() -> float:
    """The library's monotonic clock (CLOCK_MONOTONIC seconds, as time.monotonic())."""
    return _lib.fb_monotonic_seconds()


def server_opts(budget_bytes=0, max_resident=0, steps_per_quantum=0, policy=POLICY_FAIR,
                quantum_tiles=0, chunk_slots=0, long_steps=0, idle_spread=0) -> FbServerOpts:
    return FbServerOpts(int(budget_bytes), int(max_resident), int(steps_per_quantum), int(policy),
                        int(quantum_tiles), int(chunk_slots), int(long_steps), int(idle_spread))


def server_request_bytes(n_body, **opts) -> int:
    """Device bytes a request of these body counts needs on an empty server."""
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    o = server_opts(**opts)
    return int(_lib.fb_server_request_bytes(ctypes.byref(o), int(nb.shape[0]), _ptr(nb)))


class Server:
    """Continuous-batching integration server (fb_server_*).

    submit() queues an ensemble with its own t_end and fixed dt and returns
    at once; a native worker thread admits requests by device-memory budget
    and resident cap, advances every resident system in fused quanta, and
    retires finished requests."""

    def __init__(self, budget_bytes=0, max_resident=0, steps_per_quantum=0, stream=None,
                 policy=POLICY_FAIR, quantum_tiles=0, chunk_slots=0, long_steps=0, idle_spread=0):
        o = server_opts(budget_bytes, max_resident, steps_per_quantum, policy, quantum_tiles,
                        chunk_slots, long_steps, idle_spread)
        self._h = ctypes.c_void_p()
        sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(_lib.fb_server_create(ctypes.byref(o), sp, ctypes.byref(self._h)))
        self._shapes = {}

    def submit(self, n_body, mass, pos, vel, t_end, dt) -> int:
        nb = np.ascontiguousarray(n_body, dtype=np.int32)
        m = np.ascontiguousarray(mass, dtype=np.float64)
        x = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        rid = ctypes.c_int64()
        _check(_lib.fb_server_submit(self._h, int(nb.shape[0]), _ptr(nb), _ptr(m), _ptr(x), _ptr(v),
                                     float(t_end), float(dt), ctypes.byref(rid)))
        self._shapes[rid.value] = (int(nb.shape[0]), int(m.shape[0]))
        return rid.value

    def submit_gen(self, ens, t_end, dt) -> int:
        return self.submit(ens.n_body, ens.mass, ens.pos, ens.vel, t_end, dt)

    def poll(self, rid) -> int:
        st = ctypes.c_int32()
        _check(_lib.fb_server_poll(self._h, int(rid), ctypes.byref(st)))
        return st.value

    def wait(self, rid, timeout=-1.0) -> int:
        st = ctypes.c_int32()
        _check(_lib.fb_server_wait(self._h, int(rid), float(timeout), ctypes.byref(st)))
        return st.value

    def result(self, rid):
        if rid not in self._shapes:   # read or released already (or never submitted here)
            self.poll(rid)
            raise FewbodyError(E_NOTFOUND, f"request {rid} has no result to read here")
        S, N = self._shapes.pop(rid)
        pos, vel = np.empty((N, 3)), np.empty((N, 3))
        t = np.empty(S)
        status = np.empty(S, dtype=np.int32)
        steps = np.empty(S, dtype=np.int64)
        times = np.empty(3)
        _check(_lib.fb_server_result(self._h, int(rid), _ptr(pos), _ptr(vel), _ptr(t), _ptr(status),
                                     _ptr(steps), _ptr(times)))
        return {"pos": pos, "vel": vel, "t": t, "status": status, "steps": steps,
                "t_submit": times[0], "t_admit": times[1], "t_done": times[2]}

    def cancel(self, rid):
        _check(_lib.fb_server_cancel(self._h, int(rid)))

    def release(self, rid):
        _check(_lib.fb_server_release(self._h, int(rid)))
        self._shapes.pop(rid, None)

    def stats(self) -> dict:
        st = FbServerStats()
        _check(_lib.fb_server_get_stats(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in FbServerStats._fields_}

    def close(self):
        if self._h:
            _check(_lib.fb_server_destroy(self._h))
            self._h = ctypes.c_void_p()

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


def log_bytes(n_body, kind, max_records) -> int:
    nb = np.ascontiguousarray(n_body, dtype=np.int32)
    return int(_lib.fb_log_bytes(int(nb.shape[0]), _ptr(nb), int(kind), int(max_records)))
