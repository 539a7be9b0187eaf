"""ctypes binding of include/hsma.h and include/hsma_debug.h.

Argument marshalling only.  The shared library must have been built
(`python -m paper_2104_05260_amd.build` or `__graft_entry__.build()`);
there is no fallback: a missing library raises at load time.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libhsma.so")

STATUS = {
    0: "HSMA_OK", -1: "HSMA_ERR_INVALID_ARG", -2: "HSMA_ERR_NOT_NEUTRAL", -3: "HSMA_ERR_OUT_OF_DOMAIN",
    -4: "HSMA_ERR_GEOMETRY", -5: "HSMA_ERR_RANK", -6: "HSMA_ERR_NO_DEVICE", -7: "HSMA_ERR_OOM",
    -8: "HSMA_ERR_DEVICE", -9: "HSMA_ERR_BUSY", -10: "HSMA_ERR_CANCELLED",
}
GEOM_3D, GEOM_2D = 0, 1
FP64, FP32C = 0, 1


class HSMAError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class _CParams(ctypes.Structure):
    _fields_ = [
        ("geometry", ctypes.c_int), ("precision", ctypes.c_int), ("lambda_", ctypes.c_double),
        ("p", ctypes.c_int), ("K", ctypes.c_int), ("F", ctypes.c_int), ("Fw", ctypes.c_int),
        ("surface_rule", ctypes.c_int), ("near_rule", ctypes.c_int), ("M", ctypes.c_int),
        ("gamma_up", ctypes.c_double),
        ("gamma_low", ctypes.c_double), ("nz", ctypes.c_int), ("coulomb_k", ctypes.c_double),
        ("tree_order", ctypes.c_int), ("tree_theta", ctypes.c_double), ("lsq_solver", ctypes.c_int),
    ]


class _CInfo(ctypes.Structure):
    _fields_ = [
        ("nb", ctypes.c_int), ("n_rows", ctypes.c_int), ("n_check", ctypes.c_int), ("n_desc", ctypes.c_int),
        ("radius", ctypes.c_double), ("cond", ctypes.c_double), ("near_pairs", ctypes.c_int64),
        ("check_pairs", ctypes.c_int64), ("surface_pairs", ctypes.c_int64),
    ]


class _CTiming(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int64), ("step_ms", ctypes.c_double), ("check_ms", ctypes.c_double),
                ("near_ms", ctypes.c_double), ("sphere_ms", ctypes.c_double)]


class _CClass(ctypes.Structure):
    _fields_ = [("params", _CParams), ("box_len", ctypes.c_double * 3)]


class _CServerCfg(ctypes.Structure):
    _fields_ = [("params", _CParams), ("box_len", ctypes.c_double * 3), ("max_n", ctypes.c_int64),
                ("max_slots", ctypes.c_int), ("hbm_budget", ctypes.c_int64), ("queue_capacity", ctypes.c_int),
                ("n_classes", ctypes.c_int), ("classes", ctypes.POINTER(_CClass))]


REQ_DEVICE = 1


class _CRequest(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("xyz", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("box_lo", ctypes.c_double * 3), ("box_len", ctypes.c_double * 3), ("scale", ctypes.c_double),
                ("params", ctypes.POINTER(_CParams)), ("potential", ctypes.c_void_p), ("force", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("flags", ctypes.c_int), ("system_id", ctypes.c_uint64),
                ("ready_event", ctypes.c_void_p)]


class _CResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("energy", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double), ("slot", ctypes.c_int),
                ("replayed", ctypes.c_int), ("plan_class", ctypes.c_int)]


class _CMDParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("lj_epsilon", ctypes.c_double), ("lj_sigma", ctypes.c_double),
                ("lj_rcut", ctypes.c_double), ("wall_epsilon", ctypes.c_double), ("wall_sigma", ctypes.c_double),
                ("wall_rcut", ctypes.c_double), ("nh_kT", ctypes.c_double), ("nh_damping", ctypes.c_double),
                ("respa_inner", ctypes.c_int)]


class _CServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("graph_replays", ctypes.c_int64), ("affinity_hits", ctypes.c_int64),
                ("classes", ctypes.c_int), ("slots", ctypes.c_int)]


@dataclass
class Params:
    geometry: int = GEOM_3D
    precision: int = FP32C
    lam: float = 1.5
    p: int = 10
    K: int = 242
    F: int = 800
    Fw: int = 0
    surface_rule: int = 0
    near_rule: int = 0
    M: int = 10
    gamma_up: float = 0.0
    gamma_low: float = 0.0
    nz: int = 80
    coulomb_k: float = 1.0
    tree_order: int = 12
    tree_theta: float = 0.5
    lsq_solver: int = 0

    @staticmethod
    def from_workload(w, precision: Optional[int] = None) -> "Params":
        return Params(geometry=w.geometry, precision=w.precision if precision is None else precision,
                      lam=w.lam, p=w.p, K=w.K, F=w.F, Fw=w.Fw, surface_rule=w.surface_rule,
                      near_rule=w.near_rule, M=w.M, gamma_up=w.gamma_up, gamma_low=w.gamma_low, nz=w.nz)

    def _c(self) -> _CParams:
        return _CParams(self.geometry, self.precision, self.lam, self.p, self.K, self.F, self.Fw,
                        self.surface_rule, self.near_rule, self.M, self.gamma_up, self.gamma_low, self.nz,
                        self.coulomb_k, self.tree_order, self.tree_theta, self.lsq_solver)


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def _hip_runtimes_mapped():
    try:
        with open("/proc/self/maps") as f:
            maps = f.read()
    except OSError:
        return set()
    import re
    return set(re.findall(r"(/\S*libamdhip64\S*)", maps))


def load_library():
    """Loads libhsma.so once per process.

    PyTorch ships its own HIP runtime.  Importing torch first makes the
    library bind to that same runtime (one HIP runtime per process), so
    torch tensors and streams can be handed to the device entry points."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2104_05260_amd.build`")
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime before ours)
    except ImportError:
        pass
    lib = ctypes.CDLL(_LIB_PATH)
    rts = _hip_runtimes_mapped()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are loaded in this process: {sorted(rts)}")
    d, i64, vp = ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_void_p
    lib.hsma_params_default.argtypes = [ctypes.POINTER(_CParams)]
    lib.hsma_plan_create.argtypes = [ctypes.POINTER(_CParams), d, d, ctypes.POINTER(vp)]
    lib.hsma_plan_destroy.argtypes = [vp]
    lib.hsma_compute.argtypes = [vp, i64, d, d, d, d, d]
    lib.hsma_compute_device.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.hsma_compute_device_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    lib.hsma_plan_device_status.argtypes = [vp]
    lib.hsma_plan_get_info.argtypes = [vp, ctypes.POINTER(_CInfo)]
    lib.hsma_last_error.restype = ctypes.c_char_p
    lib.hsma_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.hsma_plan_set_graph.argtypes = [vp, ctypes.c_int]
    lib.hsma_plan_get_timing.argtypes = [vp, ctypes.POINTER(_CTiming)]
    lib.hsma_debug_solid_harmonics.argtypes = [ctypes.c_int, d, d, d]
    lib.hsma_debug_host_plan_create.argtypes = [ctypes.POINTER(_CParams), d, d, ctypes.POINTER(vp)]
    lib.hsma_debug_host_plan_destroy.argtypes = [vp]
    lib.hsma_debug_host_plan_get.argtypes = [vp, ctypes.c_char_p, d, i64]
    lib.hsma_debug_host_plan_get.restype = i64
    lib.hsma_server_create.argtypes = [ctypes.POINTER(_CServerCfg), ctypes.POINTER(vp)]
    lib.hsma_server_submit.argtypes = [vp, ctypes.POINTER(_CRequest), ctypes.POINTER(ctypes.c_uint64)]
    lib.hsma_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(_CResult)]
    lib.hsma_server_get_slots.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64)]
    lib.hsma_server_get_stats.argtypes = [vp, ctypes.POINTER(_CServerStats)]
    lib.hsma_md_create.argtypes = [vp, ctypes.POINTER(_CMDParams), i64, ctypes.POINTER(vp)]
    lib.hsma_md_run.argtypes = [vp, vp, ctypes.c_int, vp, vp, vp, vp, vp, ctypes.c_int, vp]
    lib.hsma_md_forces.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hsma_md_destroy.argtypes = [vp]
    lib.hsma_md_create_for_box.argtypes = [ctypes.POINTER(_CMDParams), ctypes.c_int, d, d, i64, ctypes.POINTER(vp)]
    lib.hsma_md_drift.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.hsma_md_finish.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hsma_md_thermostat.argtypes = [vp, vp, vp]
    lib.hsma_md_short_range.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hsma_md_rdf.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.c_double, vp]
    lib.hsma_md_zprofile.argtypes = [vp, vp, vp, vp, ctypes.c_int, vp]
    for name in ("hsma_md_create", "hsma_md_run", "hsma_md_forces", "hsma_md_create_for_box", "hsma_md_drift",
                 "hsma_md_finish", "hsma_md_thermostat", "hsma_md_rdf", "hsma_md_zprofile", "hsma_md_short_range"):
        getattr(lib, name).restype = ctypes.c_int
    lib.hsma_server_get_stats.restype = ctypes.c_int
    lib.hsma_server_destroy.argtypes = [vp]
    lib.hsma_server_shutdown.argtypes = [vp]
    for name in ("hsma_server_create", "hsma_server_submit", "hsma_server_wait", "hsma_server_get_slots"):
        getattr(lib, name).restype = ctypes.c_int
    lib.hsma_debug_hilbert_key.argtypes = [ctypes.c_uint32] * 3
    lib.hsma_debug_hilbert_key.restype = ctypes.c_uint32
    for name in ("hsma_plan_create", "hsma_compute", "hsma_compute_device", "hsma_compute_device_noalloc",
                 "hsma_plan_device_status",
                 "hsma_plan_get_info", "hsma_debug_solid_harmonics", "hsma_plan_set_timing", "hsma_plan_get_timing", "hsma_plan_set_graph", "hsma_debug_host_plan_create"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int):
    if st != 0:
        raise HSMAError(st, load_library().hsma_last_error().decode())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec3(v):
    a = np.ascontiguousarray(v, dtype=np.float64).reshape(3)
    return a


def solid_harmonics(p: int, xi, grad: bool = False):
    lib = load_library()
    x = _vec3(xi)
    nb = (p + 1) ** 2 - 1
    val = np.zeros(nb)
    g = np.zeros((nb, 3)) if grad else None
    _check(lib.hsma_debug_solid_harmonics(p, _dp(x), _dp(val), _dp(g)))
    return (val, g) if grad else val


def hilbert_key(x: int, y: int, z: int) -> int:
    return int(load_library().hsma_debug_hilbert_key(x, y, z))


class HostPlan:
    """Host-only part of a plan (no GPU needed), for tests."""

    def __init__(self, params: Params, box_lo, box_len):
        lib = load_library()
        self._lib = lib
        self._h = ctypes.c_void_p()
        lo, L = _vec3(box_lo), _vec3(box_len)
        cp = params._c()
        _check(lib.hsma_debug_host_plan_create(ctypes.byref(cp), _dp(lo), _dp(L), ctypes.byref(self._h)))

    def get(self, name: str) -> np.ndarray:
        n = self._lib.hsma_debug_host_plan_get(self._h, name.encode(), None, 0)
        if n < 0:
            raise KeyError(name)
        out = np.zeros(n)
        self._lib.hsma_debug_host_plan_get(self._h, name.encode(), _dp(out), n)
        return out

    def close(self):
        if self._h:
            self._lib.hsma_debug_host_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A device plan for one box and parameter set (hsma_plan_create)."""

    def __init__(self, params: Params, box_lo, box_len):
        lib = load_library()
        self._lib = lib
        self.params = params
        self._p = ctypes.c_void_p()
        lo, L = _vec3(box_lo), _vec3(box_len)
        cp = params._c()
        _check(lib.hsma_plan_create(ctypes.byref(cp), _dp(lo), _dp(L), ctypes.byref(self._p)))

    def compute(self, xyz, q, energy=True, potential=True, force=True):
        """Host arrays in, (energy, potential, force) out (hsma_compute)."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        if qq.shape[0] != x.shape[0]:
            raise ValueError("positions and charges differ in length")
        n = x.shape[0]
        e = np.zeros(1) if energy else None
        pot = np.zeros(n) if potential else None
        f = np.zeros((n, 3)) if force else None
        _check(self._lib.hsma_compute(self._p, n, _dp(x), _dp(qq), _dp(e), _dp(pot), _dp(f)))
        return (float(e[0]) if energy else None), pot, f

    def compute_device(self, xyz, q, energy=None, potential=None, force=None, stream=None):
        """Device tensors in/out (hsma_compute_device); asynchronous on
        `stream` (default: torch's current stream).  Arguments are torch
        tensors of dtype float64 on the plan's device."""
        import torch
        n = xyz.shape[0]
        for t in (xyz, q, energy, potential, force):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda):
                raise ValueError("device arguments must be contiguous float64 GPU tensors")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _check(self._lib.hsma_compute_device(self._p, ctypes.c_void_p(stream), n, ptr(xyz), ptr(q),
                                             ptr(energy), ptr(potential), ptr(force)))

    def compute_device_noalloc(self, xyz, q, energy=None, potential=None, force=None, stream=None):
        """As compute_device, through hsma_compute_device_noalloc (per-call
        working memory from the library's static scratch; n <= 16384)."""
        import torch
        n = xyz.shape[0]
        for t in (xyz, q, energy, potential, force):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda):
                raise ValueError("device arguments must be contiguous float64 GPU tensors")
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
        _check(self._lib.hsma_compute_device_noalloc(self._p, ctypes.c_void_p(stream), n, ptr(xyz), ptr(q),
                                                     ptr(energy), ptr(potential), ptr(force)))

    def device_status(self) -> int:
        st = self._lib.hsma_plan_device_status(self._p)
        return st

    def set_graph(self, enable: bool = True):
        _check(self._lib.hsma_plan_set_graph(self._p, 1 if enable else 0))

    def set_timing(self, enable: bool = True):
        _check(self._lib.hsma_plan_set_timing(self._p, 1 if enable else 0))

    def timing(self) -> dict:
        t = _CTiming()
        _check(self._lib.hsma_plan_get_timing(self._p, ctypes.byref(t)))
        return {f[0]: getattr(t, f[0]) for f in _CTiming._fields_}

    def info(self) -> dict:
        inf = _CInfo()
        _check(self._lib.hsma_plan_get_info(self._p, ctypes.byref(inf)))
        return {f[0]: getattr(inf, f[0]) for f in _CInfo._fields_}

    def close(self):
        if self._p:
            self._lib.hsma_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (hsma_server_*): requests with their own
    parameters and boxes (plan classes), host or device-resident."""

    def __init__(self, params: Params, box_len, max_n: int, max_slots: int = 8, hbm_budget: int = 0,
                 queue_capacity: int = 0, classes=()):
        lib = load_library()
        self._lib = lib
        self._s = ctypes.c_void_p()
        cfg = _CServerCfg()
        cfg.params = params._c()
        for k in range(3):
            cfg.box_len[k] = float(box_len[k])
        cfg.max_n = int(max_n)
        cfg.max_slots = int(max_slots)
        cfg.hbm_budget = int(hbm_budget)
        cfg.queue_capacity = int(queue_capacity)
        arr = (_CClass * max(1, len(classes)))()
        for i, (pp, bl) in enumerate(classes):
            arr[i].params = pp._c()
            for k in range(3):
                arr[i].box_len[k] = float(bl[k])
        cfg.n_classes = len(classes)
        cfg.classes = ctypes.cast(arr, ctypes.POINTER(_CClass)) if classes else None
        _check(lib.hsma_server_create(ctypes.byref(cfg), ctypes.byref(self._s)))
        self._keep = {}

    def slots(self):
        n, b = ctypes.c_int(), ctypes.c_int64()
        _check(self._lib.hsma_server_get_slots(self._s, ctypes.byref(n), ctypes.byref(b)))
        return n.value, b.value

    def stats(self) -> dict:
        st = _CServerStats()
        _check(self._lib.hsma_server_get_stats(self._s, ctypes.byref(st)))
        return {f[0]: getattr(st, f[0]) for f in _CServerStats._fields_}

    @staticmethod
    def _box(r, box_lo, scale, box_len):
        for k in range(3):
            r.box_lo[k] = float(box_lo[k])
            r.box_len[k] = float(box_len[k]) if box_len is not None else 0.0
        r.scale = float(scale) if scale is not None else 0.0

    def submit(self, xyz, q, box_lo, scale: float = None, potential: bool = True, force: bool = True,
               box_len=None, params: Params = None, system_id: int = 0) -> int:
        """Host arrays in; results returned by wait()."""
        x = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        qq = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        n = x.shape[0]
        pot = np.zeros(n) if potential else None
        f = np.zeros((n, 3)) if force else None
        r = _CRequest()
        r.n = n
        r.xyz = x.ctypes.data
        r.q = qq.ctypes.data
        self._box(r, box_lo, scale, box_len)
        cp = params._c() if params is not None else None
        r.params = ctypes.pointer(cp) if cp is not None else None
        r.potential = pot.ctypes.data if pot is not None else None
        r.force = f.ctypes.data if f is not None else None
        r.system_id = int(system_id)
        t = ctypes.c_uint64()
        _check(self._lib.hsma_server_submit(self._s, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (x, qq, pot, f)
        return t.value

    def submit_device(self, xyz, q, box_lo, scale: float = None, potential=None, force=None, energy=None,
                      box_len=None, params: Params = None, system_id: int = 0, ready_event=None) -> int:
        """Device-resident request: torch float64 tensors on the GPU, read and
        written in place by the step (HSMA_REQ_DEVICE)."""
        import torch
        for t in (xyz, q, potential, force, energy):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda):
                raise ValueError("device arguments must be contiguous float64 GPU tensors")
        r = _CRequest()
        r.n = xyz.shape[0]
        r.xyz = xyz.data_ptr()
        r.q = q.data_ptr()
        self._box(r, box_lo, scale, box_len)
        cp = params._c() if params is not None else None
        r.params = ctypes.pointer(cp) if cp is not None else None
        r.potential = potential.data_ptr() if potential is not None else None
        r.force = force.data_ptr() if force is not None else None
        r.energy = energy.data_ptr() if energy is not None else None
        r.flags = REQ_DEVICE
        r.system_id = int(system_id)
        r.ready_event = ready_event.cuda_event if ready_event is not None else None
        t = ctypes.c_uint64()
        _check(self._lib.hsma_server_submit(self._s, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (xyz, q, potential, force)
        return t.value

    def wait(self, ticket: int) -> dict:
        res = _CResult()
        st = self._lib.hsma_server_wait(self._s, ctypes.c_uint64(ticket), ctypes.byref(res))
        _, _, pot, f = self._keep.pop(ticket, (None, None, None, None))
        out = {k[0]: getattr(res, k[0]) for k in _CResult._fields_}
        out["status_name"] = STATUS.get(st, str(st))
        out["potential"], out["force"] = pot, f
        return out

    def shutdown(self):
        """Cancel queued requests, finish admitted ones; wait() still works."""
        if self._s:
            self._lib.hsma_server_shutdown(self._s)

    def close(self):
        if self._s:
            self._lib.hsma_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MD:
    """Velocity-Verlet MD with HSMA electrostatics (hsma_md_*): device
    tensors (float64, contiguous) are integrated in place."""

    def __init__(self, plan: Optional["Plan"], n: int, dt: float, lj_epsilon: float = 1.0, lj_sigma: float = 1.0,
                 lj_rcut: float = 0.0, wall_epsilon: float = 0.0, wall_sigma: float = 1.0, wall_rcut: float = 0.0,
                 geometry: int = GEOM_3D, box_lo=None, box_len=None, nh_kT: float = 0.0, nh_damping: float = 0.0,
                 respa_inner: int = 0):
        """With a plan: hsma_md_create.  With plan None: a driver for the
        box (hsma_md_create_for_box) whose Coulomb forces come from
        elsewhere (drift / finish around a server request)."""
        lib = load_library()
        self._lib = lib
        self._plan = plan  # kept alive: the driver uses it
        self._m = ctypes.c_void_p()
        p = _CMDParams(dt, lj_epsilon, lj_sigma, lj_rcut, wall_epsilon, wall_sigma, wall_rcut, nh_kT, nh_damping,
                       int(respa_inner))
        if plan is not None:
            _check(lib.hsma_md_create(plan._p, ctypes.byref(p), int(n), ctypes.byref(self._m)))
        else:
            lo, L = _vec3(box_lo), _vec3(box_len)
            _check(lib.hsma_md_create_for_box(ctypes.byref(p), int(geometry), _dp(lo), _dp(L), int(n),
                                              ctypes.byref(self._m)))

    @staticmethod
    def _ptr(t):
        import torch
        if t is None:
            return None
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("device arguments must be contiguous float64 GPU tensors")
        return ctypes.c_void_p(t.data_ptr())

    def run(self, x, v, f, q, m, nsteps: int, forces_valid: bool = False, thermo=None, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_run(self._m, ctypes.c_void_p(stream), int(nsteps), self._ptr(x), self._ptr(v),
                                     self._ptr(f), self._ptr(q), self._ptr(m), 1 if forces_valid else 0,
                                     self._ptr(thermo)))

    def forces(self, x, v, f, q, m, thermo_row=None, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_forces(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(v), self._ptr(f),
                                        self._ptr(q), self._ptr(m), self._ptr(thermo_row)))

    def drift(self, x, v, f, m, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_drift(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(v), self._ptr(f),
                                       self._ptr(m)))

    def finish(self, x, v, f, m, e_coulomb, thermo_row=None, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_finish(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(v), self._ptr(f),
                                        self._ptr(m), self._ptr(e_coulomb), self._ptr(thermo_row)))

    def short_range(self, x, v, f, m, e_coulomb, thermo_row=None, stream=None):
        """F += F_LJ at x and one thermo row, no kick, no thermostat: the
        start of a run whose Coulomb forces came from elsewhere
        (hsma_md_short_range)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_short_range(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(v),
                                             self._ptr(f), self._ptr(m), self._ptr(e_coulomb),
                                             self._ptr(thermo_row)))

    def thermostat(self, state, stream=None):
        """Copies the thermostat's (xi, eta, energy) into `state`, a float64
        GPU tensor of 3 entries (hsma_md_thermostat)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(self._lib.hsma_md_thermostat(self._m, ctypes.c_void_p(stream), self._ptr(state)))

    @staticmethod
    def _hist_ptr(t):
        import torch
        if t.dtype != torch.int64 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError("histograms must be contiguous int64 GPU tensors")
        return ctypes.c_void_p(t.data_ptr())

    def rdf(self, x, q, r_max: float, hist, stream=None):
        """Adds the pair-distance counts of configuration x to `hist`, an
        int64 GPU tensor of shape (3, nbins): classes (+,+), (+,-), (-,-)
        (hsma_md_rdf)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        if hist.dim() != 2 or hist.shape[0] != 3:
            raise ValueError("hist must have shape (3, nbins)")
        _check(self._lib.hsma_md_rdf(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(q),
                                     int(hist.shape[1]), float(r_max), self._hist_ptr(hist)))

    def zprofile(self, x, q, hist, stream=None):
        """Adds the z-density counts of configuration x to `hist`, an int64
        GPU tensor of shape (2, nbins): q > 0 and q < 0 (hsma_md_zprofile)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        if hist.dim() != 2 or hist.shape[0] != 2:
            raise ValueError("hist must have shape (2, nbins)")
        _check(self._lib.hsma_md_zprofile(self._m, ctypes.c_void_p(stream), self._ptr(x), self._ptr(q),
                                          int(hist.shape[1]), self._hist_ptr(hist)))

    def close(self):
        if self._m:
            self._lib.hsma_md_destroy(self._m)
            self._m = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ReplicaEnsemble:
    """MD replicas on the serving loop: every replica's state stays on the
    device; per step each replica drifts (hsma_md_drift), its Coulomb forces
    come from a device request to the server (in place, with its system id,
    so its slot replays a captured step), then it finishes the step
    (hsma_md_finish: LJ, kick, thermo).  Orchestration of C-ABI calls only."""

    def __init__(self, server: "Server", replicas, dt: float, params: Params = None, **lj):
        """replicas: list of dicts with device tensors x, v, q, m and box_lo,
        box_len (3D boxes)."""
        import torch
        self.server = server
        self.params = params
        self.reps = []
        for i, r in enumerate(replicas):
            n = r["x"].shape[0]
            dev = r["x"].device
            md = MD(None, n, dt, box_lo=r["box_lo"], box_len=r["box_len"], **lj)
            self.reps.append(dict(r, md=md, f=torch.zeros_like(r["x"]), e=torch.zeros(1, dtype=torch.float64, device=dev),
                                  ev=torch.cuda.Event(), id=i + 1))
        self.first = True

    def _coulomb(self):
        import torch
        tickets = []
        for r in self.reps:
            r["ev"].record()
            tickets.append(self.server.submit_device(r["x"], r["q"], r["box_lo"], box_len=r["box_len"],
                                                     params=self.params, force=r["f"], energy=r["e"],
                                                     system_id=r["id"], ready_event=r["ev"]))
        return [self.server.wait(t) for t in tickets]

    def step(self, thermo=None):
        """One step of every replica; thermo: optional list of 4-double
        device tensors, one per replica.  Returns the server results."""
        if self.first:
            res = self._coulomb()  # forces at the starting positions
            for r in self.reps:
                r["md"].short_range(r["x"], r["v"], r["f"], r["m"], r["e"])
            self.first = False
        for r in self.reps:
            r["md"].drift(r["x"], r["v"], r["f"], r["m"])
        res = self._coulomb()
        for k, r in enumerate(self.reps):
            r["md"].finish(r["x"], r["v"], r["f"], r["m"], r["e"], None if thermo is None else thermo[k])
        return res

    def close(self):
        for r in self.reps:
            r["md"].close()
