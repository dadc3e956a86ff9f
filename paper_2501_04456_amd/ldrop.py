"""Thin Python binding of libldrop (include/ldrop.h).

Argument marshalling only: every step of the model runs in the HIP library.
PyTorch supplies device memory (output tensors) and the HIP stream.  The
library is loaded from this package directory; if it is missing, or no GPU
is visible, construction fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
# LDROP_LIB may name another build of the same library (e.g. to compare two
# builds in one process tree); the default is the in-tree build.
LIB_PATH = os.environ.get("LDROP_LIB") or os.path.join(_HERE, "libldrop.so")
MAX_TYPES = 8

LD_OK = 0
_STATUS = {0: "LD_OK", -1: "LD_EINVAL", -2: "LD_ENOMEM", -3: "LD_EHIP", -4: "LD_ENONFINITE",
           -5: "LD_ESTATE", -6: "LD_EUNSUPPORTED"}


class LdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class NonFinite(LdError):
    pass


class ld_params(C.Structure):
    _fields_ = [
        ("n_types", C.c_int32), ("use_eps_matrix", C.c_int32),
        ("sigma", C.c_double * MAX_TYPES), ("eps", C.c_double * MAX_TYPES),
        ("mass", C.c_double * MAX_TYPES), ("gamma", C.c_double * MAX_TYPES),
        ("k_wall", C.c_double * MAX_TYPES), ("wall_offset", C.c_double * MAX_TYPES),
        ("eps_matrix", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("lj_cut", C.c_double), ("coul_cut", C.c_double), ("bjerrum", C.c_double),
        ("kT", C.c_double), ("gravity", C.c_double * 3), ("omega", C.c_double),
        ("rotation", C.c_int32), ("wall_band", C.c_int32), ("noise", C.c_int32),
        ("reserved", C.c_int32), ("jump_max", C.c_double),
    ]


class ld_radius(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_knots", C.c_int32), ("R0", C.c_double),
                ("R1", C.c_double), ("T", C.c_double), ("a", C.c_double),
                ("R_min", C.c_double), ("tab_t", C.c_double * W.RADIUS_TABLE_MAX),
                ("tab_R", C.c_double * W.RADIUS_TABLE_MAX)]


class ld_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("j_split", C.c_int32), ("comp", C.c_int32),
                ("sort_every", C.c_int32), ("cull", C.c_int32), ("graph_steps", C.c_int32),
                ("reserved", C.c_int32 * 2)]


TUNING_FIELDS = ("block", "j_split", "comp", "sort_every", "cull", "graph_steps")


class ld_ff_config(C.Structure):
    _fields_ = [("near_cut", C.c_double), ("grid", C.c_int32), ("block", C.c_int32),
                ("hidden", C.c_int32), ("judge_every", C.c_int32), ("judge_tol", C.c_double),
                ("near_mode", C.c_int32), ("parent_reach", C.c_int32)]


class ld_ff_train_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("seed", C.c_uint64), ("val_fraction", C.c_double), ("reset_scale", C.c_int32),
                ("calibrate", C.c_int32)]


class ld_ff_train_report(C.Structure):
    _fields_ = [("samples", C.c_int64), ("iterations", C.c_int64), ("final_loss", C.c_double),
                ("val_rel_rms", C.c_double), ("out_scale", C.c_double), ("gain", C.c_double),
                ("val_rel_rms_raw", C.c_double)]


class ld_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("R", C.c_double),
                ("U", C.c_double * 5), ("net_force", C.c_double * 3), ("max_force", C.c_double),
                ("max_radius", C.c_double), ("msd", C.c_double), ("bad_step", C.c_int64)]


class ld_paper_config(C.Structure):
    _fields_ = [("range_factor", C.c_double), ("kick", C.c_double),
                ("inertial_mass", C.c_double * MAX_TYPES)]


FF_DEFAULT = dict(near_cut=8.0, grid=32, block=5, hidden=128, judge_every=500, judge_tol=1e-3,
                  near_mode=0, parent_reach=0)
NEAR_RADIAL, NEAR_BLOCK = 0, 1


SYMBOLS = [
    "ld_init", "ld_destroy", "ld_last_error", "ld_forces", "ld_step", "ld_sync",
    "ld_get_positions", "ld_get_state", "ld_set_params", "ld_diagnostics", "ld_rdf",
    "ld_fractal", "ld_get_tuning", "ld_set_tuning", "ld_kernel_timing", "ld_kernel_time",
    "ld_near_kernel_time", "ld_autotune", "ld_checkpoint_save", "ld_checkpoint_load",
    "ld_set_positions",
    "ld_ff_enable", "ld_ff_mode", "ld_ff_weights_size", "ld_ff_set_weights", "ld_ff_get_weights",
    "ld_ff_grid", "ld_ff_forces", "ld_ff_mlp", "ld_ff_grads", "ld_ff_collect", "ld_ff_train",
    "ld_ff_judge", "ld_ff_stats",
    "ld_ens_init", "ld_ens_destroy", "ld_ens_set_tuning", "ld_ens_step", "ld_ens_forces",
    "ld_ens_get_positions", "ld_ens_get_state", "ld_ens_sync", "ld_ens_kernel_timing",
    "ld_ens_kernel_time",
    "ld_paper_enable", "ld_paper_disable", "ld_paper_forces", "ld_paper_get_velocities",
    "ld_paper_set_velocities", "ld_aggregates", "ld_surface_count", "ld_record_open",
    "ld_record_close", "ld_cbar_type", "ld_surface_fractal", "ld_ff_save", "ld_ff_load",
    "ld_msd", "ld_msd_reset", "ld_forces_noalloc", "ld_ens_get_tuning", "ld_ens_set_unroll",
    "ld_ens_set_rows", "ld_ens_autotune",
]

_lib = None


def lib():
    """Load libldrop.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2501_04456_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, dp, fp = C.c_void_p, C.c_void_p, C.c_void_p
        L.ld_init.argtypes = [C.POINTER(C.c_void_p), C.c_int64, vp, vp, vp,
                              C.POINTER(ld_params), C.POINTER(ld_radius), C.c_uint64, vp]
        L.ld_destroy.argtypes = [vp]
        L.ld_destroy.restype = None
        L.ld_last_error.restype = C.c_char_p
        L.ld_forces.argtypes = [vp, dp, dp, dp, dp]
        L.ld_step.argtypes = [vp, C.c_double, C.c_int64, C.POINTER(ld_radius),
                              C.POINTER(C.c_uint64), C.POINTER(ld_diag)]
        L.ld_forces_noalloc.argtypes = [C.c_int64, vp, vp, vp, C.POINTER(ld_params), vp, vp]
        L.ld_msd.argtypes = [vp, dp]
        L.ld_msd_reset.argtypes = [vp]
        L.ld_sync.argtypes = [vp]
        L.ld_get_positions.argtypes = [vp, fp, fp]
        L.ld_set_positions.argtypes = [vp, vp, vp]
        L.ld_get_state.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
        L.ld_set_params.argtypes = [vp, C.POINTER(ld_params), C.POINTER(ld_radius)]
        L.ld_diagnostics.argtypes = [vp, dp]
        L.ld_rdf.argtypes = [vp, C.c_double, C.c_int32, C.c_double, C.c_int32, vp, vp, vp, vp]
        L.ld_fractal.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int32, vp, vp]
        L.ld_get_tuning.argtypes = [vp, C.POINTER(ld_tuning)]
        L.ld_set_tuning.argtypes = [vp, C.POINTER(ld_tuning)]
        L.ld_kernel_timing.argtypes = [vp, C.c_int32]
        L.ld_kernel_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ld_near_kernel_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ld_autotune.argtypes = [vp, C.c_char_p, C.c_int32, C.POINTER(ld_tuning)]
        L.ld_checkpoint_save.argtypes = [vp, C.c_char_p]
        L.ld_checkpoint_load.argtypes = [C.POINTER(C.c_void_p), C.c_char_p, vp]
        L.ld_ens_init.argtypes = [C.POINTER(C.c_void_p), C.c_int32, vp, vp, vp, vp, vp, vp, vp,
                                  vp]
        L.ld_ens_destroy.argtypes = [vp]
        L.ld_ens_destroy.restype = None
        L.ld_ens_set_tuning.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.ld_ens_step.argtypes = [vp, C.c_double, C.c_int64]
        L.ld_ens_get_tuning.argtypes = [vp, vp]
        L.ld_ens_set_unroll.argtypes = [vp, C.c_int32]
        L.ld_ens_set_rows.argtypes = [vp, C.c_int32]
        L.ld_ens_autotune.argtypes = [vp, C.c_char_p, C.c_int32, vp]
        L.ld_ens_forces.argtypes = [vp, vp]
        L.ld_ens_get_positions.argtypes = [vp, vp, vp]
        L.ld_ens_get_state.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ld_ens_sync.argtypes = [vp]
        L.ld_ens_kernel_timing.argtypes = [vp, C.c_int32]
        L.ld_ens_kernel_time.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.ld_ff_enable.argtypes = [vp, C.POINTER(ld_ff_config)]
        L.ld_ff_mode.argtypes = [vp, C.c_int32]
        L.ld_ff_weights_size.argtypes = [vp]
        L.ld_ff_weights_size.restype = C.c_int64
        L.ld_ff_set_weights.argtypes = [vp, vp, C.c_int64, C.c_double, C.c_double]
        L.ld_ff_get_weights.argtypes = [vp, vp, C.c_int64, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.ld_ff_grid.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.ld_ff_forces.argtypes = [vp, C.c_int32, vp]
        L.ld_ff_mlp.argtypes = [vp, vp, C.c_int64, vp]
        L.ld_ff_grads.argtypes = [vp, vp, vp, C.c_int64, vp, C.POINTER(C.c_double)]
        L.ld_ff_collect.argtypes = [vp, C.c_int32, C.c_int32]
        L.ld_ff_train.argtypes = [vp, C.POINTER(ld_ff_train_cfg), C.POINTER(ld_ff_train_report)]
        L.ld_ff_judge.argtypes = [vp, C.POINTER(C.c_double)]
        L.ld_ff_stats.argtypes = [vp, vp, C.POINTER(C.c_double)]
        L.ld_paper_enable.argtypes = [vp, C.POINTER(ld_paper_config)]
        L.ld_paper_disable.argtypes = [vp]
        L.ld_paper_forces.argtypes = [vp, dp]
        L.ld_paper_get_velocities.argtypes = [vp, dp]
        L.ld_paper_set_velocities.argtypes = [vp, dp]
        L.ld_aggregates.argtypes = [vp, C.c_double, vp, vp]
        L.ld_surface_count.argtypes = [vp, C.c_double, vp]
        L.ld_ff_save.argtypes = [vp, C.c_char_p]
        L.ld_ff_load.argtypes = [vp, C.c_char_p]
        L.ld_surface_fractal.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                         vp, vp, vp]
        L.ld_record_open.argtypes = [vp, C.c_char_p, C.c_int32]
        L.ld_record_close.argtypes = [vp, C.POINTER(C.c_int64)]
        L.ld_cbar_type.argtypes = [vp, C.c_int32, C.c_double, C.c_int32, C.c_double, C.c_int32,
                                   vp, vp]
        for name in SYMBOLS:
            if name not in ("ld_destroy", "ld_last_error", "ld_ens_destroy",
                            "ld_ff_weights_size"):
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def _check(status: int):
    if status != LD_OK:
        msg = lib().ld_last_error().decode()
        raise (NonFinite if status == -4 else LdError)(status, msg)


def make_params(p: W.Params) -> ld_params:
    s = ld_params()
    T = len(p.sigma)
    s.n_types = T
    for name in ("sigma", "eps", "mass", "gamma", "k_wall", "wall_offset"):
        arr = getattr(s, name)
        for t, v in enumerate(getattr(p, name)):
            arr[t] = float(v)
    if p.eps_matrix is not None:
        s.use_eps_matrix = 1
        for a in range(T):
            for b in range(T):
                s.eps_matrix[a * MAX_TYPES + b] = float(p.eps_matrix[a][b])
    s.lj_cut, s.coul_cut, s.bjerrum, s.kT = p.lj_cut, p.coul_cut, p.bjerrum, p.kT
    for c in range(3):
        s.gravity[c] = float(p.gravity[c])
    s.omega, s.rotation, s.wall_band, s.noise = p.omega, p.rotation, p.wall_band, p.noise
    s.jump_max = p.jump_max
    return s


def make_radius(r: W.Radius) -> ld_radius:
    s = ld_radius()
    s.kind, s.R0, s.R1, s.T, s.a, s.R_min = r.kind, r.R0, r.R1, r.T, r.a, r.R_min
    if len(r.knots_t) != len(r.knots_R) or len(r.knots_t) > W.RADIUS_TABLE_MAX:
        raise ValueError("radius table: knots_t and knots_R of equal length <= 16")
    s.n_knots = len(r.knots_t)
    for k, (tk, rk) in enumerate(zip(r.knots_t, r.knots_R)):
        s.tab_t[k], s.tab_R[k] = tk, rk
    return s


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libldrop needs a ROCm GPU; torch.cuda.is_available() is False")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class System:
    """One droplet on the GPU (an ld_ctx)."""

    def __init__(self, type_, charge, pos, params: W.Params, radius: W.Radius, seed: int,
                 stream=None):
        torch = _torch()
        self._torch = torch
        dev = torch.device("cuda")
        self.stream = torch.cuda.current_stream() if stream is None else stream
        t = torch.as_tensor(np.ascontiguousarray(type_, dtype=np.int32), device=dev)
        q = torch.as_tensor(np.ascontiguousarray(charge, dtype=np.float64), device=dev)
        # pos None: the library samples the initial positions itself
        x = None if pos is None else torch.as_tensor(
            np.ascontiguousarray(np.asarray(pos, dtype=np.float32).reshape(-1, 3)), device=dev)
        self.n = int(t.numel())
        self.params = params
        self.radius = radius
        self._p = make_params(params)
        self._r = make_radius(radius)
        h = C.c_void_p()
        _check(lib().ld_init(C.byref(h), self.n, _ptr(t), _ptr(q),
                             None if x is None else _ptr(x), C.byref(self._p),
                             C.byref(self._r), int(seed) & 0xFFFFFFFFFFFFFFFF,
                             C.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def checkpoint(self, path: str):
        """Save the full state (section 2.2: stop and restart)."""
        _check(lib().ld_checkpoint_save(self.h, path.encode()))

    @classmethod
    def load(cls, path: str, w: W.Workload, stream=None) -> "System":
        """A context restored from a checkpoint of workload w (the file's
        parameters, schedule, seed and state are used; w supplies n and the
        Python-side description)."""
        torch = _torch()
        self = cls.__new__(cls)
        self._torch = torch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = C.c_void_p()
        _check(lib().ld_checkpoint_load(C.byref(h), path.encode(),
                                        C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self.n = w.n
        self.params, self.radius = w.params, w.radius
        return self

    @classmethod
    def from_workload(cls, w: W.Workload, **kw) -> "System":
        return cls(w.type, w.charge, w.pos, w.params, w.radius, w.seed, **kw)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ld_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hot path ---------------------------------------------------------
    def forces(self, ext: bool = True, S: bool = False, U: bool = False):
        """Returns dict with 'pair' [n,3], optional 'ext' [n,3], 'S' [n] (cuda FP64
        tensors) and 'U' (numpy [2])."""
        torch = self._torch
        dev = torch.device("cuda")
        Fp = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        Fe = torch.empty((self.n, 3), dtype=torch.float64, device=dev) if ext else None
        Ss = torch.empty(self.n, dtype=torch.float64, device=dev) if S else None
        Uu = np.zeros(2) if U else None
        _check(lib().ld_forces(self.h, _ptr(Fp), _ptr(Fe) if ext else None,
                               _ptr(Ss) if S else None,
                               Uu.ctypes.data_as(C.c_void_p) if U else None))
        out = {"pair": Fp}
        if ext:
            out["ext"] = Fe
        if S:
            out["S"] = Ss
        if U:
            out["U"] = Uu
        return out

    def step(self, n_steps: int, dt: float = None, radius: W.Radius = None, seed: int = None,
             diag: bool = False):
        """n_steps steps of size dt; a new radius schedule and/or noise seed
        apply from the first of them on.  diag=True waits and returns the
        state and FP64 diagnostics after the steps (a dict); a blow-up then
        raises NonFinite."""
        dt = self.dt if dt is None else dt
        r = C.byref(make_radius(radius)) if radius is not None else None
        sd = C.byref(C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF)) if seed is not None else None
        d = ld_diag() if diag else None
        _check(lib().ld_step(self.h, float(dt), int(n_steps), r, sd,
                             C.byref(d) if diag else None))
        if radius is not None:
            self.radius = radius
        if not diag:
            return None
        return {"step": d.step, "t": d.t, "R": d.R, "U": np.array(d.U[:]),
                "net_force": np.array(d.net_force[:]), "max_force": d.max_force,
                "max_radius": d.max_radius, "msd": d.msd, "bad_step": d.bad_step}

    def msd(self) -> float:
        """Mean square displacement against the reference positions."""
        v = C.c_double()
        _check(lib().ld_msd(self.h, C.byref(v)))
        return v.value

    def msd_reset(self):
        _check(lib().ld_msd_reset(self.h))

    def sync(self):
        _check(lib().ld_sync(self.h))

    # -- state --------------------------------------------------------------
    def positions(self):
        """(hi, lo) FP32 numpy arrays [n,3] in original order."""
        hi = np.zeros((self.n, 3), np.float32)
        lo = np.zeros((self.n, 3), np.float32)
        _check(lib().ld_get_positions(self.h, hi.ctypes.data_as(C.c_void_p),
                                      lo.ctypes.data_as(C.c_void_p)))
        return hi, lo

    def positions64(self) -> np.ndarray:
        hi, lo = self.positions()
        return hi.astype(np.float64) + lo.astype(np.float64)

    def positions_into(self, hi: np.ndarray, lo: np.ndarray = None):
        """Write the FP32 (hi, lo) positions, original order, into given
        C-contiguous float32 host arrays of shape [n, 3] (lo may be None)."""
        for a in (hi, lo):
            if a is not None and (a.dtype != np.float32 or a.shape != (self.n, 3)
                                  or not a.flags.c_contiguous):
                raise ValueError("positions_into needs C-contiguous float32 [n, 3] arrays")
        _check(lib().ld_get_positions(self.h, hi.ctypes.data_as(C.c_void_p),
                                      None if lo is None else lo.ctypes.data_as(C.c_void_p)))

    def set_positions(self, x, x_lo=None):
        """Replace the positions ([n,3] in original order; x_lo the low FP32
        parts or None)."""
        hi = np.ascontiguousarray(x, np.float32).reshape(self.n, 3)
        lo = None if x_lo is None else np.ascontiguousarray(x_lo, np.float32).reshape(self.n, 3)
        _check(lib().ld_set_positions(self.h, hi.ctypes.data_as(C.c_void_p),
                                      None if lo is None else lo.ctypes.data_as(C.c_void_p)))

    # -- trajectory recording -------------------------------------------
    def record_open(self, path: str, every: int = 1):
        """Record every `every`-th step's positions into `path` (binary)."""
        _check(lib().ld_record_open(self.h, os.fsencode(path), int(every)))

    def record_close(self) -> int:
        f = C.c_int64()
        _check(lib().ld_record_close(self.h, C.byref(f)))
        return f.value

    # -- aggregate statistics -------------------------------------------
    def aggregates(self, contact_factor: float = 1.1, labels: bool = False):
        """Contact-graph components: returns dict(components, aggregates,
        largest[, labels = smallest original index of each NP's component])."""
        st = np.zeros(3, np.int64)
        lab = np.zeros(self.n, np.int32) if labels else None
        _check(lib().ld_aggregates(self.h, float(contact_factor),
                                   st.ctypes.data_as(C.c_void_p),
                                   lab.ctypes.data_as(C.c_void_p) if labels else None))
        out = {"components": int(st[0]), "aggregates": int(st[1]), "largest": int(st[2])}
        if labels:
            out["labels"] = lab
        return out

    def surface_count(self, R: float = -1.0) -> np.ndarray:
        """N_surf per type (R < 0: the droplet's current radius)."""
        c = np.zeros(len(self.params.sigma), np.int64)
        _check(lib().ld_surface_count(self.h, float(R), c.ctypes.data_as(C.c_void_p)))
        return c

    def surface_fractal(self, R: float = -1.0, contact_factor: float = 1.1,
                        k_f: float = math.pi / math.sqrt(3.0), d: float = 0.0,
                        labels: bool = False):
        """Surface fractal dimension of the largest surface aggregate (the
        fractal equation at dimension two, geodesic R_g on the sphere of
        radius R; R < 0: the current radius).  Returns dict(components,
        largest, label, R_g, d, D_f[, labels: -1 off the surface])."""
        st = np.zeros(3, np.int64)
        o = np.zeros(3)
        lab = np.zeros(self.n, np.int32) if labels else None
        _check(lib().ld_surface_fractal(self.h, float(R), float(contact_factor), float(k_f),
                                        float(d), st.ctypes.data_as(C.c_void_p),
                                        o.ctypes.data_as(C.c_void_p),
                                        lab.ctypes.data_as(C.c_void_p) if labels else None))
        out = {"components": int(st[0]), "largest": int(st[1]), "label": int(st[2]),
               "R_g": float(o[0]), "d": float(o[1]), "D_f": float(o[2])}
        if labels:
            out["labels"] = lab
        return out

    # -- the paper's own scheme ------------------------------------------
    def paper_enable(self, range_factor: float = 4.0, kick: float = 0.0, inertial_mass=None):
        """Switch ld_step to the paper's scheme (pairs truncated at
        range_factor (r_i + r_j); Newton + Stokes drag; random velocity kick).
        inertial_mass per type (default: the parameters' mass)."""
        c = ld_paper_config()
        c.range_factor = float(range_factor)
        c.kick = float(kick)
        m = self.params.mass if inertial_mass is None else inertial_mass
        for t, v in enumerate(m):
            c.inertial_mass[t] = float(v)
        _check(lib().ld_paper_enable(self.h, C.byref(c)))

    def paper_disable(self):
        _check(lib().ld_paper_disable(self.h))

    def paper_forces(self) -> np.ndarray:
        F = np.zeros((self.n, 3))
        _check(lib().ld_paper_forces(self.h, F.ctypes.data_as(C.c_void_p)))
        return F

    def velocities(self) -> np.ndarray:
        v = np.zeros((self.n, 3))
        _check(lib().ld_paper_get_velocities(self.h, v.ctypes.data_as(C.c_void_p)))
        return v

    def set_velocities(self, v):
        v = np.ascontiguousarray(v, np.float64).reshape(self.n, 3)
        _check(lib().ld_paper_set_velocities(self.h, v.ctypes.data_as(C.c_void_p)))

    def state(self):
        s, t, R = C.c_int64(), C.c_double(), C.c_double()
        _check(lib().ld_get_state(self.h, C.byref(s), C.byref(t), C.byref(R)))
        return s.value, t.value, R.value

    def set_params(self, params: W.Params = None, radius: W.Radius = None):
        p = make_params(params) if params is not None else None
        r = make_radius(radius) if radius is not None else None
        _check(lib().ld_set_params(self.h, C.byref(p) if p else None,
                                   C.byref(r) if r else None))
        if params is not None:
            self.params = params
        if radius is not None:
            self.radius = radius

    def diagnostics(self) -> np.ndarray:
        out = np.zeros(10)
        _check(lib().ld_diagnostics(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    # -- post-processing ----------------------------------------------------
    def rdf(self, r_max: float, n_bins: int, V: float = 0.0, centre: int = 0):
        counts = np.zeros(n_bins, np.uint64)
        cc = np.zeros(n_bins, np.uint64)
        g = np.zeros(n_bins)
        cbar = np.zeros(n_bins)
        _check(lib().ld_rdf(self.h, r_max, n_bins, V, centre, counts.ctypes.data_as(C.c_void_p),
                            g.ctypes.data_as(C.c_void_p), cc.ctypes.data_as(C.c_void_p),
                            cbar.ctypes.data_as(C.c_void_p)))
        return counts, cc, g, cbar

    def cbar_type(self, t: int, r_max: float, n_bins: int, V: float = 0.0, centre: int = 0):
        """Eq. (8) for the NPs of type t: (counts [n_bins] uint64, cbar [n_bins])."""
        cc = np.zeros(n_bins, np.uint64)
        cb = np.zeros(n_bins)
        _check(lib().ld_cbar_type(self.h, int(t), r_max, n_bins, V, centre,
                                  cc.ctypes.data_as(C.c_void_p), cb.ctypes.data_as(C.c_void_p)))
        return cc, cb

    def fractal(self, k_f: float = 1.593, d: float = 0.0, eps0: float = 0.0,
                max_scales: int = 32):
        out = np.zeros(4)
        bc = np.zeros(max_scales, np.int64)
        _check(lib().ld_fractal(self.h, k_f, d, eps0, max_scales, out.ctypes.data_as(C.c_void_p),
                                bc.ctypes.data_as(C.c_void_p)))
        K = int(out[3])
        return out[0], out[1], out[2], K, bc[:K].copy()

    # -- performance controls -----------------------------------------------
    def tuning(self) -> dict:
        t = ld_tuning()
        _check(lib().ld_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def autotune(self, cache_path: str = None, force: bool = False) -> dict:
        t = ld_tuning()
        _check(lib().ld_autotune(self.h, cache_path.encode() if cache_path else None,
                                 1 if force else 0, C.byref(t)))
        return {k: getattr(t, k) for k in TUNING_FIELDS}

    def set_tuning(self, **kw):
        t = ld_tuning()
        _check(lib().ld_get_tuning(self.h, C.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(lib().ld_set_tuning(self.h, C.byref(t)))

    # -- learned far field --------------------------------------------------
    def ff_enable(self, **kw):
        cfg = dict(FF_DEFAULT, **kw)
        c = ld_ff_config(**cfg)
        _check(lib().ld_ff_enable(self.h, C.byref(c)))
        self.ff_cfg = cfg

    def ff_mode(self, mode: int):
        _check(lib().ld_ff_mode(self.h, int(mode)))

    def ff_weights(self):
        n = lib().ld_ff_weights_size(self.h)
        w = np.zeros(n, np.float32)
        sq, sc = C.c_double(), C.c_double()
        _check(lib().ld_ff_get_weights(self.h, w.ctypes.data_as(C.c_void_p), n, C.byref(sq),
                                       C.byref(sc)))
        return w, sq.value, sc.value

    def ff_save(self, path: str):
        """Write the learned model (configuration, scales, weights) to path."""
        _check(lib().ld_ff_save(self.h, os.fsencode(path)))

    def ff_load(self, path: str):
        """Load a model written by ff_save; the learned field must be
        enabled with the same configuration."""
        _check(lib().ld_ff_load(self.h, os.fsencode(path)))

    def ff_set_weights(self, w, sq: float, out_scale: float):
        w = np.ascontiguousarray(w, np.float32)
        _check(lib().ld_ff_set_weights(self.h, w.ctypes.data_as(C.c_void_p), w.size, sq,
                                       out_scale))

    def ff_grid(self):
        L, g = C.c_double(), C.c_int32()
        _check(lib().ld_ff_grid(self.h, C.byref(L), C.byref(g)))
        return L.value, g.value

    def ff_forces(self, part: int) -> np.ndarray:
        out = np.zeros((self.n, 3))
        _check(lib().ld_ff_forces(self.h, int(part), out.ctypes.data_as(C.c_void_p)))
        return out

    def ff_mlp(self, X) -> np.ndarray:
        X = np.ascontiguousarray(X, np.float32)
        Y = np.zeros((X.shape[0], 3), np.float32)
        _check(lib().ld_ff_mlp(self.h, X.ctypes.data_as(C.c_void_p), X.shape[0],
                               Y.ctypes.data_as(C.c_void_p)))
        return Y

    def ff_grads(self, X, T):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        g = np.zeros(lib().ld_ff_weights_size(self.h), np.float32)
        loss = C.c_double()
        _check(lib().ld_ff_grads(self.h, X.ctypes.data_as(C.c_void_p),
                                 T.ctypes.data_as(C.c_void_p), X.shape[0],
                                 g.ctypes.data_as(C.c_void_p), C.byref(loss)))
        return loss.value, g

    def ff_collect(self, reset: bool = False, max_snapshots: int = 16):
        _check(lib().ld_ff_collect(self.h, 1 if reset else 0, int(max_snapshots)))

    def ff_train(self, epochs=20, batch=8192, lr=1e-3, seed=105, val_fraction=0.1,
                 reset_scale=True, calibrate=True) -> dict:
        c = ld_ff_train_cfg(epochs=epochs, batch=batch, lr=lr, seed=seed,
                            val_fraction=val_fraction, reset_scale=1 if reset_scale else 0,
                            calibrate=1 if calibrate else 0)
        r = ld_ff_train_report()
        _check(lib().ld_ff_train(self.h, C.byref(c), C.byref(r)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    def ff_judge(self) -> float:
        v = C.c_double()
        _check(lib().ld_ff_judge(self.h, C.byref(v)))
        return v.value

    def ff_stats(self):
        out = np.zeros(4, np.int64)
        e = C.c_double()
        _check(lib().ld_ff_stats(self.h, out.ctypes.data_as(C.c_void_p), C.byref(e)))
        return {"judges": int(out[0]), "fallbacks": int(out[1]), "learned_steps": int(out[2]),
                "direct_steps": int(out[3]), "last_err": e.value}

    def kernel_timing(self, enable: bool):
        _check(lib().ld_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().ld_kernel_time(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    def near_kernel_time(self):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().ld_near_kernel_time(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value

    dt = 1e-3


class Ensemble:
    """Independent droplets stepped together (an ld_ens)."""

    def __init__(self, droplets, stream=None):
        torch = _torch()
        self._torch = torch
        dev = torch.device("cuda")
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.droplets = list(droplets)
        nd = len(self.droplets)
        off = np.zeros(nd + 1, dtype=np.int64)
        off[1:] = np.cumsum([d.n for d in self.droplets])
        self.offsets = off
        self.total = int(off[-1])
        t = torch.as_tensor(np.concatenate([d.type for d in self.droplets]).astype(np.int32),
                            device=dev)
        q = torch.as_tensor(np.concatenate([d.charge for d in self.droplets]).astype(np.float64),
                            device=dev)
        x = torch.as_tensor(np.concatenate([np.asarray(d.pos, np.float32).reshape(-1, 3)
                                            for d in self.droplets]), device=dev)
        P = (ld_params * nd)(*[make_params(d.params) for d in self.droplets])
        R = (ld_radius * nd)(*[make_radius(d.radius) for d in self.droplets])
        S = (C.c_uint64 * nd)(*[int(d.seed) & 0xFFFFFFFFFFFFFFFF for d in self.droplets])
        h = C.c_void_p()
        _check(lib().ld_ens_init(C.byref(h), nd, off.ctypes.data_as(C.c_void_p), _ptr(t), _ptr(q),
                                 _ptr(x), C.cast(P, C.c_void_p), C.cast(R, C.c_void_p),
                                 C.cast(S, C.c_void_p), C.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().ld_ens_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    ENS_TUNING = ("workgroups", "comp", "graph_steps", "unroll", "rows")

    def set_tuning(self, workgroups: int = 0, comp: int = 0, graph_steps: int = 0,
                   unroll: int = 0, rows: int = 0):
        _check(lib().ld_ens_set_tuning(self.h, workgroups, comp, graph_steps))
        if unroll:
            _check(lib().ld_ens_set_unroll(self.h, unroll))
        if rows:
            _check(lib().ld_ens_set_rows(self.h, rows))

    def tuning(self) -> dict:
        out = np.zeros(5, np.int32)
        _check(lib().ld_ens_get_tuning(self.h, out.ctypes.data_as(C.c_void_p)))
        return dict(zip(self.ENS_TUNING, map(int, out)))

    def autotune(self, cache_path: str = None, force: bool = False) -> dict:
        out = np.zeros(5, np.int32)
        _check(lib().ld_ens_autotune(self.h, cache_path.encode() if cache_path else None,
                                     1 if force else 0, out.ctypes.data_as(C.c_void_p)))
        return dict(zip(self.ENS_TUNING, map(int, out)))

    def step(self, n_steps: int, dt: float):
        _check(lib().ld_ens_step(self.h, float(dt), int(n_steps)))

    def sync(self):
        _check(lib().ld_ens_sync(self.h))

    def forces(self):
        F = self._torch.empty((self.total, 3), dtype=self._torch.float64, device="cuda")
        _check(lib().ld_ens_forces(self.h, _ptr(F)))
        return F

    def positions(self):
        """(hi, lo) FP32 numpy arrays [total,3] in original order."""
        hi = np.zeros((self.total, 3), np.float32)
        lo = np.zeros((self.total, 3), np.float32)
        _check(lib().ld_ens_get_positions(self.h, hi.ctypes.data_as(C.c_void_p),
                                          lo.ctypes.data_as(C.c_void_p)))
        return hi, lo

    def positions64(self):
        hi, lo = self.positions()
        return hi.astype(np.float64) + lo.astype(np.float64)

    def state(self):
        s, t = C.c_int64(), C.c_double()
        _check(lib().ld_ens_get_state(self.h, C.byref(s), C.byref(t)))
        return s.value, t.value

    def kernel_timing(self, enable: bool):
        _check(lib().ld_ens_kernel_timing(self.h, 1 if enable else 0))

    def kernel_time(self):
        n, ms = C.c_int64(), C.c_double()
        _check(lib().ld_ens_kernel_time(self.h, C.byref(n), C.byref(ms)))
        return n.value, ms.value


def read_trajectory(path: str) -> dict:
    """Parse a file written by ld_record_open: dict(n, n_types, every, type
    [n], step [F], t [F], R [F], x [F, n, 3] float32)."""
    raw = np.fromfile(path, dtype=np.uint8)
    if raw[:8].tobytes() != b"LDTRAJ01":
        raise ValueError(f"{path}: not a trajectory file")
    n = int(raw[8:16].view(np.int64)[0])
    n_types, every = (int(v) for v in raw[16:24].view(np.int32))
    off = 24
    typ = raw[off:off + 4 * n].view(np.int32).copy()
    off += 4 * n
    fb = 24 + 12 * n
    F = (len(raw) - off) // fb
    frames = raw[off:off + F * fb].reshape(F, fb)
    return {"n": n, "n_types": n_types, "every": every, "type": typ,
            "step": frames[:, 0:8].copy().view(np.int64)[:, 0],
            "t": frames[:, 8:16].copy().view(np.float64)[:, 0],
            "R": frames[:, 16:24].copy().view(np.float64)[:, 0],
            "x": frames[:, 24:].copy().view(np.float32).reshape(F, n, 3)}
