"""CPU FP64 oracle for the Langevin droplet-aggregation model (arXiv:2501.04456).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library: the C source (``ldo.c``) has its own header, its own Philox,
its own parameter struct, and this binding defines its own ctypes layout.

Each wrapper below cites the passage of the paper it follows; the formulas
themselves are in ``ldo.c``.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libldo.so")
MAX_TYPES = 8

CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    """Compile ldo.c into libldo.so with gcc (generic x86-64, no fast-math)."""
    srcs = [os.path.join(_HERE, f) for f in ("ldo.c", "ldo_ff.c", "ldo_paper.c", "ldo_agg.c")]
    srcs = [s for s in srcs if os.path.exists(s)]
    # written beside and renamed into place, so that a process that has the
    # old library loaded keeps its own copy
    tmp = f"{_LIB_PATH}.{os.getpid()}.tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
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


class _Paper(C.Structure):
    _fields_ = [("range_factor", C.c_double), ("kick", C.c_double),
                ("inertial_mass", C.c_double * MAX_TYPES)]


R_TABLE_MAX = 16


class _Radius(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_knots", C.c_int32), ("R0", C.c_double),
                ("R1", C.c_double), ("T", C.c_double), ("a", C.c_double),
                ("R_min", C.c_double), ("tab_t", C.c_double * R_TABLE_MAX),
                ("tab_R", C.c_double * R_TABLE_MAX)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.ldo_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.ldo_gauss3.argtypes = [C.c_int64, C.c_int64, C.c_uint64, C.c_uint32, dp]
        L.ldo_sample_ball.argtypes = [C.c_int64, C.POINTER(C.c_int32), dp, C.c_double,
                                      C.c_uint64, C.c_int64, dp]
        L.ldo_sample_ball.restype = C.c_int64
        L.ldo_radius_at.argtypes = [C.POINTER(_Radius), C.c_double]
        L.ldo_radius_at.restype = C.c_double
        L.ldo_pair_forces.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp,
                                      C.POINTER(_Params), C.POINTER(C.c_int64), C.c_int64,
                                      dp, dp, dp]
        L.ldo_external_force.argtypes = [dp, C.c_int32, C.POINTER(_Params), C.c_double, dp]
        L.ldo_run.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp, C.POINTER(C.c_int64),
                              C.POINTER(_Params), C.POINTER(_Radius), C.c_double, C.c_int64,
                              C.c_uint64, C.POINTER(C.c_int64), dp]
        L.ldo_run.restype = C.c_int64
        L.ldo_step_rows.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp,
                                    C.POINTER(C.c_int64), C.POINTER(_Params),
                                    C.POINTER(_Radius), C.c_double, C.c_uint64, C.c_int64,
                                    C.c_double, C.POINTER(C.c_int64), C.c_int64, dp]
        L.ldo_step_rows.restype = C.c_int64
        L.ldo_diagnostics.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp,
                                      C.POINTER(_Params), C.c_double, dp]
        L.ldo_msd.argtypes = [C.c_int64, dp, dp]
        L.ldo_msd.restype = C.c_double
        L.ldo_rdf.argtypes = [C.c_int64, dp, C.c_double, C.c_int32, C.c_double, dp,
                              C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), dp, dp]
        L.ldo_fractal.argtypes = [C.c_int64, dp, C.c_double, C.c_double, C.c_double,
                                  C.c_int32, dp, C.POINTER(C.c_int64)]
        L.ldo_bf16.argtypes = [C.c_double]
        L.ldo_bf16.restype = C.c_double
        L.ldo_ff_moments.argtypes = [C.c_int64, dp, dp, C.c_int, C.c_double, dp]
        L.ldo_ff_coarse.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp]
        L.ldo_ff_split.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp, C.POINTER(_Params),
                                   C.c_double, C.POINTER(C.c_int64), C.c_int64, dp, dp]
        L.ldo_ff_split_block.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp,
                                         C.POINTER(_Params), C.c_int, C.c_double, C.c_int,
                                         C.POINTER(C.c_int64), C.c_int64, dp, dp]
        L.ldo_ff_local.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp]
        L.ldo_ff_local2.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, dp, dp]
        L.ldo_ff_local_eval.argtypes = [C.c_int64, dp, C.c_int, C.c_double, dp, dp]
        L.ldo_ff_features.argtypes = [C.c_int64, dp, C.c_int, C.c_double, C.c_int, dp,
                                      C.c_double, dp]
        L.ldo_mlp_forward.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp,
                                      dp, dp, C.c_int, dp, dp, dp, dp, dp]
        L.ldo_mlp_backward.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp,
                                       dp, dp, dp, C.c_int, dp, dp, dp, dp, dp, dp]
        L.ldo_mlp_backward.restype = C.c_double
        L.ldo_paper_forces.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), dp,
                                       C.POINTER(_Params), C.POINTER(_Paper),
                                       C.POINTER(C.c_int64), C.c_int64, dp, dp]
        L.ldo_paper_run.argtypes = [C.c_int64, dp, dp, C.POINTER(C.c_int32), dp,
                                    C.POINTER(C.c_int64), C.POINTER(_Params), C.POINTER(_Paper),
                                    C.POINTER(_Radius), C.c_double, C.c_int64, C.c_uint64,
                                    C.POINTER(C.c_int64), dp]
        L.ldo_paper_run.restype = C.c_int64
        L.ldo_components.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), C.POINTER(_Params),
                                     C.c_double, C.POINTER(C.c_int64)]
        L.ldo_components.restype = C.c_int64
        L.ldo_surface_count.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32), C.POINTER(_Params),
                                        C.c_double, C.POINTER(C.c_int64)]
        L.ldo_surface_fractal.argtypes = [C.c_int64, dp, C.POINTER(C.c_int32),
                                          C.POINTER(_Params), C.c_double, C.c_double,
                                          C.c_double, C.c_double, C.POINTER(C.c_int64), dp,
                                          C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int64))


def make_params(p) -> _Params:
    """Marshal a workloads.Params into the oracle's own struct."""
    s = _Params()
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
    s.lj_cut = p.lj_cut
    s.coul_cut = p.coul_cut
    s.bjerrum = p.bjerrum
    s.kT = p.kT
    for c in range(3):
        s.gravity[c] = float(p.gravity[c])
    s.omega = p.omega
    s.rotation = p.rotation
    s.wall_band = p.wall_band
    s.noise = p.noise
    s.jump_max = p.jump_max
    return s


def make_radius(r) -> _Radius:
    s = _Radius()
    s.kind, s.R0, s.R1, s.T, s.a, s.R_min = r.kind, r.R0, r.R1, r.T, r.a, r.R_min
    kt, kr = tuple(getattr(r, "knots_t", ())), tuple(getattr(r, "knots_R", ()))
    if len(kt) != len(kr) or len(kt) > R_TABLE_MAX:
        raise ValueError("radius table: knots_t and knots_R of equal length <= 16")
    s.n_knots = len(kt)
    for k, (tk, rk) in enumerate(zip(kt, kr)):
        s.tab_t[k], s.tab_R[k] = tk, rk
    return s


# ---------------------------------------------------------------------------
# Wrappers
# ---------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block (the counter-based noise generator)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().ldo_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def gauss3(pid: int, step: int, seed: int, tag: int = 0) -> np.ndarray:
    out = np.zeros(3)
    lib().ldo_gauss3(pid, step, seed, tag, _dp(out))
    return out


def sample_ball(type_, sigma, R0: float, seed: int, max_tries: int = 100000):
    """Initial positions [n,3] (FP32 values as FP64): uniform in the ball of
    radius R0, no pair closer than sigma_ij; raises if a particle finds no
    place in max_tries candidates."""
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    x = np.zeros((len(type_), 3))
    bad = lib().ldo_sample_ball(len(type_), _ip(type_), _dp(sig), float(R0),
                                C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(max_tries), _dp(x))
    if bad:
        raise RuntimeError(f"particle {bad} found no place")
    return x


def radius_at(radius, t: float) -> float:
    """Droplet radius at time t (section 2.1; section 2.2 step (iii))."""
    return lib().ldo_radius_at(C.byref(make_radius(radius)), t)


def pair_forces(pos, type_, charge, params, rows=None):
    """Pair forces (section 2.2 step (ii)): returns (F [m,3], S [m], U [2])."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    q = np.ascontiguousarray(charge, dtype=np.float64)
    n = len(type_)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    m = n if rows is None else len(rows_a)
    F = np.zeros((m, 3))
    S = np.zeros(m)
    U = np.zeros(2)
    p = make_params(params)
    lib().ldo_pair_forces(n, _dp(pos), _ip(type_), _dp(q), C.byref(p), _lp(rows_a), m,
                          _dp(F), _dp(S), _dp(U))
    return F, S, U


def external_force(x, t: int, params, R: float) -> np.ndarray:
    """External force (section 2.2 steps (iv)-(v)) on one particle."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    F = np.zeros(3)
    lib().ldo_external_force(_dp(x), int(t), C.byref(make_params(params)), R, _dp(F))
    return F


class State:
    """Oracle trajectory state: FP64 positions, step counter and time."""

    def __init__(self, w, pos=None, ids=None):
        self.w = w
        self.x = np.array(w.pos if pos is None else pos, dtype=np.float64).reshape(-1, 3).copy()
        self.type = np.ascontiguousarray(w.type, dtype=np.int32)
        self.q = np.ascontiguousarray(w.charge, dtype=np.float64)
        self.ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64)
        self.step = 0
        self.t = 0.0
        self.params = w.params
        self.radius = w.radius
        self.seed = w.seed

    def run(self, n_steps: int, dt: float = None) -> int:
        """Overdamped Euler-Maruyama steps (section 2.2 step (vi))."""
        dt = self.w.dt if dt is None else dt
        st = C.c_int64(self.step)
        tt = C.c_double(self.t)
        bad = lib().ldo_run(len(self.type), _dp(self.x), _ip(self.type), _dp(self.q),
                            _lp(self.ids), C.byref(make_params(self.params)),
                            C.byref(make_radius(self.radius)), dt, n_steps, self.seed,
                            C.byref(st), C.byref(tt))
        self.step = st.value
        self.t = tt.value
        return bad

    def step_rows(self, rows, dt: float = None):
        """New positions of `rows` after one step from the current state
        (section 2.2 step (vi)); the state itself is not advanced."""
        dt = self.w.dt if dt is None else dt
        rows_a = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros((len(rows_a), 3))
        bad = lib().ldo_step_rows(len(self.type), _dp(self.x), _ip(self.type), _dp(self.q),
                                  _lp(self.ids), C.byref(make_params(self.params)),
                                  C.byref(make_radius(self.radius)), dt, self.seed, self.step,
                                  self.t, _lp(rows_a), len(rows_a), _dp(out))
        return out, bad

    def diagnostics(self, R=None) -> np.ndarray:
        R = radius_at(self.radius, self.t) if R is None else R
        out = np.zeros(10)
        lib().ldo_diagnostics(len(self.type), _dp(self.x), _ip(self.type), _dp(self.q),
                              C.byref(make_params(self.params)), R, _dp(out))
        return out


def msd(x, x0) -> float:
    """Mean square displacement mean_i |x_i - x0_i|^2 (the diagnostics'
    mean square displacement; free diffusion gives 6 D t)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, 3)
    assert x.shape == x0.shape
    return float(lib().ldo_msd(len(x), _dp(x), _dp(x0)))


def rdf(x, r_max: float, n_bins: int, V: float, centre=(0.0, 0.0, 0.0)):
    """RDF Eq. (6) and radial concentration Eq. (8) (section 3.2).
    Returns (pair counts, centre counts, g, cbar)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    n = len(x)
    counts = np.zeros(n_bins, dtype=np.uint64)
    cc = np.zeros(n_bins, dtype=np.uint64)
    g = np.zeros(n_bins)
    cbar = np.zeros(n_bins)
    ctr = np.ascontiguousarray(centre, dtype=np.float64)
    lib().ldo_rdf(n, _dp(x), r_max, n_bins, V, _dp(ctr),
                  counts.ctypes.data_as(C.POINTER(C.c_uint64)),
                  cc.ctypes.data_as(C.POINTER(C.c_uint64)), _dp(g), _dp(cbar))
    return counts, cc, g, cbar


def fractal(x, k_f: float, d: float, eps0: float, max_scales: int = 32):
    """Eqs. (2)-(4) and box counting (section 3.1).
    Returns (R_g, D_f, D_box, n_scales, box_counts)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(4)
    bc = np.zeros(max_scales, dtype=np.int64)
    lib().ldo_fractal(len(x), _dp(x), k_f, d, eps0, max_scales, _dp(out), _lp(bc))
    K = int(out[3])
    return out[0], out[1], out[2], K, bc[:K].copy()


# ---------------------------------------------------------------------------
# Learned far field (the residual model of the far Coulomb sum)
# ---------------------------------------------------------------------------

def bf16(v: float) -> float:
    return lib().ldo_bf16(float(v))


def qhat(charge, params):
    """Charges in field units: q sqrt(kT l_B)."""
    return np.asarray(charge, np.float64) * np.sqrt(params.kT * params.bjerrum)


def ff_moments(x, qh, G: int, L: float) -> np.ndarray:
    """(Q, Px, Py, Pz) per cell of the G^3 grid over [-L, L]^3."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    qh = np.ascontiguousarray(qh, np.float64)
    out = np.zeros((G ** 3, 4))
    lib().ldo_ff_moments(len(x), _dp(x), _dp(qh), G, L, _dp(out))
    return out


def ff_coarse(mom, G: int, L: float, B: int = 5) -> np.ndarray:
    """Field at every cell centre from the cells outside its B^3 block."""
    mom = np.ascontiguousarray(mom, np.float64)
    E = np.zeros((G ** 3, 3))
    lib().ldo_ff_coarse(G, L, B, _dp(mom), _dp(E))
    return E


def ff_split(x, type_, charge, params, rc: float, rows=None):
    """(F_near [m,3], E_far [m,3]) split at rc."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(type_, np.int32)
    q = np.ascontiguousarray(charge, np.float64)
    rows_a = None if rows is None else np.ascontiguousarray(rows, np.int64)
    m = len(t) if rows is None else len(rows_a)
    Fn = np.zeros((m, 3))
    Ef = np.zeros((m, 3))
    lib().ldo_ff_split(len(t), _dp(x), _ip(t), _dp(q), C.byref(make_params(params)), rc,
                       _lp(rows_a), m, _dp(Fn), _dp(Ef))
    return Fn, Ef


def ff_split_block(x, type_, charge, params, G: int, L: float, B: int = 5, rows=None):
    """(F_near [m,3], E_far [m,3]) with the near region = the B^3 block of
    grid cells around each particle's cell."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(type_, np.int32)
    q = np.ascontiguousarray(charge, np.float64)
    rows_a = None if rows is None else np.ascontiguousarray(rows, np.int64)
    m = len(t) if rows is None else len(rows_a)
    Fn = np.zeros((m, 3))
    Ef = np.zeros((m, 3))
    lib().ldo_ff_split_block(len(t), _dp(x), _ip(t), _dp(q), C.byref(make_params(params)), G,
                             L, B, _lp(rows_a), m, _dp(Fn), _dp(Ef))
    return Fn, Ef


def ff_local(mom, G: int, L: float, B: int = 5) -> np.ndarray:
    """[G^3, 19]: E, J (xx xy xz yy yz zz), H (xxx xxy xxz xyy xyz xzz yyy yyz
    yzz zzz) of the far cells' monopole + dipole field at every cell centre."""
    mom = np.ascontiguousarray(mom, np.float64)
    out = np.zeros((G ** 3, 19))
    lib().ldo_ff_local(G, L, B, _dp(mom), _dp(out))
    return out


def ff_local2(mom, G: int, L: float, B: int = 5, D: int = 2) -> np.ndarray:
    """Two-level version of ff_local (parents beyond D enter as a whole)."""
    mom = np.ascontiguousarray(mom, np.float64)
    out = np.zeros((G ** 3, 19))
    lib().ldo_ff_local2(G, L, B, D, _dp(mom), _dp(out))
    return out


def ff_local_eval(x, G: int, L: float, loc) -> np.ndarray:
    """Second-order local expansion evaluated at the points x [m,3]."""
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    loc = np.ascontiguousarray(loc, np.float64)
    E = np.zeros((len(x), 3))
    lib().ldo_ff_local_eval(len(x), _dp(x), G, L, _dp(loc), _dp(E))
    return E


def ff_features(x, G: int, L: float, B: int, mom, sq: float) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
    mom = np.ascontiguousarray(mom, np.float64)
    K = 4 * B ** 3 + 3
    X = np.zeros((len(x), K))
    lib().ldo_ff_features(len(x), _dp(x), G, L, B, _dp(mom), sq, _dp(X))
    return X


def mlp_forward(X, W, bf16_mode: bool = False, save: bool = False):
    """W = dict(W1 [K,H], b1, W2 [H,H], b2, W3 [H,O], b3)."""
    X = np.ascontiguousarray(X, np.float64)
    m, K = X.shape
    H = W["W1"].shape[1]
    O = W["W3"].shape[1]
    ws = [np.ascontiguousarray(W[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    Y = np.zeros((m, O))
    sv = [np.zeros((m, H)) for _ in range(4)] if save else [None] * 4
    lib().ldo_mlp_forward(m, K, H, O, _dp(X), *[_dp(w) for w in ws], 1 if bf16_mode else 0,
                          _dp(Y), *[_dp(a) for a in sv])
    return (Y, sv) if save else Y


def mlp_backward(X, T, W, bf16_mode: bool = False):
    """(loss, grads dict) for the mean-squared loss."""
    X = np.ascontiguousarray(X, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    m, K = X.shape
    H = W["W1"].shape[1]
    O = W["W3"].shape[1]
    ws = [np.ascontiguousarray(W[k], np.float64) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    g = {k: np.zeros_like(v) for k, v in zip(("W1", "b1", "W2", "b2", "W3", "b3"), ws)}
    loss = lib().ldo_mlp_backward(m, K, H, O, _dp(X), _dp(T), *[_dp(w) for w in ws],
                                  1 if bf16_mode else 0,
                                  *[_dp(g[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    return loss, g


# ---------------------------------------------------------------------------
# The paper's own scheme (section 2.2 steps (i)-(vi) read literally)
# ---------------------------------------------------------------------------

def make_paper(range_factor: float, kick: float, inertial_mass) -> _Paper:
    s = _Paper()
    s.range_factor = float(range_factor)
    s.kick = float(kick)
    for t, m in enumerate(inertial_mass):
        s.inertial_mass[t] = float(m)
    return s


def paper_forces(pos, type_, charge, params, range_factor: float, rows=None):
    """Pair forces truncated at range_factor (r_i + r_j), r = sigma/2 (section
    2.2 steps (i)-(ii)): returns (F [m,3], S [m]) for all particles or the
    listed rows."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    q = np.ascontiguousarray(charge, dtype=np.float64)
    n = len(type_)
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    k = n if rows is None else len(rows_a)
    F = np.zeros((k, 3))
    S = np.zeros(k)
    m = make_paper(range_factor, 0.0, [1.0] * MAX_TYPES)
    lib().ldo_paper_forces(n, _dp(pos), _ip(type_), _dp(q), C.byref(make_params(params)),
                           C.byref(m), None if rows is None else _lp(rows_a), k, _dp(F), _dp(S))
    return F, S


class PaperState:
    """Oracle state of the paper's scheme: FP64 positions and velocities."""

    def __init__(self, w, range_factor: float, kick: float, inertial_mass, pos=None, vel=None):
        self.w = w
        self.x = np.array(w.pos if pos is None else pos, dtype=np.float64).reshape(-1, 3).copy()
        self.v = (np.zeros_like(self.x) if vel is None
                  else np.array(vel, dtype=np.float64).reshape(-1, 3).copy())
        self.type = np.ascontiguousarray(w.type, dtype=np.int32)
        self.q = np.ascontiguousarray(w.charge, dtype=np.float64)
        self.m = make_paper(range_factor, kick, inertial_mass)
        self.step = 0
        self.t = 0.0

    def run(self, n_steps: int, dt: float = None) -> int:
        """Steps (iii)-(vi): Newton + Stokes drag, velocity kick, x += dt v."""
        dt = self.w.dt if dt is None else dt
        st = C.c_int64(self.step)
        tt = C.c_double(self.t)
        bad = lib().ldo_paper_run(len(self.type), _dp(self.x), _dp(self.v), _ip(self.type),
                                  _dp(self.q), None, C.byref(make_params(self.w.params)),
                                  C.byref(self.m), C.byref(make_radius(self.w.radius)), dt,
                                  n_steps, self.w.seed, C.byref(st), C.byref(tt))
        self.step, self.t = st.value, tt.value
        return bad


# ---------------------------------------------------------------------------
# Aggregate statistics (section 2.1: number of sub-aggregates; section 1: N_surf)
# ---------------------------------------------------------------------------

def components(x, type_, params, contact_factor: float = 1.1):
    """Connected components of the contact graph (r < contact_factor
    sigma_ij): returns (count, labels = smallest index of each component)."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    labels = np.zeros(len(type_), np.int64)
    n = lib().ldo_components(len(type_), _dp(x), _ip(type_), C.byref(make_params(params)),
                             contact_factor, _lp(labels))
    return n, labels


def surface_fractal(x, type_, params, R: float, contact_factor: float = 1.1,
                    k_f: float = math.pi / math.sqrt(3.0), d: float = 0.0):
    """Surface fractal dimension of the largest surface aggregate: returns
    (stats [components, largest size, its label], out [R_g, d, D_f],
    labels (-1 off the surface))."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    stats = np.zeros(3, np.int64)
    out = np.zeros(3)
    labels = np.zeros(len(type_), np.int64)
    lib().ldo_surface_fractal(len(type_), _dp(x), _ip(type_), C.byref(make_params(params)), R,
                              contact_factor, k_f, d, _lp(stats), _dp(out), _lp(labels))
    return stats, out, labels


def surface_count(x, type_, params, R: float) -> np.ndarray:
    """N_surf per type: NPs with | |x| - R | < sigma_t / 2."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
    type_ = np.ascontiguousarray(type_, dtype=np.int32)
    counts = np.zeros(len(params.sigma), np.int64)
    lib().ldo_surface_count(len(type_), _dp(x), _ip(type_), C.byref(make_params(params)), R,
                            _lp(counts))
    return counts
