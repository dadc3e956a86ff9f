"""Seeded synthetic droplet workloads.

This module only *generates inputs*: particle counts, type assignments,
per-particle charges, per-type parameters, droplet-radius schedules, time
steps, seeds and initial positions.  It holds none of the model's force or
update arithmetic, so the GPU library's callers and the CPU oracle can both
take their inputs from it without sharing any of the computation under test.

The paper (section 2.1) places NPs of several types uniformly at random in a
sphere of the initial droplet radius; the workloads below make that concrete
in reduced units (lengths in units of the type-0 diameter, energies in kT):

* ``config_small``  - N=1000, one type, alternating charges +-0.5, harmonic
  wall shrinking linearly 40 -> 15 over 1000 steps of dt=1e-3.
* ``config_medium`` - N=32768, two types 70/30 (sigma 1/1.5, eps 1/2,
  charges +1/-1), gravity, centrifugal term, square-law drying to a dry
  aggregate at step 2e4 (dt=5e-4).
* ``config_large``  - N=250000, three types 50/30/20 (sigma 1/1.3/2, eps
  1/1.5/3, charges +1/-1/0) in a sphere of 300, the full set of external
  forces, linear shrink 300 -> 112.5 over 1e4 steps of dt=5e-4.
* ``config_ensemble`` - 256 independent droplets, N log-uniform in
  [500, 8000], two-type mixes, volume fraction 1e-3, square-law drying with a
  per-droplet rate multiplier in [0.5, 2].
* ``config_learned`` - the medium system's composition scaled to N=250000
  for the learned far field.
* ``surface_clusters`` - positions and types only: patches of NPs on the
  droplet surface plus interior NPs, for the surface statistics.

Type fractions are assigned in index blocks (the first round(f0 N) particles
are type 0, ...); positions are i.i.d., so this is equal in law to a shuffle.
Positions are rejection-sampled so that no pair starts closer than its
contact distance sigma_ij, then rounded to FP32.

Per-type defaults: Stokes drag gamma_t = sigma_t (gamma_0 = 1) and buoyant
mass m_t = sigma_t^3 (uniform density contrast), both relative to type 0.
"""
from __future__ import annotations

import copy
import dataclasses
import math
from typing import Optional

import numpy as np

MAX_TYPES = 8

RADIUS_CONST = 0
RADIUS_LINEAR = 1
RADIUS_SQUARE_LAW = 2
RADIUS_TABLE = 3
RADIUS_TABLE_MAX = 16

NOISE_OFF = 0
NOISE_GAUSS = 1
NOISE_FIXED = 2


@dataclasses.dataclass
class Params:
    """Physical parameters of one droplet (all reduced units)."""
    sigma: list
    eps: list
    mass: list
    gamma: list
    k_wall: list
    wall_offset: list
    eps_matrix: Optional[list] = None   # T x T, or None for Lorentz-Berthelot
    lj_cut: float = 2.5                 # in units of sigma_ij
    coul_cut: float = 0.0               # <= 0: all pairs
    bjerrum: float = 0.7
    kT: float = 1.0
    gravity: tuple = (0.0, 0.0, 0.0)
    omega: float = 0.0
    rotation: int = 0                   # 0 isotropic, 1 about z
    wall_band: int = 0
    noise: int = NOISE_GAUSS
    jump_max: float = 0.5

    @property
    def n_types(self) -> int:
        return len(self.sigma)


@dataclasses.dataclass
class Radius:
    kind: int = RADIUS_CONST
    R0: float = 0.0
    R1: float = 0.0
    T: float = 0.0
    a: float = 0.0
    R_min: float = 0.0
    knots_t: tuple = ()      # RADIUS_TABLE: increasing knot times
    knots_R: tuple = ()      # RADIUS_TABLE: radii at the knots


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    type: np.ndarray        # int32 [n]
    charge: np.ndarray      # float64 [n]
    pos: np.ndarray         # float32 [n, 3]
    params: Params
    radius: Radius
    dt: float
    n_steps: int
    seed: int

    def replace(self, **kw) -> "Workload":
        w = copy.copy(self)
        for k, v in kw.items():
            setattr(w, k, v)
        return w


# ---------------------------------------------------------------------------
# Position sampling
# ---------------------------------------------------------------------------

def _ball(rng: np.random.Generator, m: int, R: float) -> np.ndarray:
    v = rng.standard_normal((m, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = R * rng.random(m) ** (1.0 / 3.0)
    return v * r[:, None]


def sample_positions(type_: np.ndarray, sigma: list, R0: float, seed: int,
                     max_rounds: int = 200) -> np.ndarray:
    """Uniform positions in a ball of radius R0 with every pair at least
    sigma_ij = (sigma_i + sigma_j)/2 apart; returns float32 [n, 3]."""
    from scipy.spatial import cKDTree

    n = len(type_)
    rng = np.random.Generator(np.random.Philox(key=seed))
    sig = np.asarray(sigma, dtype=np.float64)[type_]
    x = _ball(rng, n, R0)
    reach = float(np.max(sigma))
    for _ in range(max_rounds):
        x32 = x.astype(np.float32).astype(np.float64)
        pairs = cKDTree(x32).query_pairs(reach, output_type="ndarray")
        if len(pairs) == 0:
            return x32.astype(np.float32)
        i, j = pairs[:, 0], pairs[:, 1]
        d = np.linalg.norm(x32[i] - x32[j], axis=1)
        bad = d < 0.5 * (sig[i] + sig[j])
        if not np.any(bad):
            return x32.astype(np.float32)
        redo = np.unique(np.maximum(i[bad], j[bad]))
        x[redo] = _ball(rng, len(redo), R0)
    raise RuntimeError("rejection sampling did not converge")


def _blocks(n: int, fractions) -> np.ndarray:
    counts = [int(round(f * n)) for f in fractions[:-1]]
    counts.append(n - sum(counts))
    return np.repeat(np.arange(len(fractions), dtype=np.int32), counts)


def dry_radius(type_: np.ndarray, sigma: list, phi_rcp: float = 0.64) -> float:
    """Radius of the dry aggregate: all NP volume at random close packing."""
    s3 = float(np.sum(np.asarray(sigma, dtype=np.float64)[type_] ** 3))
    return (s3 / (8.0 * phi_rcp)) ** (1.0 / 3.0)


def _stokes(sigma):
    return [s / sigma[0] for s in sigma]


def _buoyant(sigma):
    return [(s / sigma[0]) ** 3 for s in sigma]


# ---------------------------------------------------------------------------
# The workloads
# ---------------------------------------------------------------------------

def config_small(n: int = 1000, seed: int = 1, with_positions: bool = True) -> Workload:
    """N=1000, one type (sigma=1, eps=1), charges +0.5 (even index) / -0.5,
    kT=1, gamma=1, LJ cut 2.5, Coulomb over all pairs with l_B=0.7, harmonic
    wall k=50 at R(t) shrinking linearly 40 -> 15 over 1000 steps of 1e-3."""
    scale = (n / 1000.0) ** (1.0 / 3.0)
    R0 = 40.0 * scale
    type_ = np.zeros(n, dtype=np.int32)
    charge = np.where(np.arange(n) % 2 == 0, 0.5, -0.5).astype(np.float64)
    sigma = [1.0]
    p = Params(sigma=sigma, eps=[1.0], mass=[1.0], gamma=[1.0], k_wall=[50.0],
               wall_offset=[0.0], bjerrum=0.7, kT=1.0)
    dt, steps = 1e-3, 1000
    R = Radius(kind=RADIUS_LINEAR, R0=R0, R1=15.0 * scale, T=steps * dt)
    pos = sample_positions(type_, sigma, R0, seed) if with_positions else None
    return Workload("small", n, type_, charge, pos, p, R, dt, steps, seed)


def config_medium(n: int = 32768, seed: int = 2, with_positions: bool = True) -> Workload:
    """N=32768, 70/30 of (sigma 1.0/1.5, eps 1.0/2.0, LB mixing, charges
    +1/-1), gravity 0.05 along -z, isotropic centrifugal omega=0.02, wall
    k=100, square-law drying R^2 = R0^2 - 2 a t from R0=120 (scaled to keep
    the volume fraction) to the dry radius at step 2e4, dt=5e-4."""
    scale = (n / 32768.0) ** (1.0 / 3.0)
    R0 = 120.0 * scale
    sigma = [1.0, 1.5]
    type_ = _blocks(n, [0.7, 0.3])
    charge = np.where(type_ == 0, 1.0, -1.0).astype(np.float64)
    dt, steps = 5e-4, 20000
    Rdry = dry_radius(type_, sigma)
    a = (R0 * R0 - Rdry * Rdry) / (2.0 * steps * dt)
    p = Params(sigma=sigma, eps=[1.0, 2.0], mass=_buoyant(sigma), gamma=_stokes(sigma),
               k_wall=[100.0, 100.0], wall_offset=[0.0, 0.0], bjerrum=0.7, kT=1.0,
               gravity=(0.0, 0.0, -0.05), omega=0.02)
    R = Radius(kind=RADIUS_SQUARE_LAW, R0=R0, a=a, R_min=Rdry)
    pos = sample_positions(type_, sigma, R0, seed) if with_positions else None
    return Workload("medium", n, type_, charge, pos, p, R, dt, steps, seed)


def config_large(n: int = 250000, seed: int = 3, with_positions: bool = True) -> Workload:
    """N=250000, 50/30/20 of (sigma 1/1.3/2, eps 1/1.5/3, LB, charges
    +1/-1/0) uniform in R0=300 (scaled with n to keep the volume fraction),
    kT=1, wall k=50 shrinking linearly by the small config's ratio 15/40 over
    1e4 steps of dt=5e-4, plus gravity 0.05 along -z and omega=0.02."""
    scale = (n / 250000.0) ** (1.0 / 3.0)
    R0 = 300.0 * scale
    sigma = [1.0, 1.3, 2.0]
    type_ = _blocks(n, [0.5, 0.3, 0.2])
    charge = np.select([type_ == 0, type_ == 1], [1.0, -1.0], 0.0).astype(np.float64)
    dt, steps = 5e-4, 10000
    p = Params(sigma=sigma, eps=[1.0, 1.5, 3.0], mass=_buoyant(sigma), gamma=_stokes(sigma),
               k_wall=[50.0] * 3, wall_offset=[0.0] * 3, bjerrum=0.7, kT=1.0,
               gravity=(0.0, 0.0, -0.05), omega=0.02)
    R = Radius(kind=RADIUS_LINEAR, R0=R0, R1=R0 * 15.0 / 40.0, T=steps * dt)
    pos = sample_positions(type_, sigma, R0, seed) if with_positions else None
    return Workload("large", n, type_, charge, pos, p, R, dt, steps, seed)


def config_learned(n: int = 250000, seed: int = 5, with_positions: bool = True) -> Workload:
    """The medium system's composition, externals and drying law at N=250000
    with R0 scaled to keep the initial volume fraction."""
    w = config_medium(n=n, seed=seed, with_positions=with_positions)
    w.name = "learned"
    return w


@dataclasses.dataclass
class Ensemble:
    name: str
    droplets: list          # list[Workload]
    dt: float
    n_steps: int

    @property
    def offsets(self) -> np.ndarray:
        o = np.zeros(len(self.droplets) + 1, dtype=np.int64)
        o[1:] = np.cumsum([d.n for d in self.droplets])
        return o


def config_ensemble(n_drop: int = 256, n_min: int = 500, n_max: int = 8000, seed: int = 4,
                    phi: float = 1e-3, with_positions: bool = True) -> Ensemble:
    """Independent droplets: N_d = round(exp U[ln n_min, ln n_max]); type-0
    fraction U[0.2, 0.8] of (sigma 1/1.5, eps 1/2, LB, charges +1/-1); wall
    k=50, kT=1, l_B=0.7, no gravity or rotation; R0 from volume fraction phi;
    square-law drying that would reach the dry radius at the last step, with
    the rate multiplied by U[0.5, 2]; droplet d has noise seed 4000 + d."""
    rng = np.random.Generator(np.random.Philox(key=seed))
    dt, steps = 1e-3, 5000
    sigma = [1.0, 1.5]
    drops = []
    for d in range(n_drop):
        nd = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        f0 = rng.uniform(0.2, 0.8)
        mult = rng.uniform(0.5, 2.0)
        type_ = _blocks(nd, [f0, 1.0 - f0])
        charge = np.where(type_ == 0, 1.0, -1.0).astype(np.float64)
        s3 = float(np.sum(np.asarray(sigma)[type_] ** 3))
        R0 = (s3 / (8.0 * phi)) ** (1.0 / 3.0)
        Rdry = dry_radius(type_, sigma)
        a = mult * (R0 * R0 - Rdry * Rdry) / (2.0 * steps * dt)
        p = Params(sigma=sigma, eps=[1.0, 2.0], mass=_buoyant(sigma), gamma=_stokes(sigma),
                   k_wall=[50.0, 50.0], wall_offset=[0.0, 0.0], bjerrum=0.7, kT=1.0)
        R = Radius(kind=RADIUS_SQUARE_LAW, R0=R0, a=a, R_min=Rdry)
        pos = sample_positions(type_, sigma, R0, 4000 + d) if with_positions else None
        drops.append(Workload(f"drop{d}", nd, type_, charge, pos, p, R, dt, steps, 4000 + d))
    return Ensemble("ensemble", drops, dt, steps)


CONFIGS = {
    "small": config_small,
    "medium": config_medium,
    "large": config_large,
    "learned": config_learned,
}


def surface_clusters(n_surf: int, n_in: int, R: float, sigma=(1.0, 1.6), seed: int = 0,
                     n_centres: int = 12, spread: float = 3.0, frac1: float = 0.3):
    """Positions (FP64, [n, 3]) and types of NPs in patches on the surface of
    a droplet of radius R plus NPs inside it, in a random order.

    Patch centres are uniform on the sphere; each surface NP picks a centre,
    moves from it by a Gaussian tangential offset of scale ``spread`` (a
    length) and sits within a quarter diameter of the surface radially.
    Interior NPs are uniform in the ball of radius 0.9 R.  Type 1 with
    probability ``frac1``.  NPs may overlap (inputs for post-processing, not
    for stepping)."""
    rng = np.random.default_rng(seed)
    sig = np.asarray(sigma, dtype=np.float64)
    centres = rng.normal(size=(n_centres, 3))
    centres /= np.linalg.norm(centres, axis=1)[:, None]
    k = rng.integers(0, n_centres, n_surf)
    d = centres[k] + rng.normal(scale=spread / R, size=(n_surf, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    typ_s = (rng.random(n_surf) < frac1).astype(np.int32)
    r = R + rng.uniform(-0.24, 0.24, n_surf) * sig[typ_s]
    xs = d * r[:, None]
    u = rng.normal(size=(n_in, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    xi = u * (0.9 * R * rng.random(n_in) ** (1.0 / 3.0))[:, None]
    typ_i = (rng.random(n_in) < frac1).astype(np.int32)
    x = np.concatenate([xs, xi])
    typ = np.concatenate([typ_s, typ_i])
    perm = rng.permutation(n_surf + n_in)
    return x[perm], typ[perm]
