"""GPU parity of the paper's own scheme (section 2.2 steps (i)-(vi) read
literally: pairs truncated at range_factor (r_i + r_j), Newton + Stokes drag,
random velocity kick) against the FP64 oracle, through the C ABI.

Both sides compute the pair terms in FP64 from the same FP64 positions; the
GPU takes q_hat = q sqrt(kT l_B) from the FP32 charge slot of its position
array (relative rounding <= 2^-24 per charge), so forces agree to
max_i |dF_i| <= 2.5e-7 S_i (two roundings plus FP64 sums).  Trajectories: positions
within 1e-4 sigma and velocities within 1e-4 after 100 steps (the noise's
Box-Muller runs in FP32 on the GPU and in FP64 in the oracle)."""
import numpy as np
import pytest

from paper_2501_04456_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ld():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_04456_amd import ldrop
    ldrop.lib()
    return ldrop


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.lib()
    return oracle


def band_wall(w):
    """The paper's spring: equilibrium one radius inside the surface, acting
    only within one radius of it."""
    p = w.params
    p.wall_band = 1
    p.wall_offset = [0.5 * s for s in p.sigma]
    return w


CASES = {
    "small": lambda: W.config_small(),
    "medium3000": lambda: W.config_medium(n=3000, seed=21),
    "large3000": lambda: W.config_large(n=3000, seed=22),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("factor", [4.0, 2.5, 9.0])
def test_paper_forces(ld, orc, case, factor):
    w = CASES[case]()
    s = ld.System.from_workload(w)
    s.paper_enable(range_factor=factor)
    Fg = s.paper_forces()
    Fo, So = orc.paper_forces(w.pos, w.type, w.charge, w.params, factor)
    dF = np.linalg.norm(Fg - Fo, axis=1)
    assert np.all(dF <= 2.5e-7 * So), (case, factor, (dF / np.maximum(So, 1e-300)).max())
    # the truncation matters at these sizes (differs from the all-pairs sum)
    if factor == 2.5:
        Fa, _, _ = orc.pair_forces(w.pos, w.type, w.charge, w.params)
        assert np.abs(Fa - Fo).max() > 1e-6


@pytest.mark.parametrize("case,kick,band", [("small", 0.05, False), ("medium3000", 0.02, True),
                                            ("large3000", 0.0, True)])
def test_paper_trajectory(ld, orc, case, kick, band):
    w = CASES[case]()
    if band:
        band_wall(w)
    # inertial masses differ from the buoyant masses
    mass = [1.5 * m + 0.2 for m in w.params.mass]
    steps = 100
    s = ld.System.from_workload(w)
    s.paper_enable(range_factor=4.0, kick=kick, inertial_mass=mass)
    s.step(steps, w.dt)
    s.sync()
    st = orc.PaperState(w, 4.0, kick, mass)
    assert st.run(steps, w.dt) == -1
    xg = s.positions64()
    vg = s.velocities()
    assert np.abs(xg - st.x).max() <= 1e-4, np.abs(xg - st.x).max()
    assert np.abs(vg - st.v).max() <= 1e-4 * max(1.0, np.abs(st.v).max())
    step, t, _ = s.state()
    assert step == steps and t == pytest.approx(steps * w.dt, rel=1e-12)
    # the system moved
    assert np.abs(st.x - w.pos).max() > 1e-3


def test_paper_drag_decay_and_velocity_io(ld):
    """No forces (no LJ, no charge, no wall): v_n = a^n v_0 with
    a = 1 - gamma dt / m; set/get velocities round-trip in original order."""
    w = W.config_small(n=500, seed=4)
    p = w.params
    p.eps = [0.0]
    p.k_wall = [0.0]
    w.charge = np.zeros(w.n)
    s = ld.System.from_workload(w)
    m = 2.5
    s.paper_enable(range_factor=4.0, kick=0.0, inertial_mass=[m])
    rng = np.random.default_rng(3)
    v0 = rng.normal(size=(w.n, 3))
    s.set_velocities(v0)
    assert np.array_equal(s.velocities(), v0)
    n, dt = 40, w.dt
    s.step(n, dt)
    s.sync()
    a = 1 - p.gamma[0] * dt / m
    assert np.allclose(s.velocities(), a ** n * v0, rtol=1e-12, atol=0)
    x = s.positions64()
    assert np.allclose(x, w.pos + dt * v0 * a * (1 - a ** n) / (1 - a), rtol=0, atol=1e-9)


def test_paper_mode_guards_and_back(ld, orc):
    w = W.config_small(n=300, seed=6)
    s = ld.System.from_workload(w)
    s.paper_enable(range_factor=4.0, kick=0.01)
    with pytest.raises(RuntimeError):
        s.ff_enable(grid=8, block=3, hidden=16)
    with pytest.raises(RuntimeError):
        s.paper_enable(range_factor=-1.0)
    s.step(10, w.dt)
    s.paper_disable()
    with pytest.raises(RuntimeError):
        s.velocities()
    # back on the overdamped scheme: from the initial positions again, the
    # forces match the all-pairs oracle
    s.set_positions(w.pos)
    Fo, So, _ = orc.pair_forces(w.pos.astype(np.float64), w.type, w.charge, w.params)
    Fg = s.forces(ext=False)["pair"].cpu().numpy()
    assert np.all(np.linalg.norm(Fg - Fo, axis=1) <= 1e-5 * So)
    s.step(5, w.dt)
    assert s.state()[0] == 15
    x = s.positions64()
    assert np.isfinite(x).all() and np.abs(x - w.pos.astype(np.float64)).max() > 0
