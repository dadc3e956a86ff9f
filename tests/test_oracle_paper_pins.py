"""Pins for the oracle of the paper's own scheme (section 2.2 steps (i)-(vi)
read literally): pair forces truncated at range_factor (r_i + r_j), Newton's
equation with Stokes drag and a random velocity vector of fixed magnitude.

Each test checks it against something other than itself: the all-pairs
oracle where the two definitions coincide, truncation and Newton's third
law, closed forms of the drag decay and terminal velocity, the damped
harmonic trap through the scheme's 2x2 linear map raised to the n-th power
(numpy), and the kick's magnitude and isotropy.
"""
import numpy as np
import pytest

from paper_2501_04456_amd import workloads as W


def params(**kw):
    p = W.Params(sigma=[1.0, 1.6], eps=[1.0, 2.0], mass=[1.0, 4.1], gamma=[1.0, 1.6],
                 k_wall=[0.0, 0.0], wall_offset=[0.0, 0.0], bjerrum=0.7, kT=1.0,
                 noise=W.NOISE_OFF)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def cluster(n, seed, box=6.0, dmin=0.9):
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        x = rng.uniform(-box, box, 3)
        if all(np.linalg.norm(x - y) >= dmin for y in pts):
            pts.append(x)
    return np.array(pts)


def test_paper_forces_equal_all_pairs_when_everything_is_in_range(oracle_lib):
    x = cluster(60, 1)
    typ = (np.arange(60) % 2).astype(np.int32)
    q = np.where(np.arange(60) % 3 == 0, 1.0, -1.0)
    p = params(lj_cut=1e3, coul_cut=0.0)
    Fa, Sa, _ = oracle_lib.pair_forces(x, typ, q, p)
    Fp, Sp = oracle_lib.paper_forces(x, typ, q, p, range_factor=1e3)
    assert np.allclose(Fp, Fa, rtol=1e-12, atol=1e-12 * Sa.max())
    assert np.allclose(Sp, Sa, rtol=1e-12)


def test_paper_forces_one_type_equal_truncated_all_pairs(oracle_lib):
    """One type: range_factor (r + r) = range_factor sigma is the same radius
    for LJ and Coulomb, which the all-pairs oracle expresses as lj_cut =
    range_factor and coul_cut = range_factor sigma."""
    x = cluster(80, 2, box=5.0, dmin=1.2)
    typ = np.zeros(80, np.int32)
    q = np.where(np.arange(80) % 2 == 0, 1.0, -1.0)
    p = params(sigma=[1.3], eps=[1.0], mass=[1.0], gamma=[1.0], k_wall=[0.0],
               wall_offset=[0.0], lj_cut=3.0, coul_cut=3.0 * 1.3)
    Fa, Sa, _ = oracle_lib.pair_forces(x, typ, q, p)
    Fp, _ = oracle_lib.paper_forces(x, typ, q, p, range_factor=3.0)
    assert np.allclose(Fp, Fa, rtol=1e-12, atol=1e-12 * Sa.max())
    # and it differs from the untruncated sum
    Fu, _ = oracle_lib.paper_forces(x, typ, q, p, range_factor=1e3)
    assert np.abs(Fu - Fp).max() > 1e-3


@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 1)])
def test_paper_range_is_per_type_pair(oracle_lib, ta, tb):
    """Two particles: just inside range_factor (r_a + r_b) they feel the full
    LJ + Coulomb pair force (the all-pairs oracle's two-body value); just
    outside, nothing."""
    p = params(lj_cut=1e3, coul_cut=0.0)
    f = 4.0
    rint = f * 0.5 * (p.sigma[ta] + p.sigma[tb])
    typ = np.array([ta, tb], np.int32)
    q = np.array([1.0, -1.0])
    for r, inside in ((rint * (1 - 1e-9), True), (rint * (1 + 1e-9), False)):
        x = np.array([[0.1, 0.2, 0.3], [0.1 + r, 0.2, 0.3]])
        Fp, _ = oracle_lib.paper_forces(x, typ, q, p, range_factor=f)
        if inside:
            Fa, _, _ = oracle_lib.pair_forces(x, typ, q, p)
            assert np.allclose(Fp, Fa, rtol=1e-12, atol=0)
            assert np.abs(Fp).max() > 0
        else:
            assert np.all(Fp == 0.0)


def test_paper_forces_newton3_and_far_particles(oracle_lib):
    x = cluster(70, 3)
    typ = (np.arange(70) % 2).astype(np.int32)
    q = np.where(np.arange(70) % 2 == 0, 1.0, -1.0)
    p = params()
    F, S = oracle_lib.paper_forces(x, typ, q, p, range_factor=4.0)
    assert np.abs(F.sum(0)).max() <= 1e-12 * S.sum()
    # particles beyond everyone's range change nothing
    far = x[:10] + np.array([1e4, 0, 0])
    x2 = np.vstack([x, far])
    F2, _ = oracle_lib.paper_forces(x2, np.concatenate([typ, typ[:10]]),
                                    np.concatenate([q, q[:10]]), p, range_factor=4.0)
    assert np.array_equal(F2[:70], F)


def lone(p, x0, dt, steps, seed=1, R0=1e6):
    R = W.Radius(kind=W.RADIUS_CONST, R0=R0)
    x0 = np.asarray(x0, np.float64).reshape(-1, 3)
    n = len(x0)
    return W.Workload("t", n, np.zeros(n, np.int32), np.zeros(n), x0, p, R, dt, steps, seed)


def one(**kw):
    base = dict(sigma=[1.0], eps=[0.0], mass=[1.0], gamma=[2.0], k_wall=[0.0],
                wall_offset=[0.0])
    base.update(kw)
    return params(**base)


def test_drag_decay_closed_form(oracle_lib):
    """No force: v_n = a^n v_0 and x_n = x_0 + dt v_0 a (1 - a^n) / (1 - a),
    a = 1 - gamma dt / m."""
    m, g, dt, n = 0.5, 2.0, 1e-3, 300
    w = lone(one(gamma=[g]), [[1.0, 2.0, 3.0]], dt, n)
    v0 = np.array([[0.3, -0.2, 0.5]])
    st = oracle_lib.PaperState(w, 4.0, 0.0, [m], vel=v0)
    assert st.run(n, dt) == -1
    a = 1 - g * dt / m
    assert np.allclose(st.v, a ** n * v0, rtol=1e-12)
    assert np.allclose(st.x, w.pos + dt * v0 * a * (1 - a ** n) / (1 - a), rtol=1e-12)
    assert st.step == n and st.t == pytest.approx(n * dt, rel=1e-12)


def test_terminal_velocity(oracle_lib):
    """Gravity on the buoyant mass m_b: v_n = (m_b g / gamma) (1 - a^n)."""
    mb, mi, g, dt, n = 2.0, 3.0, 4.0, 1e-2, 2000
    gz = -0.05
    w = lone(one(mass=[mb], gamma=[g], gravity=(0.0, 0.0, gz)), [[0.0, 0.0, 0.0]], dt, n)
    st = oracle_lib.PaperState(w, 4.0, 0.0, [mi])
    st.run(n, dt)
    a = 1 - g * dt / mi
    vinf = mb * gz / g
    assert st.v[0, 2] == pytest.approx(vinf * (1 - a ** n), rel=1e-11)
    assert st.v[0, 0] == 0.0 and st.v[0, 1] == 0.0


def test_damped_trap_linear_map(oracle_lib):
    """A wall at R_w = 0 is a full harmonic trap F = -k x.  Per component the
    scheme is the linear map (v, x) -> (a v - (k dt / m) x,
    (1 - k dt^2 / m) x + dt a v); its n-th power (numpy) gives the state."""
    k, m, g, dt, n = 30.0, 1.5, 0.4, 5e-3, 400
    w = lone(one(k_wall=[k], gamma=[g]), [[0.3, -0.2, 0.5]], dt, n, R0=0.0)
    v0 = np.array([[0.1, 0.0, -0.2]])
    st = oracle_lib.PaperState(w, 4.0, 0.0, [m], vel=v0)
    st.run(n, dt)
    a = 1 - g * dt / m
    M = np.array([[a, -k * dt / m], [dt * a, 1 - k * dt * dt / m]])
    Mn = np.linalg.matrix_power(M, n)
    for c in range(3):
        v, x = Mn @ np.array([v0[0, c], w.pos[0, c]])
        assert st.v[0, c] == pytest.approx(v, rel=1e-9, abs=1e-14)
        assert st.x[0, c] == pytest.approx(x, rel=1e-9, abs=1e-14)
    # it oscillates: the trap's frequency makes x change sign
    assert np.sign(st.x[0, 0]) != np.sign(w.pos[0, 0]) or abs(st.x[0, 0]) < abs(w.pos[0, 0])


def test_kick_magnitude_and_isotropy(oracle_lib):
    """From rest with no force, one step adds exactly `kick` to |v| (minus the
    drag on zero velocity: nothing), in a direction uniform on the sphere."""
    n, kick, dt = 4000, 0.7, 1e-3
    x0 = np.stack([np.arange(n) * 10.0, np.zeros(n), np.zeros(n)], 1)
    w = lone(one(), x0, dt, 1)
    st = oracle_lib.PaperState(w, 4.0, kick, [1.0])
    st.run(1, dt)
    speed = np.linalg.norm(st.v, axis=1)
    assert np.allclose(speed, kick, rtol=1e-12)
    u = st.v / kick
    assert np.abs(u.mean(0)).max() < 4.0 / np.sqrt(n)
    assert np.allclose((u ** 2).mean(0), 1.0 / 3.0, atol=0.03)
    assert np.allclose(st.x, x0 + dt * st.v, rtol=1e-12)


def test_paper_forces_rows_select():
    """Rows mode returns exactly the listed rows of the all-rows result."""
    import oracle
    oracle.lib()
    w = W.config_small(n=400, seed=9)
    F, S = oracle.paper_forces(w.pos, w.type, w.charge, w.params, 4.0)
    rows = np.array([399, 0, 17, 17, 250])
    Fr, Sr = oracle.paper_forces(w.pos, w.type, w.charge, w.params, 4.0, rows=rows)
    assert np.array_equal(Fr, F[rows]) and np.array_equal(Sr, S[rows])


def test_wall_uses_the_new_radius(oracle_lib):
    """Step (iii) precedes step (iv): with R shrinking linearly 10 -> 5 over
    T = 1 and dt = 0.1, an NP at |x| = 9.8 (inside R(0) = 10, outside
    R(0.1) = 9.5) gets v_1 = -dt k (9.8 - 9.5) / m along x from the first
    step."""
    k, m, dt = 50.0, 2.0, 0.1
    w = lone(one(k_wall=[k]), [[9.8, 0.0, 0.0]], dt, 1)
    w.radius = W.Radius(kind=W.RADIUS_LINEAR, R0=10.0, R1=5.0, T=1.0)
    st = oracle_lib.PaperState(w, 4.0, 0.0, [m])
    assert st.run(1, dt) == -1
    assert st.v[0, 0] == pytest.approx(-dt * k * (9.8 - 9.5) / m, rel=1e-12)
    assert st.v[0, 1] == 0.0 and st.v[0, 2] == 0.0
