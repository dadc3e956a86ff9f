"""Pins for the oracle's aggregate statistics: the contact-graph components
(the paper's number of sub-aggregates) against scipy's kd-tree pairs and
sparse-graph connected components, and against hand-built chains; N_surf
against constructed shells."""
import math

import numpy as np
import pytest

from paper_2501_04456_amd import workloads as W


def params(sigma):
    T = len(sigma)
    return W.Params(sigma=list(sigma), eps=[1.0] * T, mass=[1.0] * T, gamma=[1.0] * T,
                    k_wall=[0.0] * T, wall_offset=[0.0] * T, bjerrum=0.7, kT=1.0)


def scipy_labels(x, typ, sigma, f):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    sig = np.asarray(sigma)[typ]
    pairs = cKDTree(x).query_pairs(f * sig.max(), output_type="ndarray")
    i, j = pairs[:, 0], pairs[:, 1]
    d = np.linalg.norm(x[i] - x[j], axis=1)
    keep = d < f * 0.5 * (sig[i] + sig[j])
    n = len(x)
    g = coo_matrix((np.ones(keep.sum()), (i[keep], j[keep])), shape=(n, n))
    nc, lab = connected_components(g, directed=False)
    # canonical label: the smallest index of each component
    first = np.full(nc, n)
    np.minimum.at(first, lab, np.arange(n))
    return nc, first[lab]


@pytest.mark.parametrize("seed,f", [(1, 1.1), (2, 1.3), (3, 1.6)])
def test_components_match_scipy(oracle_lib, seed, f):
    rng = np.random.default_rng(seed)
    n = 1500
    x = rng.uniform(-9.0, 9.0, (n, 3))
    typ = (rng.random(n) < 0.3).astype(np.int32)
    sigma = [1.0, 1.8]
    nc, lab = oracle_lib.components(x, typ, params(sigma), f)
    nc2, lab2 = scipy_labels(x, typ, sigma, f)
    assert nc == nc2
    assert np.array_equal(lab, lab2)
    assert 1 < nc < n      # neither everything nor nothing is connected


def test_components_chains():
    import oracle
    oracle.lib()
    p = params([1.0])
    # a chain spaced 1.05 sigma is one component at factor 1.1, all
    # singletons at factor 1.0
    x = np.stack([np.arange(20) * 1.05, np.zeros(20), np.zeros(20)], 1)
    typ = np.zeros(20, np.int32)
    nc, lab = oracle.components(x, typ, p, 1.1)
    assert nc == 1 and np.all(lab == 0)
    nc, lab = oracle.components(x, typ, p, 1.0)
    assert nc == 20 and np.array_equal(lab, np.arange(20))
    # two chains apart, interleaved indices
    y = x + np.array([0.0, 50.0, 0.0])
    z = np.empty((40, 3))
    z[0::2], z[1::2] = x, y
    nc, lab = oracle.components(z, np.zeros(40, np.int32), p, 1.1)
    assert nc == 2 and np.all(lab[0::2] == 0) and np.all(lab[1::2] == 1)


def test_surface_count_shells():
    import oracle
    oracle.lib()
    p = params([1.0, 2.0])
    R = 10.0
    rng = np.random.default_rng(4)
    u = rng.normal(size=(12, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    # radii relative to R: type 0 counts within 0.5, type 1 within 1.0
    r = np.array([10.4, 9.6, 10.6, 9.4, 10.0, 12.0, 10.9, 9.1, 11.1, 8.9, 10.0, 5.0])
    typ = np.array([0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1], np.int32)
    x = u * r[:, None]
    c = oracle.surface_count(x, typ, p, R)
    assert list(c) == [3, 3]


# ---- surface fractal dimension (the fractal equation at dimension two) ----

KF2 = math.pi / math.sqrt(3.0)


def on_sphere(dirs, R):
    d = np.asarray(dirs, dtype=np.float64)
    return R * d / np.linalg.norm(d, axis=1)[:, None]


def rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def hex_disk(a):
    """Hexagonal lattice points (spacing 1) within radius a of a lattice point."""
    i, j = np.meshgrid(np.arange(-2 * a, 2 * a + 1), np.arange(-2 * a, 2 * a + 1))
    p = (i + 0.5 * j).ravel().astype(np.float64)
    q = (j * math.sqrt(3.0) / 2).ravel()
    m = p * p + q * q <= a * a
    return p[m], q[m]


def exp_map(p, q, R):
    """Points of the tangent plane at the north pole carried onto the sphere
    of radius R along geodesics (distances from the pole are kept)."""
    rho = np.hypot(p, q)
    phi = np.arctan2(q, p)
    t = rho / R
    return R * np.stack([np.sin(t) * np.cos(phi), np.sin(t) * np.sin(phi), np.cos(t)], 1)


def test_surface_fractal_two_nps():
    """Two NPs in contact on the sphere: the centre is their bisector, so R_g
    is half the geodesic distance R theta."""
    import oracle
    oracle.lib()
    R, theta = 10.0, 0.09
    x = on_sphere([[1.0, 0.0, 0.0], [math.cos(theta), math.sin(theta), 0.0]], R)
    typ = np.zeros(2, np.int32)
    st, out, lab = oracle.surface_fractal(x, typ, params([1.0]), R, 1.1)
    assert list(st) == [1, 2, 0] and list(lab) == [0, 0]
    assert out[0] == pytest.approx(R * theta / 2, rel=1e-12)
    assert out[1] == 1.0
    assert out[2] == pytest.approx(math.log(2 / KF2) / math.log(R * theta), rel=1e-12)


def test_surface_fractal_ring_is_geodesic():
    """M NPs on the small circle at polar angle alpha about an axis: every
    geodesic distance from the axis is R alpha, so R_g = R alpha (the chord
    2 R sin(alpha/2) and the projected radius R sin(alpha) differ by ~1 %);
    a smaller ring elsewhere is another, smaller component."""
    import oracle
    oracle.lib()
    rng = np.random.default_rng(7)
    R, alpha, M = 20.0, 0.6, 80
    phi = 2 * math.pi * np.arange(M) / M
    ring = np.stack([np.sin(alpha) * np.cos(phi), np.sin(alpha) * np.sin(phi),
                     np.full(M, math.cos(alpha))], 1)
    small = np.stack([np.sin(0.2) * np.cos(phi[:40] * 2), np.sin(0.2) * np.sin(phi[:40] * 2),
                      np.full(40, -math.cos(0.2))], 1)
    Q = rotation(rng)
    # the small ring first, so the largest component's label is not 0
    x = on_sphere(np.concatenate([small, ring]) @ Q.T, R)
    typ = np.zeros(len(x), np.int32)
    st, out, lab = oracle.surface_fractal(x, typ, params([1.0]), R, 1.1)
    assert list(st) == [2, M, 40]
    assert np.all(lab[:40] == 0) and np.all(lab[40:] == 40)
    assert out[0] == pytest.approx(R * alpha, rel=1e-12)
    assert abs(out[0] - 2 * R * math.sin(alpha / 2)) > 0.1
    assert out[2] == pytest.approx(math.log(M / KF2) / math.log(2 * R * alpha), rel=1e-12)


@pytest.mark.parametrize("R", [30.0, 1e5])
def test_surface_fractal_compact_hex_disk_is_two_dimensional(R):
    """A hexagonal disk (spacing sigma) laid on the sphere along geodesics
    from its centre: R_g equals the planar radius of gyration (geodesic
    distances from the centre are kept, and the six-fold symmetry puts the
    mean direction at the centre) on a curved and a nearly flat sphere, and
    with k_f = pi / sqrt(3) (twice the hexagonal packing fraction, the planar
    analogue of the 3-D compact prefactor) its D_f is 2."""
    import oracle
    oracle.lib()
    p, q = hex_disk(12)
    x = exp_map(p, q, R)
    typ = np.zeros(len(x), np.int32)
    st, out, lab = oracle.surface_fractal(x, typ, params([1.0]), R, 1.1)
    assert st[0] == 1 and st[1] == len(p)
    assert out[0] == pytest.approx(math.sqrt(np.mean(p * p + q * q)), rel=1e-11)
    assert abs(out[2] - 2.0) < 1e-3
    # the 3-D analogue reproduces the paper's compact prefactor 1.593
    assert math.pi / (3 * math.sqrt(2.0)) * (5.0 / 3.0) ** 1.5 == pytest.approx(1.593, abs=5e-4)


def clustered_surface(seed, sigma, R=25.0):
    return W.surface_clusters(1200, 600, R, sigma, seed)


@pytest.mark.parametrize("seed,f", [(11, 1.1), (12, 1.4)])
def test_surface_fractal_components_match_scipy(seed, f):
    """Labels of surface NPs = scipy's components of the contact graph among
    the surface NPs only; -1 elsewhere; the largest and its R_g recomputed
    with numpy (arccos of the normalised mean direction)."""
    import oracle
    oracle.lib()
    sigma = [1.0, 1.6]
    R = 25.0
    x, typ = clustered_surface(seed, sigma=sigma, R=R)
    st, out, lab = oracle.surface_fractal(x, typ, params(sigma), R, f)
    sig = np.asarray(sigma)[typ]
    surf = np.abs(np.linalg.norm(x, axis=1) - R) < 0.5 * sig
    ids = np.flatnonzero(surf)
    nc, lab_s = scipy_labels(x[ids], typ[ids], sigma, f)
    want = np.full(len(x), -1)
    want[ids] = ids[lab_s]
    assert np.array_equal(lab, want)
    assert st[0] == nc
    sizes = np.bincount(lab[ids], minlength=len(x))
    big = int(np.argmax(sizes))            # first maximum = smallest label
    assert st[1] == sizes[big] and st[2] == big
    mem = lab == big
    u = x[mem] / np.linalg.norm(x[mem], axis=1)[:, None]
    u0 = u.sum(0) / np.linalg.norm(u.sum(0))
    rg = R * math.sqrt(np.mean(np.arccos(np.clip(u @ u0, -1, 1)) ** 2))
    assert out[0] == pytest.approx(rg, rel=1e-10)
    assert out[1] == pytest.approx(sig[mem].mean(), rel=1e-12)
    assert 1 < st[0] < len(ids)


def test_surface_fractal_rotation_invariant():
    import oracle
    oracle.lib()
    sigma = [1.0, 1.6]
    x, typ = clustered_surface(13, sigma=sigma)
    st, out, lab = oracle.surface_fractal(x, typ, params(sigma), 25.0, 1.2)
    Q = rotation(np.random.default_rng(5))
    st2, out2, lab2 = oracle.surface_fractal(x @ Q.T, typ, params(sigma), 25.0, 1.2)
    assert np.array_equal(st, st2) and np.array_equal(lab, lab2)
    assert np.allclose(out, out2, rtol=1e-9, atol=0)


def test_surface_fractal_degenerate():
    import oracle
    oracle.lib()
    p = params([1.0])
    x = np.array([[0.0, 0.0, 5.0], [0.0, 3.0, 0.0], [1.0, 1.0, 1.0]])
    typ = np.zeros(3, np.int32)
    # no NP within half a diameter of the surface
    st, out, lab = oracle.surface_fractal(x, typ, p, 9.0)
    assert list(st) == [0, 0, -1] and np.all(np.isnan(out)) and np.all(lab == -1)
    # one surface NP: R_g = 0, no dimension
    st, out, lab = oracle.surface_fractal(x, typ, p, 5.2)
    assert list(st) == [1, 1, 0] and list(lab) == [0, -1, -1]
    assert out[0] == 0.0 and out[1] == 1.0 and math.isnan(out[2])
    # an explicit d replaces the mean diameter
    st, out, _ = oracle.surface_fractal(on_sphere([[1, 0, 0], [1, 0.08, 0]], 10.0), np.zeros(2, np.int32),
                                        p, 10.0, 1.1, KF2, 2.0)
    assert out[1] == 2.0


def test_surface_fractal_tie_takes_the_smaller_label():
    import oracle
    oracle.lib()
    R = 20.0
    phi = 2 * math.pi * np.arange(30) / 30
    ring = lambda z: np.stack([0.2 * np.cos(phi), 0.2 * np.sin(phi), np.full(30, z)], 1)
    x = on_sphere(np.concatenate([ring(1.0), ring(-1.0)]), R)
    x = x[::-1].copy()                  # the ring at z < 0 now holds the smaller indices
    st, out, lab = oracle.surface_fractal(x, np.zeros(60, np.int32), params([1.0]), R, 1.1)
    assert list(st) == [2, 30, 0]
    assert np.all(lab[:30] == 0) and np.all(lab[30:] == 30)


def test_surface_fractal_membership_band():
    """Only NPs within half a diameter of the surface take part: NPs at
    0.4 and 0.6 diameters from it (inside and outside, two types), spread
    over the sphere so that none are in contact, are labelled exactly by
    | |x| - R | < sigma_t / 2."""
    import oracle
    oracle.lib()
    p = params([1.0, 2.0])
    R = 30.0
    rng = np.random.default_rng(8)
    u = rng.normal(size=(16, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    typ = np.array([0, 1] * 8, np.int32)
    sig = np.array([1.0, 2.0])[typ]
    f = np.array([0.4, -0.4, 0.6, -0.6] * 4)
    r = R + f * sig
    x = u * r[:, None]
    st, out, lab = oracle.surface_fractal(x, typ, p, R, 1.1)
    want = np.abs(r - R) < 0.5 * sig
    assert np.array_equal(lab >= 0, want) and want.sum() == 8
    assert st[0] == 8                      # all singletons
