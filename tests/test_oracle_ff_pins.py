"""Pins for the learned-far-field part of the oracle: BF16 rounding against
torch, moments against conservation and single-particle dipoles, the coarse
multipole field against exact point-charge sums, the near/far splits (radial
and block) against the (pinned) full pair sum and brute force, the local
expansion against finite differences of Coulomb's law, Laplace's equation
and its Taylor remainder, the feature layout, and the MLP forward / backward
against torch (CPU, FP64) and finite differences."""
import math

import numpy as np
import pytest
import torch

from paper_2501_04456_amd import workloads as W


def test_bf16_matches_torch(oracle_lib):
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.integers(-6, 6, 3000),
                           [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -(1.0 + 2 ** -8),
                            0.0, 65504.0, 1e30, -3.5e-20]])
    ref = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([oracle_lib.bf16(v) for v in vals])
    assert np.array_equal(got, ref)


def ball(n, R, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * (R * rng.random(n) ** (1 / 3))[:, None]


def test_moments_conservation_and_dipole(oracle_lib):
    x = ball(2000, 30.0, 1)
    q = np.where(np.arange(2000) % 3 == 0, 1.0, -0.5)
    G, L = 8, 32.0
    m = oracle_lib.ff_moments(x, q, G, L)
    assert m[:, 0].sum() == pytest.approx(q.sum(), abs=1e-9)
    # total dipole about the origin = sum over cells (P_c + Q_c centre_c)
    h = 2 * L / G
    idx = np.arange(G ** 3)
    cen = np.stack([(idx % G + 0.5) * h - L, ((idx // G) % G + 0.5) * h - L,
                    (idx // G ** 2 + 0.5) * h - L], 1)
    tot = (m[:, 1:] + m[:, :1] * cen).sum(0)
    assert np.allclose(tot, (q[:, None] * x).sum(0), rtol=1e-10, atol=1e-8)
    # a single particle: its cell holds q and q * offset
    one = oracle_lib.ff_moments(np.array([[3.0, -5.0, 12.0]]), np.array([2.0]), G, L)
    k = np.flatnonzero(one[:, 0])
    assert len(k) == 1
    c = cen[k[0]]
    assert np.allclose(one[k[0], 1:], 2.0 * (np.array([3.0, -5.0, 12.0]) - c))


def test_coarse_field_equals_point_charges_at_centres(oracle_lib):
    """Charges sitting exactly at cell centres have no dipole: the coarse
    field at a cell centre is the exact field of every charge outside the
    5^3 block around it (the far sum of ldo_ff_split with r_c = 0)."""
    G, L = 12, 24.0
    h = 2 * L / G
    rng = np.random.default_rng(2)
    cells = rng.choice(G ** 3, 300, replace=False)
    cen = lambda k: np.array([(k % G + 0.5) * h - L, ((k // G) % G + 0.5) * h - L,
                              (k // G ** 2 + 0.5) * h - L])
    x = np.array([cen(k) for k in cells])
    q = rng.uniform(-1, 1, len(cells))
    p = W.Params(sigma=[1e-3], eps=[0.0], mass=[1], gamma=[1], k_wall=[0], wall_offset=[0],
                 kT=1.0, bjerrum=1.0)
    m = oracle_lib.ff_moments(x, q, G, L)
    assert np.abs(m[:, 1:]).max() < 1e-12
    E = oracle_lib.ff_coarse(m, G, L, 5)
    for t in [0, 77, 500, G ** 3 - 1, int(cells[5])]:
        ct = cen(t)
        tz, ty, tx = t // G ** 2, (t // G) % G, t % G
        far = [i for i, k in enumerate(cells)
               if max(abs(k % G - tx), abs((k // G) % G - ty), abs(k // G ** 2 - tz)) > 2]
        xs = np.vstack([x[far], ct[None]])
        qs = np.concatenate([q[far], [0.0]])
        _, Ef = oracle_lib.ff_split(xs, np.zeros(len(xs), np.int32), qs, p, 0.0,
                                    rows=[len(xs) - 1])
        assert np.allclose(E[t], Ef[0], rtol=1e-12, atol=1e-14)


def test_coarse_dipole_accuracy(oracle_lib):
    """A +q/-q pair of small separation d in a distant cell: the dipole term
    reproduces the exact field to O((d/r)^2)."""
    G, L = 16, 32.0
    h = 2 * L / G
    src = np.array([[20.3, -7.1, 3.3], [20.3 + 0.4, -7.1 - 0.3, 3.3 + 0.2]])
    q = np.array([1.0, -1.0])
    m = oracle_lib.ff_moments(src, q, G, L)
    E = oracle_lib.ff_coarse(m, G, L, 5)
    t = (G // 2) * G * G + (G // 2) * G + 1          # a cell far from the pair
    ct = np.array([(1 + 0.5) * h - L, (G // 2 + 0.5) * h - L, (G // 2 + 0.5) * h - L])
    p = W.Params(sigma=[1e-3], eps=[0.0], mass=[1], gamma=[1], k_wall=[0], wall_offset=[0],
                 kT=1.0, bjerrum=1.0)
    _, Ef = oracle_lib.ff_split(np.vstack([src, ct[None]]), np.zeros(3, np.int32),
                                np.array([1.0, -1.0, 0.0]), p, 0.0, rows=[2])
    r = np.linalg.norm(src.mean(0) - ct)
    # the pair's dipole sits off the cell centre: error O((a/r)) relative, with
    # a the distance from the cell centre (below half a cell diagonal)
    assert np.linalg.norm(E[t] - Ef[0]) <= np.linalg.norm(Ef[0]) * 4 * (0.9 * h / r)


def test_split_sums_to_full_pair_force(oracle_lib):
    w = W.config_medium(n=400, seed=3)
    x = w.pos.astype(np.float64)
    F, S, _ = oracle_lib.pair_forces(x, w.type, w.charge, w.params)
    qh = oracle_lib.qhat(w.charge, w.params)
    # any cut beyond the largest LJ range (2.5 x 1.5) splits the sum exactly
    for rc in (3.76, 8.0, 20.0, 1e9):
        Fn, Ef = oracle_lib.ff_split(x, w.type, w.charge, w.params, rc)
        assert np.all(np.abs(Fn + qh[:, None] * Ef - F) <= 1e-12 * S[:, None] + 1e-15)
    # r_c = 0: everything is far, and the far sum is the pure Coulomb force
    Fn, Ef = oracle_lib.ff_split(x, w.type, w.charge, w.params, 0.0)
    assert np.all(Fn == 0)
    pc = W.Params(**{**w.params.__dict__})
    pc.eps = [0.0, 0.0]
    Fc, Sc, _ = oracle_lib.pair_forces(x, w.type, w.charge, pc)
    assert np.all(np.abs(qh[:, None] * Ef - Fc) <= 1e-12 * Sc[:, None] + 1e-15)
    Fn, Ef = oracle_lib.ff_split(x, w.type, w.charge, w.params, 1e9)
    assert np.all(Ef == 0)


def test_split_block_partition_and_membership(oracle_lib):
    """The block split partitions the pair sum (F_near + q_hat E_far = the
    pinned full pair force), and E_far is the brute-force Coulomb field of
    exactly the particles whose cells lie outside the B^3 block."""
    w = W.config_medium(n=600, seed=4)
    x = w.pos.astype(np.float64)
    F, S, _ = oracle_lib.pair_forces(x, w.type, w.charge, w.params)
    qh = oracle_lib.qhat(w.charge, w.params)
    L = float(np.abs(x).max()) * 1.001
    for G, B in ((8, 5), (16, 3), (6, 1), (4, 7)):
        Fn, Ef = oracle_lib.ff_split_block(x, w.type, w.charge, w.params, G, L, B)
        assert np.all(np.abs(Fn + qh[:, None] * Ef - F) <= 1e-12 * S[:, None] + 1e-15)
        h = 2 * L / G
        cell = np.clip(np.floor((x + L) / h).astype(int), 0, G - 1)
        for i in (0, 17, 333, 599):
            out = np.abs(cell - cell[i]).max(1) > B // 2
            d = x[i] - x[out]
            r = np.linalg.norm(d, axis=1)
            ref = (qh[out, None] * d / r[:, None] ** 3).sum(0)
            assert np.allclose(Ef[i], ref, rtol=1e-11, atol=1e-14)
    # a block covering the whole grid: nothing is far
    Fn, Ef = oracle_lib.ff_split_block(x, w.type, w.charge, w.params, 4, L, 7)
    assert np.all(Ef == 0)


def _cell_centre(k, G, L):
    h = 2 * L / G
    return np.array([(k % G + 0.5) * h - L, ((k // G) % G + 0.5) * h - L,
                     (k // G ** 2 + 0.5) * h - L])


def _fd_derivs(field, c, eps):
    """Central finite differences of a vector field: E(c), J[a][b] = dE_a/dx_b
    and H[a][b][e] = d2E_a/dx_b dx_e."""
    I = np.eye(3)
    E0 = field(c)
    J = np.zeros((3, 3))
    H = np.zeros((3, 3, 3))
    for b in range(3):
        J[:, b] = (field(c + eps * I[b]) - field(c - eps * I[b])) / (2 * eps)
        for e in range(3):
            H[:, b, e] = (field(c + eps * (I[b] + I[e])) - field(c + eps * (I[b] - I[e]))
                          - field(c - eps * (I[b] - I[e])) + field(c - eps * (I[b] + I[e]))) \
                / (4 * eps * eps)
    return E0, J, H


_JI = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
_HI = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1), (1, 1, 2),
       (1, 2, 2), (2, 2, 2)]


def _unpack(o):
    J = np.array([o[3 + _JI.index(tuple(sorted((a, b))))] for a in range(3) for b in range(3)])
    H = np.array([o[9 + _HI.index(tuple(sorted((a, b, e))))]
                  for a in range(3) for b in range(3) for e in range(3)])
    return o[:3], J.reshape(3, 3), H.reshape(3, 3, 3)


@pytest.mark.parametrize("kind", ["charge", "dipole"])
def test_local_expansion_matches_finite_differences(oracle_lib, kind):
    """A point charge at a cell centre (monopole only) and a tight +q/-q pair
    about a cell centre (dipole only): the local expansion's E, J and H at a
    distant cell centre are the exact field's value and its first and second
    derivatives there (central finite differences of Coulomb's law)."""
    G, L = 16, 32.0
    h = 2 * L / G
    s = 3 * G * G + 4 * G + 5
    cs = _cell_centre(s, G, L)
    if kind == "charge":
        src, q = cs[None], np.array([1.7])
    else:
        d = np.array([0.3, -0.2, 0.25]) * 1e-3 * h
        src, q = np.stack([cs + d / 2, cs - d / 2]), np.array([2.0, -2.0])
    m = oracle_lib.ff_moments(src, q, G, L)
    loc = oracle_lib.ff_local(m, G, L, 5)

    def field(pt):
        r = pt[None] - src
        return (q[:, None] * r / np.linalg.norm(r, axis=1)[:, None] ** 3).sum(0)

    for t in (12 * G * G + 9 * G + 13, 3 * G * G + 4 * G + 11, 0, G ** 3 - 1):
        ct = _cell_centre(t, G, L)
        E, J, H = _unpack(loc[t])
        E0, J0, H0 = _fd_derivs(field, ct, 0.005 * h)
        # finite-difference truncation is O((eps / r)^2) ~ 1e-5 of each tensor
        assert np.allclose(E, E0, rtol=0, atol=1e-7 * np.abs(E0).max())
        assert np.allclose(J, J0, rtol=0, atol=1e-4 * np.abs(J0).max())
        assert np.allclose(H, H0, rtol=0, atol=1e-4 * np.abs(H0).max())
    # inside the block: nothing
    assert np.all(loc[s] == 0)


def test_local_expansion_is_harmonic_and_converges(oracle_lib):
    """The far field is divergence- and curl-free at every cell centre
    (J traceless and symmetric by construction, H traces zero), and the
    expansion evaluated at an offset d from the centre of a cell far from a
    single source has error O(|d|^3)."""
    G, L = 12, 30.0
    x = ball(3000, 28.0, 8)
    q = np.where(np.arange(3000) % 2 == 0, 1.0, -0.7)
    m = oracle_lib.ff_moments(x, q, G, L)
    loc = oracle_lib.ff_local(m, G, L, 5)
    occ = np.flatnonzero(np.abs(loc).sum(1))
    for t in occ[::37]:
        E, J, H = _unpack(loc[t])
        scale_j = np.abs(J).max()
        scale_h = np.abs(H).max()
        assert abs(np.trace(J)) <= 1e-12 * scale_j
        for d in range(3):
            assert abs(H[0, 0, d] + H[1, 1, d] + H[2, 2, d]) <= 1e-12 * scale_h
    # Taylor remainder: one source charge, target cell 5 cells away
    G, L = 16, 32.0
    h = 2 * L / G
    s = 8 * G * G + 8 * G + 2
    cs = _cell_centre(s, G, L)
    m = oracle_lib.ff_moments(cs[None], np.array([1.0]), G, L)
    loc = oracle_lib.ff_local(m, G, L, 5)
    t = 8 * G * G + 8 * G + 7
    ct = _cell_centre(t, G, L)
    u = np.array([0.31, -0.22, 0.4])
    errs = []
    for f in (0.4, 0.2, 0.1):
        pt = ct + f * h * u
        approx = oracle_lib.ff_local_eval(pt[None], G, L, loc)[0]
        r = pt - cs
        exact = r / np.linalg.norm(r) ** 3
        errs.append(np.linalg.norm(approx - exact))
    # cubic remainder: halving d divides the error by about 8
    assert 6.0 < errs[0] / errs[1] < 10.0 and 6.0 < errs[1] / errs[2] < 10.0
    assert np.allclose(oracle_lib.ff_local_eval(ct[None], G, L, loc)[0], loc[t, :3], rtol=1e-15)


def test_two_level_expansion(oracle_lib):
    """Two-level grouping: a reach covering the whole parent grid is the
    one-level expansion; a point charge at a parent centre (so the parent's
    monopole is exact and its dipole zero) gives, at targets whose parent is
    beyond the reach, the exact field and its derivatives (finite
    differences of Coulomb's law); and every reach keeps the method's
    accuracy on a droplet (error within a few tens of percent of one level
    for reach >= 2)."""
    G, L = 12, 30.0
    x = ball(2500, 28.0, 9)
    q = np.where(np.arange(2500) % 3 == 0, 1.0, -0.6)
    m = oracle_lib.ff_moments(x, q, G, L)
    one = oracle_lib.ff_local(m, G, L, 5)
    assert np.allclose(oracle_lib.ff_local2(m, G, L, 5, G // 2), one, rtol=1e-11,
                       atol=1e-13 * np.abs(one).max())
    # a point charge at the centre of parent (1, 1, 1): the corner shared by
    # cells 2..3 along each axis
    G, L = 16, 32.0
    h = 2 * L / G
    src = np.array([[-L + 3 * h, -L + 3 * h, -L + 3 * h]])
    m = oracle_lib.ff_moments(src, np.array([1.3]), G, L)
    D = 2
    loc = oracle_lib.ff_local2(m, G, L, 5, D)

    def field(pt):
        r = pt - src[0]
        return 1.3 * r / np.linalg.norm(r) ** 3

    for t in ((12, 9, 13), (14, 2, 3), (9, 15, 15), (2, 13, 1)):
        tx, ty, tz = t
        assert max(abs(tx // 2 - 1), abs(ty // 2 - 1), abs(tz // 2 - 1)) > D
        k = (tz * G + ty) * G + tx
        ct = np.array([-L + (tx + 0.5) * h, -L + (ty + 0.5) * h, -L + (tz + 0.5) * h])
        E, J, H = _unpack(loc[k])
        E0, J0, H0 = _fd_derivs(field, ct, 0.005 * h)
        assert np.allclose(E, E0, rtol=0, atol=1e-9 * np.abs(E0).max())
        assert np.allclose(J, J0, rtol=0, atol=1e-4 * np.abs(J0).max())
        assert np.allclose(H, H0, rtol=0, atol=1e-4 * np.abs(H0).max())
    # accuracy on a droplet against the exact far field
    w = W.config_medium(n=6000, seed=6)
    x = w.pos.astype(np.float64)
    qh = oracle_lib.qhat(w.charge, w.params)
    L = float(np.float32(np.abs(w.pos).max()) * np.float32(1 + 2 ** -10))
    G, B = 16, 5
    rows = np.arange(0, 6000, 7)
    Fn, Ef = oracle_lib.ff_split_block(x, w.type, w.charge, w.params, G, L, B, rows=rows)
    F = Fn + qh[rows, None] * Ef
    m = oracle_lib.ff_moments(x, qh, G, L)
    med = {}
    for D in (0, 2, 3):
        loc = oracle_lib.ff_local(m, G, L, B) if D == 0 else oracle_lib.ff_local2(m, G, L, B, D)
        El = oracle_lib.ff_local_eval(x[rows], G, L, loc)
        rel = np.linalg.norm(qh[rows, None] * (El - Ef), axis=1) / np.linalg.norm(F, axis=1)
        med[D] = np.median(rel)
    assert med[0] < 3e-3 and med[2] < 1.3 * med[0] and med[3] < 1.2 * med[0], med


def test_local_expansion_accuracy_on_a_droplet(oracle_lib):
    """The method's own error: exact block near field plus the local
    expansion of the far cells' monopoles and dipoles reproduces the exact
    Coulomb force within the dipole-truncation bound (median well below
    1e-2 of the force, at a few cells per block half width)."""
    w = W.config_medium(n=6000, seed=6)
    x = w.pos.astype(np.float64)
    qh = oracle_lib.qhat(w.charge, w.params)
    L = float(np.float32(np.abs(w.pos).max()) * np.float32(1 + 2 ** -10))
    G, B = 12, 5
    rows = np.arange(0, 6000, 7)
    Fn, Ef = oracle_lib.ff_split_block(x, w.type, w.charge, w.params, G, L, B, rows=rows)
    m = oracle_lib.ff_moments(x, qh, G, L)
    loc = oracle_lib.ff_local(m, G, L, B)
    El = oracle_lib.ff_local_eval(x[rows], G, L, loc)
    F = Fn + qh[rows, None] * Ef
    rel = np.linalg.norm(qh[rows, None] * (El - Ef), axis=1) / np.linalg.norm(F, axis=1)
    # the centre-only coarse field is far worse: the expansion is doing work
    Ec = oracle_lib.ff_coarse(m, G, L, B)
    cell = np.clip(np.floor((x[rows] + L) / (2 * L / G)).astype(int), 0, G - 1)
    k = (cell[:, 2] * G + cell[:, 1]) * G + cell[:, 0]
    relc = np.linalg.norm(qh[rows, None] * (Ec[k] - Ef), axis=1) / np.linalg.norm(F, axis=1)
    assert np.median(rel) < 3e-3
    assert np.median(relc) > 3 * np.median(rel)


def test_feature_layout(oracle_lib):
    G, L, B = 8, 16.0, 5
    h = 2 * L / G
    x = np.array([[1.3, -2.2, 5.9]])
    m = oracle_lib.ff_moments(x, np.array([0.7]), G, L)
    X = oracle_lib.ff_features(x, G, L, B, m, 0.5)
    assert X.shape == (1, 4 * 125 + 3)
    # the centre cell of the 5^3 block is entry 62 (dz = dy = dx = 0)
    k = np.flatnonzero(m[:, 0])[0]
    assert X[0, 4 * 62] == pytest.approx(0.7 / 0.5)
    assert np.allclose(X[0, 4 * 62 + 1:4 * 62 + 4], m[k, 1:] / (0.5 * h))
    nz = np.flatnonzero(X[0, :500])
    assert set(nz) <= {248, 249, 250, 251}
    cx = (np.floor((x[0] + L) / h) + 0.5) * h - L
    assert np.allclose(X[0, 500:], (x[0] - cx) / h)
    # a particle in the corner cell sees zeros outside the grid
    y = np.array([[-L + 0.1, -L + 0.1, -L + 0.1]])
    Xc = oracle_lib.ff_features(y, G, L, B, oracle_lib.ff_moments(y, np.array([1.0]), G, L),
                                1.0)
    assert Xc[0, 4 * 62] == 1.0 and np.count_nonzero(Xc[0, :500]) <= 4


def random_mlp(K, H, O, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((K, H)) * scale / math.sqrt(K),
            "b1": rng.standard_normal(H) * 0.1,
            "W2": rng.standard_normal((H, H)) * scale / math.sqrt(H),
            "b2": rng.standard_normal(H) * 0.1,
            "W3": rng.standard_normal((H, O)) * scale / math.sqrt(H),
            "b3": rng.standard_normal(O) * 0.1}


def torch_mlp(X, W, bf16=False):
    r = (lambda t: t.float().to(torch.bfloat16).double()) if bf16 else (lambda t: t)
    T = {k: torch.tensor(v, dtype=torch.float64) for k, v in W.items()}
    a = r(torch.tensor(X, dtype=torch.float64))
    z1 = a @ r(T["W1"]) + T["b1"]
    a1 = r(torch.nn.functional.silu(z1))
    z2 = a1 @ r(T["W2"]) + T["b2"]
    a2 = r(torch.nn.functional.silu(z2))
    return (a2 @ r(T["W3"]) + T["b3"]).numpy()


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_forward_matches_torch(oracle_lib, bf16):
    W_ = random_mlp(503, 128, 3, 1)
    X = np.random.default_rng(2).standard_normal((64, 503))
    Y = oracle_lib.mlp_forward(X, W_, bf16_mode=bf16)
    assert np.allclose(Y, torch_mlp(X, W_, bf16), rtol=1e-12, atol=1e-13)


def test_mlp_backward_finite_differences(oracle_lib):
    K, H, O = 11, 7, 3
    W_ = random_mlp(K, H, O, 4, scale=1.0)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((9, K))
    T = rng.standard_normal((9, O))
    loss, g = oracle_lib.mlp_backward(X, T, W_)
    Y = oracle_lib.mlp_forward(X, W_)
    assert loss == pytest.approx(np.mean((Y - T) ** 2), rel=1e-13)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = W_[name].reshape(-1)
        for k in range(0, flat.size, max(1, flat.size // 12)):
            Wp = {kk: v.copy() for kk, v in W_.items()}
            Wm = {kk: v.copy() for kk, v in W_.items()}
            Wp[name].reshape(-1)[k] += eps
            Wm[name].reshape(-1)[k] -= eps
            lp = np.mean((oracle_lib.mlp_forward(X, Wp) - T) ** 2)
            lm = np.mean((oracle_lib.mlp_forward(X, Wm) - T) ** 2)
            assert g[name].reshape(-1)[k] == pytest.approx((lp - lm) / (2 * eps), rel=1e-6,
                                                           abs=1e-9)
    # and agrees with torch autograd
    Tw = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in W_.items()}
    a1 = torch.nn.functional.silu(torch.tensor(X) @ Tw["W1"] + Tw["b1"])
    a2 = torch.nn.functional.silu(a1 @ Tw["W2"] + Tw["b2"])
    L_ = ((a2 @ Tw["W3"] + Tw["b3"] - torch.tensor(T)) ** 2).mean()
    L_.backward()
    for k in Tw:
        assert np.allclose(g[k], Tw[k].grad.numpy(), rtol=1e-11, atol=1e-13)
