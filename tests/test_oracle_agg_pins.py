"""Pins for the oracle's aggregate statistics: the contact-graph components
(the paper's number of sub-aggregates) against scipy's kd-tree pairs and
sparse-graph connected components, and against hand-built chains; N_surf
against constructed shells."""
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
