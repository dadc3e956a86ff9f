"""Statistical agreement of long runs.  Beyond a few hundred steps the GPU
and oracle trajectories part chaotically, so the medium droplet recipe
(scaled to N = 800: 70/30 charged mix, gravity, rotation, square-law drying
to random close packing at step 2e4, dt = 5e-4) is run 15000 steps -- three
quarters of the way to the dry radius, before the final compression that
this time step cannot follow -- on both sides with the same seeds, and the
macrostates are compared: radius of gyration, mean distance from the
centre, fraction of NPs within one diameter of the wall, and mean contact
number (neighbours closer than 1.1 sigma_ij).  Over the three seeds the
oracle's R_g and mean radius vary by about 0.3 %, its surface fraction by
about 0.015 and its contact number by about 0.02."""
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


def macro(x, typ, sigma, R):
    from scipy.spatial import cKDTree
    com = x.mean(0)
    rg = np.sqrt(((x - com) ** 2).sum(1).mean())
    rad = np.linalg.norm(x, axis=1)
    sig = np.asarray(sigma)[typ]
    surf = np.mean(np.abs(rad - R) < sig)
    pr = cKDTree(x).query_pairs(1.1 * max(sigma), output_type="ndarray")
    d = np.linalg.norm(x[pr[:, 0]] - x[pr[:, 1]], axis=1)
    contacts = (d < 1.1 * 0.5 * (sig[pr[:, 0]] + sig[pr[:, 1]])).sum()
    return rg, rad.mean(), surf, 2.0 * contacts / len(x)


@pytest.mark.parametrize("seed", [2, 12, 22])
def test_medium_drying_macrostate(ld, orc, seed):
    steps = 15000
    w = W.config_medium(n=800, seed=seed)
    print(f"medium drying N={w.n} seed={seed} steps={steps}", flush=True)
    s = ld.System.from_workload(w)
    s.step(steps, w.dt)
    s.sync()
    xg = s.positions64()
    step, t, R = s.state()
    st = orc.State(w)
    assert st.run(steps, w.dt) == -1
    assert step == steps and R == pytest.approx(orc.radius_at(w.radius, st.t), rel=1e-12)
    rg_g, mr_g, sf_g, cn_g = macro(xg, w.type, w.params.sigma, R)
    rg_o, mr_o, sf_o, cn_o = macro(st.x, w.type, w.params.sigma, R)
    assert abs(rg_g - rg_o) <= 0.015 * rg_o, (rg_g, rg_o)
    assert abs(mr_g - mr_o) <= 0.015 * mr_o, (mr_g, mr_o)
    assert abs(sf_g - sf_o) <= 0.06, (sf_g, sf_o)
    assert abs(cn_g - cn_o) <= 0.1, (cn_g, cn_o)
    print(f"seed {seed}: R_g {rg_g:.4f}/{rg_o:.4f} mean r {mr_g:.4f}/{mr_o:.4f} "
          f"surface {sf_g:.4f}/{sf_o:.4f} contacts {cn_g:.3f}/{cn_o:.3f} "
          f"max |dx| {np.abs(xg - st.x).max():.3g}", flush=True)
