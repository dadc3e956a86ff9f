"""Write the expected values of the large droplet's first 20 steps.

The large workload (N = 250000, three types 50/30/20, sigma 1/1.3/2, eps
1/1.5/3, charges +1/-1/0, R0 = 300, the full external forces, overdamped
Langevin with dt = 5e-4, Philox seed 3) is stepped 20 times by the CPU FP64
oracle alone.  For a fixed sample of rows the file keeps, at every step
k = 0 .. 19 (before the k-th update), the oracle's pair force on the row and
its conditioning scale S_i = sum_j |f_ij|, a flag for rows that have an LJ
pair within 1e-5 (relative) of its cutoff at that state, a stiffness bound
D_i (how fast the row's pair force can change when the row or a partner
moves: sum over partners of |df/dr| + |f|/r, Lennard-Jones within the cutoff
plus Coulomb over all pairs), and the rows' positions before every step
and after step 20.  D_i lets a test compare forces taken at two states that
differ by a small distance delta: |F(x) - F(x')| <= 2 delta D_i.

Rows: 160 drawn at random, the 64 rows whose nearest neighbour is closest
relative to the pair's contact distance (the stiffest LJ pairs of the
initial state), and the first and last particle.

Only the oracle and the seeded workload generator are called.  On eight
host cores the run takes about half an hour.

Usage: python tests/golden/make_large_first20.py [out.npz]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_04456_amd import workloads as W  # noqa: E402

STEPS = 20
OUT = os.path.join(HERE, "large_first20.npz")


def pos_digest(pos) -> str:
    return hashlib.sha256(np.ascontiguousarray(pos, np.float32).tobytes()).hexdigest()


def pick_rows(w) -> np.ndarray:
    from scipy.spatial import cKDTree
    x = w.pos.astype(np.float64)
    sig = np.asarray(w.params.sigma)[w.type]
    d, j = cKDTree(x).query(x, k=2)
    ratio = d[:, 1] / (0.5 * (sig + sig[j[:, 1]]))
    stiff = np.argsort(ratio, kind="stable")[:64]
    rnd = np.random.default_rng(2025).choice(w.n, 160, replace=False)
    return np.unique(np.concatenate([rnd, stiff, [0, w.n - 1]])).astype(np.int64)


def near_cutoff(w, x, rows, rel=1e-5) -> np.ndarray:
    """Rows with an LJ pair within `rel` of its cutoff at positions x."""
    from scipy.spatial import cKDTree
    sig = np.asarray(w.params.sigma)[w.type]
    reach = w.params.lj_cut * max(w.params.sigma) * (1 + 2 * rel)
    tree = cKDTree(x)
    out = np.zeros(len(rows), bool)
    for k, i in enumerate(rows):
        for j in tree.query_ball_point(x[i], reach):
            if j == i:
                continue
            rc = w.params.lj_cut * 0.5 * (sig[i] + sig[j])
            if abs(np.linalg.norm(x[i] - x[j]) - rc) <= rel * rc:
                out[k] = True
    return out


def stiffness(w, x, rows) -> np.ndarray:
    """D_i = sum_j |f'(r_ij)| + |f(r_ij)| / r_ij over the row's pairs (the
    Lennard-Jones law within its cutoff, Coulomb for all pairs): a bound on
    the change of the pair force per unit relative displacement."""
    p = w.params
    sig = np.asarray(p.sigma)[w.type]
    eps = np.asarray(p.eps)[w.type]
    qh = np.asarray(w.charge) * np.sqrt(p.kT * p.bjerrum)
    out = np.zeros(len(rows))
    for k, i in enumerate(rows):
        r = np.linalg.norm(x - x[i], axis=1)
        r[i] = np.inf
        s_ij = 0.5 * (sig[i] + sig)
        lj = r < p.lj_cut * s_ij
        rl = r[lj]
        s6 = (s_ij[lj] / rl) ** 6
        e = 24.0 * np.sqrt(eps[i] * eps[lj])
        f = e * (2.0 * s6 * s6 - s6) / rl
        fp = e * (-26.0 * s6 * s6 + 7.0 * s6) / (rl * rl)
        out[k] = np.sum(np.abs(fp) + np.abs(f) / rl) + np.sum(3.0 * np.abs(qh[i] * qh) / r ** 3)
    return out


def main(out_path: str = OUT) -> None:
    oracle.build()
    w = W.config_large()
    rows = pick_rows(w)
    st = oracle.State(w)
    m = len(rows)
    F = np.zeros((STEPS, m, 3))
    S = np.zeros((STEPS, m))
    amb = np.zeros((STEPS, m), bool)
    D = np.zeros((STEPS, m))
    X = np.zeros((STEPS + 1, m, 3))
    t0 = time.time()
    for k in range(STEPS):
        X[k] = st.x[rows]
        F[k], S[k], _ = oracle.pair_forces(st.x, w.type, w.charge, w.params, rows=rows)
        amb[k] = near_cutoff(w, st.x, rows)
        D[k] = stiffness(w, st.x, rows)
        bad = st.run(1, w.dt)
        if bad != -1:
            raise SystemExit(f"the oracle flagged step {bad}")
        print(f"step {k + 1}/{STEPS} done ({time.time() - t0:.0f} s)", flush=True)
    X[STEPS] = st.x[rows]
    np.savez_compressed(out_path, rows=rows, F=F, S=S, near_cutoff=amb, D=D, x=X,
                        x20=st.x[rows],
                        n=np.int64(w.n), seed=np.int64(w.seed), dt=np.float64(w.dt),
                        steps=np.int64(STEPS), pos_sha256=np.array(pos_digest(w.pos)))
    print("wrote", out_path)


if __name__ == "__main__":
    main(*sys.argv[1:])
