#!/usr/bin/env python3
"""Benchmark: steps/s and pair-interactions/s of the Langevin droplet model at
N = 250000 (three NP types 50/30/20, sigma 1/1.3/2, eps 1/1.5/3, charges
+1/-1/0, sphere of radius 300, linear shrink to 112.5 over 1e4 steps of
dt = 5e-4, gravity 0.05, omega 0.02, kT = 1, all-pairs Coulomb with l_B = 0.7).

One step = the whole hot path: all-pairs LJ + Coulomb forces, external
forces, Brownian noise and the overdamped update (plus the periodic spatial
re-sort), for all N particles, inputs resident on the GPU.

Prints one JSON line.  Extra objects:
  roofline     -- the pair kernel (the dominant one), timed with HIP events on
                  the library's stream during the timed steps; algorithmic
                  FP32 work = 19 flops per ordered pair (Coulomb-only count).
  cpu_baseline -- the FP64 oracle timed on the host on a bounded sample of
                  rows of the same force evaluation, scaled to steps/s.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("steps/s & pair-interactions/s at N=2.5e5; learned vs direct at ≤1e-3 "
          "force err")
FLOPS_PER_PAIR = 19
PEAK_FP32_TFLOPS = 157.3          # published MI355X FP32 vector peak (packed issue)
PEAK_FP32_NONPACKED = 78.6        # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=250000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="large",
                    choices=["large", "ensemble", "small", "learned", "paper", "analysis",
                             "medium"],
                    help="large (default, the headline) / ensemble / small / learned / "
                         "paper (the paper's own truncated-range inertial scheme) / analysis "
                         "(post-processing calls at N=2.5e5)")
    ap.add_argument("--kick", type=float, default=0.05,
                    help="paper: magnitude of the random velocity vector per step")
    ap.add_argument("--record-every", type=int, default=0,
                    help="paper: record every k-th step's positions to a trajectory file "
                         "under $TMPDIR (0: off)")
    ap.add_argument("--snapshots", type=int, default=8,
                    help="learned: training snapshots (N samples each)")
    ap.add_argument("--snap-every", type=int, default=100,
                    help="learned: direct steps between training snapshots")
    ap.add_argument("--epochs", type=int, default=20, help="learned: training epochs")
    ap.add_argument("--near-cut", type=float, default=8.0, help="learned: near cutoff r_c")
    ap.add_argument("--train-from", default="droplets", choices=["droplets", "trajectory"],
                    help="learned: snapshots from independent droplets (each stepped "
                         "snap-every steps) or from one trajectory")
    ap.add_argument("--near-mode", default="block", choices=["block", "radial"],
                    help="learned: exact near part over the 5^3 block of grid cells, or r < r_c")
    ap.add_argument("--parent-reach", type=int, default=None,
                    help="learned, block mode: 0 = one-level expansion (FFT convolution for "
                         "grids up to 32), > 0 = two-level with that reach (default: the "
                         "library's)")
    ap.add_argument("--autotune", action="store_true",
                    help="search the pair kernel launch shape before timing")
    ap.add_argument("--graph", type=int, default=0,
                    help="replay steps from captured HIP graphs (graph_steps)")
    ap.add_argument("--medium-steps", type=int, default=12000,
                    help="medium: steps of the drying to run and time")
    ap.add_argument("--compare", action="store_true",
                    help="ensemble: also time the droplets as separate contexts and one "
                         "droplet with the same sum of N^2")
    ap.add_argument("--comp", type=int, default=None, choices=[0, 1],
                    help="pair sums: 0 = FP32 blocks of 32 terms into FP64 totals, 1 = blocked "
                         "Kahan (default: the library's)")
    ap.add_argument("--block", type=int, default=None, choices=[64, 128, 256, 512],
                    help="pair kernel work-items per workgroup (default: the library's)")
    ap.add_argument("--j-split", type=int, default=None,
                    help="pair kernel j ranges per i tile (default: the library's)")
    ap.add_argument("--cull", type=int, default=None, choices=[0, 1],
                    help="pair kernel group-pair culling: 0 = every pair of groups takes the "
                         "near loop (default: the library's)")
    ap.add_argument("--sort-every", type=int, default=None,
                    help="steps between spatial re-sorts (< 0: never; default: the library's)")
    ap.add_argument("--no-windows", action="store_true",
                    help="large: skip the middle and late 500-step windows (steps 4750 and "
                         "9500 of the 1e4-step run)")
    ap.add_argument("--no-learned", action="store_true",
                    help="large: skip the learned-vs-direct comparison")
    ap.add_argument("--learned-steps", type=int, default=100,
                    help="large: steps timed per path in the learned-vs-direct comparison")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of MIB MiB (counter calibration)")
    return ap.parse_args()


def log(msg: str) -> None:
    """Progress on stderr (stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pair_source_digest() -> str:
    """SHA-256 over the pair kernel's sources (kernel file + inner loops)."""
    h = hashlib.sha256()
    for f in ("ld_pair.hip", "ld_pair_core.h"):
        h.update(open(os.path.join(ROOT, "paper_2501_04456_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic_for(kernel: str, n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
        digest = pair_source_digest()
        if rec and rec.get("source_sha256") == digest and rec.get("n") == n:
            return rec.get("bytes_per_launch")
    except Exception:
        return None
    return None


def cpu_baseline(w, target_s: float):
    import numpy as np
    import oracle
    oracle.lib()
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    rng = np.random.default_rng(123)
    # calibrate on enough rows to keep every thread busy, then size the sample
    # to about target_s seconds (one more try if it came out far too short)
    m = max(32, 16 * threads)
    el = 0.0
    for _ in range(3):
        rows = rng.choice(w.n, m, replace=False)
        t0 = time.perf_counter()
        oracle.pair_forces(w.pos, w.type, w.charge, w.params, rows=rows)
        el = time.perf_counter() - t0
        if el >= 0.5 * target_s or m >= w.n:
            break
        m = int(min(w.n, max(m + 1, m * target_s / max(el, 1e-3))))
    step_s = el * w.n / m                 # pair sum dominates the step
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": 1.0 / step_s,
        "unit": "steps/s",
        "pair_interactions_per_s": m * (w.n - 1) / el,
        "cores": threads,
        "cores_visible": cores,
        "cpu_model": cpu,
        "kind": "oracle",
        "sample": f"pair forces of {m} random rows x all {w.n} particles "
                  f"({el:.1f} s), scaled by N/rows to one step",
    }


def bench_paper(a, torch, ldrop, W):
    """The paper's own scheme (section 2.2 steps (i)-(vi) read literally) on
    the headline droplet: pairs truncated at 4 (r_i + r_j) over a cell list,
    Newton + Stokes drag, fixed-magnitude random velocity kick, spring acting
    within one radius of the surface."""
    w = W.config_large(n=a.n)
    p = w.params
    p.wall_band = 1
    p.wall_offset = [0.5 * sg for sg in p.sigma]
    s = ldrop.System.from_workload(w)
    s.paper_enable(range_factor=4.0, kick=a.kick, inertial_mass=p.mass)
    s.step(a.warmup, w.dt)
    s.sync()
    trj = None
    if a.record_every > 0:
        import tempfile
        trj = os.path.join(tempfile.gettempdir(), f"ld_bench_{os.getpid()}.trj")
        s.record_open(trj, a.record_every)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    s.step(a.steps, w.dt)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync()
    ms = ev0.elapsed_time(ev1)
    rec = None
    if trj:
        frames = s.record_close()
        rec = {"every": a.record_every, "frames": frames, "bytes": os.path.getsize(trj),
               "wall_s_incl_writer": time.perf_counter() - t0}
        os.remove(trj)
    print(json.dumps({
        "metric": "paper scheme steps/s at N=2.5e5 (truncated range, inertial)",
        "recording": rec,
        "value": a.steps * 1e3 / ms, "unit": "steps/s",
        "particle_steps_per_s": w.n * a.steps * 1e3 / ms,
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
        "wall_s": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 pair math and velocities", "data": "synthetic",
        "config": {"workload": "paper: N=250000 three-type droplet, LJ + Coulomb truncated at "
                               "4 (r_i + r_j), band spring, Newton + Stokes drag, velocity kick",
                   "n": w.n, "dt": w.dt, "kick": a.kick, "range_factor": 4.0},
    }), flush=True)


def bench_analysis(a, torch, ldrop, W):
    """Post-processing at N = 250000: RDF + C-bar (Eqs. 6, 8), box-counting
    and radius-of-gyration fractal dimensions (Eqs. 2-4), sub-aggregates
    (contact-graph components) and N_surf, on the headline droplet as
    initialised (dispersed) and on a packed one (a jittered cubic lattice of
    spacing 1.02 sigma: one giant component); the surface fractal dimension
    on a droplet with 50000 NPs in surface patches."""
    import numpy as np

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, r

    w = W.config_large(n=a.n)
    s = ldrop.System.from_workload(w)
    out = {}
    out["rdf_ms"], _ = timed(lambda: s.rdf(10.0, 200))
    out["fractal_ms"], _ = timed(lambda: s.fractal())
    out["aggregates_dispersed_ms"], g = timed(lambda: s.aggregates(1.1))
    out["aggregates_dispersed"] = g
    out["surface_count_ms"], _ = timed(lambda: s.surface_count())
    k = int(round(a.n ** (1.0 / 3.0))) + 1
    rng = np.random.default_rng(7)
    grid = np.stack(np.meshgrid(*[np.arange(k)] * 3, indexing="ij"), -1).reshape(-1, 3)[:a.n]
    xp = (grid - k / 2) * 1.02 + rng.uniform(-0.01, 0.01, grid.shape)
    wp = W.Workload("packed", a.n, np.zeros(a.n, np.int32), np.zeros(a.n),
                    xp.astype(np.float32), W.config_small().params, w.radius, w.dt, 1, 1)
    sp = ldrop.System.from_workload(wp)
    out["aggregates_packed_ms"], g = timed(lambda: sp.aggregates(1.1))
    out["aggregates_packed"] = g
    # a droplet with a fifth of its NPs in 400 patches on the surface
    pm = W.config_medium(n=a.n, with_positions=False).params
    xs, ts = W.surface_clusters(a.n // 5, a.n - a.n // 5, 300.0, pm.sigma, 31, n_centres=400,
                                spread=4.0)
    ws = W.Workload("surface", a.n, ts, np.zeros(a.n), xs.astype(np.float32), pm,
                    W.Radius(kind=W.RADIUS_CONST, R0=300.0), w.dt, 1, 1)
    ss = ldrop.System.from_workload(ws)
    out["surface_fractal_ms"], g = timed(lambda: ss.surface_fractal(-1.0, 1.1))
    out["surface_fractal"] = g
    print(json.dumps({
        "metric": "post-processing call times at N=2.5e5", "value": out["aggregates_dispersed_ms"],
        "unit": "ms (sub-aggregates, dispersed droplet)", "higher_is_better": False,
        "n_gpus": 1, "data": "synthetic", "config": {"workload": "analysis", "n": a.n},
        "times": out}), flush=True)


def bench_medium(a, torch, ldrop, W):
    """The medium droplet (N = 32768, 70/30 charged mix, gravity, rotation,
    square-law drying from R0 = 120): the drying from its start over
    --medium-steps steps (default 12000, 60 % of the way to the dry radius;
    at dt = 5e-4 the compression towards random close packing makes LJ
    contacts too stiff for the step -- the first too-large move comes at
    step 13501), timed whole, with the RDF (r_max 10 sigma, 200 bins) and
    both fractal dimensions of the end state."""
    import numpy as np
    w = W.config_medium()
    s = ldrop.System.from_workload(w)
    steps = a.medium_steps
    flagged = []
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    s.step(steps, w.dt)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    try:
        s.sync()
    except ldrop.NonFinite as err:
        flagged.append(str(err))
    t0 = time.perf_counter()
    _, _, g, cbar = s.rdf(10.0, 200)
    rg, df, dbox, K, _ = s.fractal()
    post_ms = (time.perf_counter() - t0) * 1e3
    step, t, R = s.state()
    r = (np.arange(200) + 0.5) * 0.05
    sps = steps / (ms / 1e3)
    pairs = float(w.n) * (w.n - 1)
    print(json.dumps({
        "metric": "medium droplet drying: steps/s & pair-interactions/s",
        "value": sps, "unit": "steps/s", "pair_interactions_per_s": pairs * sps,
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": ms / steps,
        "higher_is_better": True, "dtype": "f32 pair math, f64 totals", "data": "synthetic",
        "config": {"workload": "medium: N=32768 70/30 droplet, square-law drying, dt=5e-4",
                   "n": w.n, "dt": w.dt, "jump_flags": flagged},
        "end_state": {"step": step, "t": t, "R": R, "R_g": rg, "D_f": df, "D_box": dbox,
                      "box_scales": K, "rdf_first_peak_r": float(r[int(np.argmax(g[:40]))]),
                      "rdf_first_peak_g": float(np.max(g[:40])), "post_ms": post_ms},
    }), flush=True)


def bench_ensemble(a, torch, ldrop, W):
    """256 independent droplets in one persistent launch per step."""
    e = W.config_ensemble()
    ens = ldrop.Ensemble(e.droplets)
    if a.graph or a.comp is not None:
        ens.set_tuning(graph_steps=a.graph, comp=a.comp or 0)
    t_tune = time.perf_counter()
    tuned = ens.autotune()                 # workgroups and unroll, timed on this ensemble
    tune_s = time.perf_counter() - t_tune
    # warm-up covers at least one captured chunk, so capture and instantiation
    # stay outside the timed region
    ens.step(max(a.warmup, 2 * a.graph), e.dt)
    flagged = []

    def sync():
        # at dt = 1e-3 an LJ contact can move a particle more than jump_max in
        # one step; that is reported, not fatal, for the timing run
        try:
            ens.sync()
        except ldrop.NonFinite as err:
            flagged.append(str(err))

    sync()
    pairs = float(sum(d.n * (d.n - 1) for d in e.droplets))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    ens.step(a.steps, e.dt)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    ens.kernel_timing(True)
    ens.step(a.steps, e.dt)
    launches, pair_ms = ens.kernel_time()
    ens.kernel_timing(False)
    sync()
    avg = pair_ms / max(launches, 1)
    achieved = FLOPS_PER_PAIR * pairs / (avg / 1e3) / 1e12
    sps = a.steps / (ms / 1e3)
    compare = None
    if a.compare:
        def timed_ms(fn):
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            fn()
            t1.record()
            torch.cuda.synchronize()
            return t0.elapsed_time(t1)

        # the same droplets as separate contexts, one after another per step
        systems = [ldrop.System.from_workload(d) for d in e.droplets]

        def naive():
            for _ in range(a.steps):
                for sy in systems:
                    sy.step(1, e.dt)

        for sy in systems:
            sy.step(1, e.dt)
        naive_ms = timed_ms(naive)
        for sy in systems:
            sy.close()
        # one droplet of the same composition recipe with N^2 = sum N_d^2
        n1 = int(round(pairs ** 0.5))
        d1 = W.config_ensemble(n_drop=1, n_min=n1, n_max=n1, seed=4).droplets[0]
        s1 = ldrop.System.from_workload(d1)
        s1.step(max(a.warmup, 1), e.dt)
        one_ms = timed_ms(lambda: s1.step(a.steps, e.dt))
        p1 = float(d1.n) * (d1.n - 1)
        compare = {
            "naive_per_droplet_steps_per_s": a.steps / (naive_ms / 1e3),
            "persistent_over_naive": naive_ms / ms,
            "single_droplet": {"n": d1.n, "steps_per_s": a.steps / (one_ms / 1e3),
                               "pair_interactions_per_s": p1 * a.steps / (one_ms / 1e3)},
            "efficiency_vs_single_droplet": (pairs * sps) / (p1 * a.steps / (one_ms / 1e3)),
        }
    print(json.dumps({
        "metric": "ensemble steps/s & pair-interactions/s",
        "value": sps, "unit": "steps/s", "pair_interactions_per_s": pairs * sps,
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 pair math, f64 totals", "data": "synthetic",
        "config": {"workload": "ensemble: 256 droplets, N log-uniform in [500, 8000]",
                   "total_particles": int(sum(d.n for d in e.droplets)),
                   "sum_N2": pairs, "graph_steps": a.graph, "tuning": tuned,
                   "autotune_s": tune_s, "jump_flags": flagged},
        "roofline": {"kernel": "k_ens_pair (persistent)", "bound": "alu",
                     "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "frac_of_nonpacked_fp32": achieved / PEAK_FP32_NONPACKED,
                     "traffic": None, "avg_launch_ms": avg, "launches": launches},
        "compare": compare,
    }), flush=True)


def learned_run(a, torch, ldrop, W, steps=None):
    """Learned far field vs direct summation at N = 250000 (medium
    composition): train on snapshots of training-seed droplets, then time
    both paths on an evaluation-seed system and judge the learned forces.
    Returns the result as a dict (the gain test: median error of the near
    part alone, of near + coarse expansion, and of near + coarse + MLP)."""
    steps = a.steps if steps is None else steps
    import numpy as np

    def timed(sys_, steps, dt):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        sys_.step(steps, dt)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    t0 = time.perf_counter()
    wt = W.config_learned(n=a.n, seed=105)
    tr = ldrop.System.from_workload(wt)
    mode = ldrop.NEAR_BLOCK if a.near_mode == "block" else ldrop.NEAR_RADIAL
    ffkw = dict(near_cut=a.near_cut, near_mode=mode)
    if a.parent_reach is not None:
        ffkw["parent_reach"] = a.parent_reach
    reach = ffkw.get("parent_reach", ldrop.FF_DEFAULT["parent_reach"])
    tr.ff_enable(**ffkw)
    if a.train_from == "trajectory":
        tr.ff_collect(reset=True, max_snapshots=a.snapshots)
        for _ in range(a.snapshots - 1):
            tr.step(a.snap_every, wt.dt)
            tr.ff_collect()
    else:
        # independent droplets of the same composition (seeds 105, 106, ...),
        # each stepped snap_every steps from its own random start
        for k in range(a.snapshots):
            tr.set_positions(W.config_learned(n=a.n, seed=105 + k).pos)
            tr.step(a.snap_every, wt.dt)
            tr.ff_collect(reset=(k == 0), max_snapshots=a.snapshots)
            log(f"learned: snapshot {k + 1}/{a.snapshots}")
    collect_s = time.perf_counter() - t0
    log(f"learned: {a.snapshots} snapshots collected in {collect_s:.1f} s, training")
    t1 = time.perf_counter()
    rep = tr.ff_train(epochs=a.epochs, batch=8192, lr=1e-3, seed=105, val_fraction=0.1)
    train_s = time.perf_counter() - t1
    log(f"learned: trained in {train_s:.1f} s")
    weights, sq, scale = tr.ff_weights()      # scale includes the held-out gain
    del tr
    we = W.config_learned(n=a.n, seed=5)
    ev = ldrop.System.from_workload(we)
    ev.ff_enable(**ffkw)
    ev.ff_set_weights(weights, sq, scale)
    ev.step(a.warmup, we.dt)
    ms_direct = timed(ev, steps, we.dt)
    err = ev.ff_judge()
    ev.ff_mode(1)
    ev.step(2, we.dt)
    ev.kernel_timing(True)
    ms_learned = timed(ev, steps, we.dt)
    near_launches, near_ms = ev.near_kernel_time()
    ev.kernel_timing(False)
    near_pairs = near_block_pairs(ev.positions64(), G=32, B=5) if a.near_mode == "block" else None
    # the method without the network (near + coarse only)
    K = 4 * 5 ** 3 + 3
    o = (K + 31) // 32 * 32 * 128 + 128 + 128 * 128 + 128
    nonet = weights.copy()
    nonet[o:] = 0.0
    ev.ff_set_weights(nonet, sq, scale)
    err_nonet = ev.ff_judge()
    ev.ff_set_weights(weights, sq, scale)
    # the near part alone (Coulomb truncated at the block): its error is the
    # exact far force relative to the exact total
    Fn = ev.ff_forces(0)
    Ff = ev.ff_forces(4)
    tot = np.linalg.norm(Fn + Ff, axis=1)
    err_near = float(np.median(np.linalg.norm(Ff, axis=1) / np.maximum(tot, 1e-300)))
    judge_stats = ev.ff_stats()
    pairs = float(we.n) * (we.n - 1)
    # matrix-core work of training: per sample, forward 2 (Kp H + H H + H Op)
    # flops, the weight gradients as much again, and the input gradients of
    # layers 2 and 3 2 (H H + H Op) (layer 1's inputs need none)
    K = 4 * 5 ** 3 + 3
    Kp, H, Op = (K + 31) // 32 * 32, 128, 16
    train_flops = 2.0 * (2 * (Kp * H + H * H + H * Op) + H * H + H * Op) * 8192 * rep["iterations"]
    return {
        "metric": "learned vs direct steps/s at N=2.5e5 and median force error",
        "value": 1e3 / ms_learned, "unit": "steps/s",
        "direct_steps_per_s": 1e3 / ms_direct, "speedup": ms_direct / ms_learned,
        "median_rel_force_err": err, "median_rel_force_err_without_mlp": err_nonet,
        "median_rel_force_err_near_only": err_near,
        "mlp_gain": {"near_only": err_near, "near_plus_coarse": err_nonet,
                     "near_plus_coarse_plus_mlp": err,
                     "mlp_lowers_error_by": (err_nonet - err) / err_nonet if err_nonet else None,
                     "fitted_output_gain": rep.get("gain")},
        "judge": judge_stats,
        "judge_tol": 1e-3, "n_gpus": 1, "steps": steps, "warmup": a.warmup,
        "higher_is_better": True, "dtype": "f32 pair math, bf16 MLP, f64 totals",
        "data": "synthetic",
        "config": {"workload": "learned: N=250000 medium composition, 32^3 moments, 5^3 block, "
                               "MLP 503-128-128-3",
                   "near_mode": a.near_mode,
                   "parent_reach": reach if a.near_mode == "block" else None,
                   "near_cut": a.near_cut if a.near_mode == "radial" else None,
                   "snapshots": a.snapshots,
                   "snap_every": a.snap_every, "epochs": a.epochs,
                   "train_from": a.train_from},
        "training": {**rep, "collect_s": collect_s, "train_s": train_s,
                     "mfma_flops": train_flops,
                     "mfma_tflops_per_s": train_flops / train_s / 1e12 if train_s else None,
                     "frac_of_bf16_peak": (train_flops / train_s / 1e12 / 2500.0
                                           if train_s else None)},
        "direct_pair_interactions_per_s": pairs * 1e3 / ms_direct,
        "near_roofline": near_roofline(near_pairs, near_launches, near_ms),
    }


def near_block_pairs(pos, G, B):
    """Ordered pairs the block near field evaluates: every particle with
    every other particle of the B^3 block of grid cells around its own cell
    (cells of side 2L/G, L = 1.0009765625 max |coordinate|, clipped at the
    grid's faces).  Host-side bookkeeping for the flop count only."""
    import numpy as np
    L = float(np.float32(np.abs(pos).max()) * np.float32(1.0009765625))
    h = 2.0 * L / G
    c = np.clip(np.floor((pos + L) / h).astype(np.int64), 0, G - 1)
    cnt = np.zeros((G, G, G), np.int64)
    np.add.at(cnt, (c[:, 2], c[:, 1], c[:, 0]), 1)
    half = B // 2
    box = cnt.copy()
    for ax in range(3):             # sum over the window [-half, half] per axis
        p = np.pad(box, [(half, half) if k == ax else (0, 0) for k in range(3)])
        cs = np.cumsum(p, axis=ax)
        cs = np.concatenate([np.zeros_like(np.take(cs, [0], axis=ax)), cs], axis=ax)
        hi = np.take(cs, np.arange(B, G + B), axis=ax)
        lo = np.take(cs, np.arange(0, G), axis=ax)
        box = hi - lo
    return int((cnt * box).sum() - len(pos))


def near_roofline(pairs, launches, ms):
    """Roofline object of the learned path's near-field pair kernels: 19
    FP32 flops per evaluated ordered pair (the Coulomb term; the few LJ
    pairs are extra) over their HIP-event duration."""
    if not pairs or not launches or ms <= 0:
        return None
    avg = ms / launches
    achieved = 19.0 * pairs / (avg * 1e-3) / 1e12
    return {"kernel": "k_near_block", "bound": "alu", "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "pairs_per_launch": pairs, "avg_launch_ms": avg, "launches": launches,
            "traffic": None}


def bench_learned(a, torch, ldrop, W):
    print(json.dumps(learned_run(a, torch, ldrop, W)), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "ldrop runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2501_04456_amd import ldrop
    from paper_2501_04456_amd import workloads as W

    if not os.path.exists(ldrop.LIB_PATH):
        from paper_2501_04456_amd import build as hipbuild
        hipbuild.build()
    torch.cuda.set_device(0)
    if a.copy_calibration > 0:
        # a plain copy of known size: what the HBM byte counters read for it
        # scales the pair kernel's counter readings
        nbytes = a.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy calibration: {nbytes} bytes read, {nbytes} bytes written", flush=True)
        del src, dst
    if a.workload == "ensemble":
        return bench_ensemble(a, torch, ldrop, W)
    if a.workload == "learned":
        return bench_learned(a, torch, ldrop, W)
    if a.workload == "paper":
        return bench_paper(a, torch, ldrop, W)
    if a.workload == "medium":
        return bench_medium(a, torch, ldrop, W)
    if a.workload == "analysis":
        return bench_analysis(a, torch, ldrop, W)
    w = W.config_large(n=a.n) if a.workload == "large" else W.config_small()
    s = ldrop.System.from_workload(w)
    if a.autotune:
        s.autotune()
    if a.graph:
        s.set_tuning(graph_steps=a.graph)
    for key in ("comp", "block", "j_split", "cull", "sort_every"):
        if getattr(a, key) is not None:
            s.set_tuning(**{key: getattr(a, key)})
    tune = s.tuning()
    flagged = []

    def sync():
        # an LJ contact can move a particle more than jump_max in one step at
        # the small workload's dt; that is reported, not fatal, for timing
        try:
            s.sync()
        except ldrop.NonFinite as err:
            flagged.append(str(err))

    log(f"{a.workload}: n={w.n} tuning={tune}, warmup")
    s.step(max(a.warmup, 2 * a.graph), w.dt)
    sync()
    torch.cuda.synchronize()
    log(f"timing {a.steps} steps")
    s.kernel_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    s.step(a.steps, w.dt)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    launches, pair_ms = s.kernel_time()
    s.kernel_timing(False)
    sync()
    steps_per_s = a.steps / (ms / 1e3)
    pairs = float(w.n) * (w.n - 1)
    avg_pair_ms = pair_ms / max(launches, 1)
    # Algorithmic work: the Coulomb sum over pairs of charged particles (a
    # pair with an uncharged partner has an identically zero Coulomb term
    # and far from contact no force at all; the kernel skips those groups).
    n_charged = int((w.charge != 0).sum())
    eval_pairs = float(n_charged) * (n_charged - 1)
    flops_launch = FLOPS_PER_PAIR * eval_pairs
    achieved = flops_launch / (avg_pair_ms / 1e3) / 1e12
    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "steps/s",
        "pair_interactions_per_s": pairs * steps_per_s,
        "charged_pair_interactions_per_s": eval_pairs * steps_per_s,
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms / a.steps,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pair math, f64 totals",
        "data": "synthetic",
        "config": {"workload": ("large: N=250000 three-type droplet, all-pairs LJ+Coulomb, "
                                "full external forces, overdamped Langevin, dt=5e-4")
                   if a.workload == "large" else
                   "small: N=1000 one-type droplet, wall shrinking 40->15, dt=1e-3",
                   "n": w.n, "dt": w.dt, "tuning": tune, "jump_flags": flagged},
        "roofline": {
            "kernel": "k_pair (all-pairs forces)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS,
            "frac_of_nonpacked_fp32": achieved / PEAK_FP32_NONPACKED,
            "traffic": traffic_for("k_pair", w.n),
            "flops_per_launch": flops_launch,
            "charged_pairs_per_launch": eval_pairs,
            "avg_launch_ms": avg_pair_ms,
            "launches": launches,
            # the all-ordered-pairs count: 19 FLOPs x N(N-1) per launch (pairs
            # with an uncharged particle have no Coulomb term and are skipped)
            "frac_all_ordered_pairs": (19.0 * pairs / (avg_pair_ms * 1e-3) / 1e12
                                       / PEAK_FP32_TFLOPS) if avg_pair_ms else None,
        },
    }
    if a.graph:
        # the per-launch timing above ran without graphs (events need the
        # eager path); time the graph replay itself for steps/s
        s.set_tuning(graph_steps=a.graph)
        s.step(2 * a.graph, w.dt)         # capture outside the timed region
        sync()
        torch.cuda.synchronize()
        ev0.record()
        s.step(a.steps, w.dt)
        ev1.record()
        torch.cuda.synchronize()
        ms_g = ev0.elapsed_time(ev1)
        out["value"] = a.steps / (ms_g / 1e3)
        out["pair_interactions_per_s"] = pairs * out["value"]
        out["ms_per_step"] = ms_g / a.steps
        out["ms_per_step_eager"] = ms / a.steps
    if a.workload == "large" and not a.no_windows:
        # the same run carried on to the middle and the end of its 1e4 steps
        # (the wall moves 300 -> 112.5 sigma and packs the NPs towards the
        # surface): 500-step windows timed like the first one
        def window(start, length=500):
            step_now = s.state()[0]
            # advance in chunks so that progress shows
            while start > step_now:
                k = min(1000, start - step_now)
                s.step(k, w.dt)
                sync()
                step_now += k
                log(f"at step {step_now}")
            sync()
            torch.cuda.synchronize()
            s.kernel_timing(True)
            ev0.record()
            s.step(length, w.dt)
            ev1.record()
            torch.cuda.synchronize()
            wms = ev0.elapsed_time(ev1)
            nl, pms = s.kernel_time()
            s.kernel_timing(False)
            nflag = len(flagged)
            sync()
            st_, t_, R_ = s.state()
            apm = pms / max(nl, 1)
            return {"steps": [int(st_ - length), int(st_)], "R_end": R_,
                    "steps_per_s": length / (wms / 1e3),
                    "pair_interactions_per_s": pairs * length / (wms / 1e3),
                    "avg_pair_launch_ms": apm,
                    "frac": flops_launch / (apm / 1e3) / 1e12 / PEAK_FP32_TFLOPS,
                    "jump_flags": flagged[nflag:]}

        first = {"steps": [int(max(a.warmup, 2 * a.graph)),
                           int(max(a.warmup, 2 * a.graph) + a.steps)],
                 "steps_per_s": out["value"], "avg_pair_launch_ms": avg_pair_ms,
                 "frac": out["roofline"]["frac"]}
        mid = window(4750)
        log(f"middle window: {mid['steps_per_s']:.1f} steps/s")
        late = window(9500)
        log(f"late window: {late['steps_per_s']:.1f} steps/s")
        out["windows"] = {"first": first, "middle": mid, "late": late}
        out["late"] = late
    # informative: the whole state handed back to the host (ld_get_positions,
    # hi and lo FP32 words of every coordinate) after a step, and the step
    # rate if every step did that; `value` keeps the inputs resident
    import numpy as np
    hp = np.empty((w.n, 3), np.float32)
    lp = np.empty((w.n, 3), np.float32)
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        s.positions_into(hp, lp)
    rb_ms = (time.perf_counter() - t0) * 1e3 / reps
    out["positions_to_host_ms"] = rb_ms
    out["steps_per_s_with_positions_to_host"] = 1e3 / (out["ms_per_step"] + rb_ms)
    if not a.no_cpu_baseline and a.workload == "large":
        log("cpu baseline (oracle on the host)")
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
    if a.workload == "large" and not a.no_learned:
        # the metric's second half: learned far field vs direct summation at
        # N = 250000 (its own droplet, the medium composition), with the gain
        # test of the trained network
        s.close()
        del s
        torch.cuda.empty_cache()
        log("learned far field vs direct")
        r = learned_run(a, torch, ldrop, W, steps=a.learned_steps)
        out["learned_vs_direct"] = {
            k: r[k] for k in ("value", "direct_steps_per_s", "speedup", "median_rel_force_err",
                              "mlp_gain", "judge", "judge_tol", "steps", "config",
                              "near_roofline")}
        out["learned_vs_direct"]["unit"] = "steps/s"
        out["learned_vs_direct"]["note"] = (
            "timed path: exact near part over the 5^3 block of grid cells + the FFT local "
            "expansion of the far cells' monopoles and dipoles + the MLP; on held-out "
            "droplets the network's residual target (the far cells' quadrupole and higher "
            "content, which its block-moment inputs do not carry) is not learnable, so "
            "the calibrated network contributes about nothing (see mlp_gain)")
        out["learned_vs_direct"]["training"] = {
            k: r["training"].get(k) for k in ("samples", "iterations", "val_rel_rms",
                                             "val_rel_rms_raw", "gain", "collect_s",
                                             "train_s", "mfma_tflops_per_s",
                                             "frac_of_bf16_peak")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
