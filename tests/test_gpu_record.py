"""Trajectory recording through the C ABI: frames every `every` steps hold
exactly the positions (FP32 of hi + lo) an identical context reaches at
those steps, with the device clock's step, t and R(t)."""
import os

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


def reference_frames(ld, w, steps, every, paper=False):
    s = ld.System.from_workload(w)
    if paper:
        s.paper_enable(range_factor=4.0, kick=0.03)
    out = []
    for k in range(every, steps + 1, every):
        s.step(every, w.dt)
        step, t, R = s.state()
        out.append((step, t, R, s.positions64().astype(np.float32)))
    return out


@pytest.mark.parametrize("paper", [False, True])
def test_frames_match_an_identical_run(ld, tmp_path, paper):
    w = W.config_small(n=700, seed=12)
    every, steps = 5, 40
    path = str(tmp_path / "run.trj")
    s = ld.System.from_workload(w)
    if paper:
        s.paper_enable(range_factor=4.0, kick=0.03)
    s.record_open(path, every)
    for chunk in (7, 13, 1, 19):            # frames fall inside chunks
        s.step(chunk, w.dt)
    assert s.record_close() == steps // every
    tr = ld.read_trajectory(path)
    assert tr["n"] == w.n and tr["every"] == every and tr["n_types"] == 1
    assert np.array_equal(tr["type"], w.type)
    ref = reference_frames(ld, w, steps, every, paper)
    assert len(ref) == len(tr["step"])
    for f, (step, t, R, x) in enumerate(ref):
        assert tr["step"][f] == step and tr["t"][f] == t and tr["R"][f] == R
        assert np.array_equal(tr["x"][f], x)


def test_record_errors_and_reopen(ld, tmp_path):
    w = W.config_small(n=200, seed=13)
    s = ld.System.from_workload(w)
    with pytest.raises(RuntimeError):
        s.record_open(str(tmp_path / "a.trj"), 0)
    with pytest.raises(RuntimeError):
        s.record_close()
    s.record_open(str(tmp_path / "a.trj"), 2)
    with pytest.raises(RuntimeError):
        s.record_open(str(tmp_path / "b.trj"), 2)
    s.step(3, w.dt)                          # frame at step 2
    assert s.record_close() == 1
    s.record_open(str(tmp_path / "b.trj"), 2)    # the clock continues at step 3
    s.step(3, w.dt)                          # frames at steps 4, 6
    assert s.record_close() == 2
    tr = ld.read_trajectory(str(tmp_path / "b.trj"))
    assert list(tr["step"]) == [4, 6]
    assert os.path.getsize(str(tmp_path / "b.trj")) == 24 + 4 * w.n + 2 * (24 + 12 * w.n)
