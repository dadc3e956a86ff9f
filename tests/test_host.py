"""Host-side logic that needs no GPU: the trajectory file reader against a
file written here in the documented frame format, and the marshalling of
radius schedules into the C structure."""
import struct

import numpy as np
import pytest

from paper_2501_04456_amd import ldrop
from paper_2501_04456_amd import workloads as W


def test_read_trajectory_format(tmp_path):
    n, every = 5, 20
    typ = np.array([0, 1, 1, 0, 2], np.int32)
    rng = np.random.default_rng(0)
    frames = [(20, 0.02, 39.5, rng.normal(size=(n, 3)).astype(np.float32)),
              (40, 0.04, 39.0, rng.normal(size=(n, 3)).astype(np.float32))]
    p = tmp_path / "t.ldtraj"
    with open(p, "wb") as f:
        f.write(b"LDTRAJ01" + struct.pack("<qii", n, 3, every) + typ.tobytes())
        for step, t, R, x in frames:
            f.write(struct.pack("<qdd", step, t, R) + x.tobytes())
        f.write(b"\x00" * 7)            # a frame cut short is ignored
    d = ldrop.read_trajectory(str(p))
    assert (d["n"], d["n_types"], d["every"]) == (n, 3, every)
    assert np.array_equal(d["type"], typ)
    assert list(d["step"]) == [20, 40] and list(d["t"]) == [0.02, 0.04]
    assert list(d["R"]) == [39.5, 39.0]
    for k, (_, _, _, x) in enumerate(frames):
        assert np.array_equal(d["x"][k], x)
    bad = tmp_path / "bad"
    bad.write_bytes(b"NOTATRAJ" + b"\x00" * 64)
    with pytest.raises(ValueError):
        ldrop.read_trajectory(str(bad))


def test_radius_marshalling():
    r = ldrop.make_radius(W.Radius(kind=W.RADIUS_TABLE, knots_t=(0.0, 1.0, 2.5),
                                   knots_R=(10.0, 8.0, 9.0)))
    assert r.kind == 3 and r.n_knots == 3
    assert list(r.tab_t[:3]) == [0.0, 1.0, 2.5] and list(r.tab_R[:3]) == [10.0, 8.0, 9.0]
    s = ldrop.make_radius(W.Radius(kind=W.RADIUS_SQUARE_LAW, R0=5.0, a=2.0, R_min=1.0))
    assert (s.kind, s.n_knots, s.R0, s.a, s.R_min) == (2, 0, 5.0, 2.0, 1.0)
    with pytest.raises(ValueError):
        ldrop.make_radius(W.Radius(kind=W.RADIUS_TABLE, knots_t=(0.0, 1.0), knots_R=(1.0,)))
    with pytest.raises(ValueError):
        ldrop.make_radius(W.Radius(kind=W.RADIUS_TABLE, knots_t=tuple(range(17)),
                                   knots_R=(1.0,) * 17))
