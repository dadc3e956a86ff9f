"""ld_forces_noalloc (pair forces with the scratch in a static device array)
through the C ABI against ld_forces of a context on the same particles, two
calls in a row, the second smaller: max |dF_i| <= 1e-5 S_i (S_i from the
oracle) between the two entry points and against the oracle, median
|dF|/|F| <= 1e-5; sizes beyond the array are refused."""
import ctypes as C

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


def noalloc(ld, w):
    import torch
    dev = torch.device("cuda")
    t = torch.as_tensor(np.ascontiguousarray(w.type, np.int32), device=dev)
    q = torch.as_tensor(np.ascontiguousarray(w.charge, np.float64), device=dev)
    x = torch.as_tensor(np.ascontiguousarray(w.pos, np.float32), device=dev)
    F = torch.full((w.n, 3), float("nan"), dtype=torch.float64, device=dev)
    p = ld.make_params(w.params)
    st = ld.lib().ld_forces_noalloc(w.n, C.c_void_p(t.data_ptr()), C.c_void_p(q.data_ptr()),
                                    C.c_void_p(x.data_ptr()), C.byref(p),
                                    C.c_void_p(F.data_ptr()),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, ld.lib().ld_last_error()
    torch.cuda.synchronize()
    return F.cpu().numpy()


def check(ld, w):
    import oracle
    print(f"no-alloc forces n={w.n}", flush=True)
    Fs = noalloc(ld, w)
    Fc = ld.System.from_workload(w).forces(ext=False)["pair"].cpu().numpy()
    Fo, So, _ = oracle.pair_forces(w.pos, w.type, w.charge, w.params)
    for F in (Fc, Fo):
        dF = np.linalg.norm(Fs - F, axis=1)
        assert np.all(dF <= 1e-5 * So), (dF / np.maximum(So, 1e-300)).max()
        nrm = np.linalg.norm(F, axis=1)
        assert np.median(dF[nrm > 0] / nrm[nrm > 0]) <= 1e-5


def test_noalloc_matches_ld_forces_twice(ld):
    check(ld, W.config_large(n=3001, seed=41))   # three types, ragged tail
    check(ld, W.config_small(n=700, seed=42))    # smaller, one type: old contents unused


def test_noalloc_limits(ld):
    import torch
    w = W.config_small(n=700, seed=43)
    p = ld.make_params(w.params)
    dev = torch.device("cuda")
    big = 65537
    t = torch.zeros(big, dtype=torch.int32, device=dev)
    q = torch.zeros(big, dtype=torch.float64, device=dev)
    x = torch.zeros((big, 3), dtype=torch.float32, device=dev)
    F = torch.zeros((big, 3), dtype=torch.float64, device=dev)
    args = [C.c_void_p(a.data_ptr()) for a in (t, q, x)]
    assert ld.lib().ld_forces_noalloc(big, *args, C.byref(p), C.c_void_p(F.data_ptr()),
                                      None) == -1
    assert b"65536" in ld.lib().ld_last_error()
    host = np.zeros((700, 3), np.float32)
    assert ld.lib().ld_forces_noalloc(700, *args[:2], host.ctypes.data_as(C.c_void_p),
                                      C.byref(p), C.c_void_p(F.data_ptr()), None) == -1
