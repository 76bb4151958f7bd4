"""pp_evaluate_noalloc through the C ABI: the same result as pp_evaluate (the
existing entry point, whose working buffers the library allocates), with
nothing allocated by the call.  Two calls in a row, the second on a smaller
circuit, then the first again; LDS-resident and tiled, FP64 and FP32."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _noalloc(lib, c, out):
    import torch
    return lib.pp_evaluate_noalloc(c._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                   ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_evaluate_two_calls(api, dtype):
    import torch
    from paper_2502_10685_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(4242)
    big = W.random_circuit(rng, 10, 3000, W.obs_z(10, [0, 1]))   # tiled, 4^10 weights
    small = W.random_circuit(rng, 8, 1200, W.obs_tfim(8))        # tiled, 4^8 weights
    tiny = W.random_circuit(rng, 6, 2000, W.obs_z(6, [2]))       # LDS-resident
    cs = [api.Circuit.from_workload(w, dtype=dtype) for w in (big, small, tiny)]
    want = [float(c.evaluate().item()) for c in cs]  # also puts each schedule on the device
    torch.cuda.synchronize()
    out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    t0, l0 = torch.cuda.memory_allocated(), L.memory_in_use()
    print(f"noalloc {dtype}: n=10 then n=8 then n=6 then n=10", flush=True)
    for i, c in zip((0, 1, 2, 3), (cs[0], cs[1], cs[2], cs[0])):
        L.check(_noalloc(lib, c, out[i]))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert L.memory_in_use() == l0 and torch.cuda.memory_allocated() == t0  # nothing allocated
    assert got[0] == want[0] and got[1] == want[1] and got[2] == want[2] and got[3] == want[0]
    tol = 1e-12 if dtype == "f64" else 1e-5
    for v, w in zip(got[:3], (big, small, tiny)):
        assert abs(v - oracle.expval_sv(w)) <= tol
    # the circuits' own weights are untouched: evaluating again gives the same
    assert [float(c.evaluate().item()) for c in cs] == want
    for c in cs:
        c.close()


def test_noalloc_new_theta_and_errors(api):
    import torch
    from paper_2502_10685_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(77)
    w = W.random_circuit(rng, 9, 2500, W.obs_z(9, [0]))
    c = api.Circuit.from_workload(w)
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    # schedule not on the device yet
    assert _noalloc(lib, c, out[0]) == L.PP_ERR_STATE
    c.evaluate()
    th = rng.uniform(0, 2 * np.pi, size=w.n_params)
    c.set_theta(th)  # new angles are read at the next call
    L.check(_noalloc(lib, c, out[0]))
    torch.cuda.synchronize()
    assert abs(float(out[0].item()) - oracle.expval_sv(w.with_theta(th))) <= 1e-12
    assert float(out[0].item()) == float(c.evaluate().item())
    # a working set larger than the array: n = 11 in FP64 (32 MiB of weights)
    w11 = W.random_circuit(rng, 11, 300, W.obs_z(11, [0]))
    c11 = api.Circuit.from_workload(w11)
    c11.evaluate()
    assert _noalloc(lib, c11, out[1]) == L.PP_ERR_CAPACITY
    assert b"exceeds" in lib.pp_last_error()
    # tracked and SPARSE circuits are not served by this entry point
    ct = api.Circuit.from_workload(w, track=True)
    ct.evaluate()
    assert _noalloc(lib, ct, out[1]) == L.PP_ERR_STATE
    cs = api.Circuit.from_workload(w, engine="sparse")
    cs.evaluate()
    assert _noalloc(lib, cs, out[1]) == L.PP_ERR_STATE
    for o in (c, c11, ct, cs):
        o.close()
