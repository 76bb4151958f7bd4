"""Kernel timing (pp_profile_enable / pp_profile_read) as bench.py uses it:
every tile pass is counted once, in the single-circuit and the batched
path, the timed totals are positive and no longer than the wall time, and
nothing is recorded while timing is off."""
import sys
import time

import numpy as np
import pytest

from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def test_profile_counts_tile_passes(api):
    import torch
    from paper_2502_10685_amd import _lib as L
    print("profile: n=9,10 tiled circuits", flush=True)
    sys.stdout.flush()
    wcs = [W.random_circuit(np.random.default_rng(70 + i), 9 + i % 2, 240) for i in range(4)]
    cs = [api.Circuit.from_workload(w) for w in wcs]
    for c in cs:
        c.evaluate()
    torch.cuda.synchronize()
    passes = [int(c.stats()["passes"]) for c in cs]
    assert min(passes) > 1
    out = torch.empty(len(cs), dtype=torch.float64, device="cuda")
    api.evaluate_batch(cs, out)
    torch.cuda.synchronize()
    L.profile_enable(True)
    try:
        L.profile_read()
        t0 = time.perf_counter()
        cs[0].evaluate()
        torch.cuda.synchronize()
        wall1 = (time.perf_counter() - t0) * 1e3
        p1 = L.profile_read()
        t0 = time.perf_counter()
        api.evaluate_batch(cs, out)
        torch.cuda.synchronize()
        wall2 = (time.perf_counter() - t0) * 1e3
        p2 = L.profile_read()
    finally:
        L.profile_enable(False)
    launches1, ms1 = p1["tile_pass"]
    assert launches1 == passes[0]
    assert 0.0 < ms1 <= wall1
    # batched: pass l of the circuits that share a tile size is one launch
    launches2, ms2 = p2["tile_pass"]
    assert max(passes) <= launches2 <= sum(passes)
    assert 0.0 < ms2 <= wall2
    cs[1].evaluate()
    torch.cuda.synchronize()
    assert L.profile_read() == {}
    for c in cs:
        c.close()


def test_profile_records_no_tile_pass_without_passes(api):
    """A tiled circuit with no gates has no tile pass: the timing records
    none (the bracketing events are only kept around launches)."""
    import torch
    from paper_2502_10685_amd import _lib as L
    print("profile: n=8, no gates", flush=True)
    wc = W.make_circuit(8, W._arrays([], [], [], []), 0, W.obs_z(8, [0, 1]), np.zeros(0))
    c = api.Circuit.from_workload(wc)
    assert float(c.evaluate().item()) == 1.0  # <0|Z0 Z1|0>
    torch.cuda.synchronize()
    L.profile_enable(True)
    try:
        L.profile_read()
        ev = float(c.evaluate().item())
        torch.cuda.synchronize()
        prof = L.profile_read()
    finally:
        L.profile_enable(False)
    assert ev == 1.0
    assert "tile_pass" not in prof
    c.close()
