"""Device memory through the allocator hook (pp_set_allocator): the Python
binding hands the library torch's caching allocator; an allocator that fails
gives PP_ERR_NOMEM and leaves the circuit usable."""
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


def test_library_memory_comes_from_torch(api):
    """The weights of an n = 11 circuit (4^11 doubles, 32 MiB) are allocated
    by torch's caching allocator when the circuit is first evaluated."""
    import torch
    from paper_2502_10685_amd._lib import memory_in_use
    api.set_allocator()  # torch's caching allocator (the binding's default)
    w = W.random_circuit(11, 11, 300, W.obs_z(11, [0, 1]))
    c = api.Circuit.from_workload(w)
    torch.cuda.synchronize()
    t0, l0 = torch.cuda.memory_allocated(), memory_in_use()[0]
    v = float(c.evaluate().item())
    t1, l1 = torch.cuda.memory_allocated(), memory_in_use()[0]
    assert abs(v - oracle.expval_sv(w)) <= 1e-12
    assert l1 - l0 >= 8 * 4 ** 11
    assert t1 - t0 >= 8 * 4 ** 11  # torch accounts for the library's blocks
    c.close()
    assert memory_in_use()[0] <= l0


def test_failing_allocator_gives_nomem_and_circuit_stays_usable(api):
    """With an allocator that returns NULL, the first evaluation fails with
    PP_ERR_NOMEM; with memory back, the same circuit evaluates correctly.
    Blocks made by torch's allocator are still returned to it."""
    from paper_2502_10685_amd._lib import PauliPropError, PP_ERR_NOMEM
    calls = {"alloc": 0, "free": 0}

    def no_memory(nbytes):
        calls["alloc"] += 1
        return None

    def never(ptr):
        calls["free"] += 1

    for n, m in ((10, 500), (6, 400)):  # tiled and LDS-resident
        w = W.random_circuit(20 + n, n, m, W.obs_z(n, [0]))
        api.set_allocator()
        c = api.Circuit.from_workload(w)  # angles and observable uploaded
        api.set_allocator(no_memory, never)
        try:
            with pytest.raises(PauliPropError) as ei:
                c.evaluate()
            assert ei.value.status == PP_ERR_NOMEM
            with pytest.raises(PauliPropError) as ei:
                c.gradient()
            assert ei.value.status == PP_ERR_NOMEM
        finally:
            api.set_allocator()
        assert calls["alloc"] >= 1 and calls["free"] == 0
        v = float(c.evaluate().item())
        assert abs(v - oracle.expval_sv(w)) <= 1e-12
        ev, g = c.gradient()
        assert abs(float(ev.item()) - v) <= 1e-12
        c.close()
    assert calls["free"] == 0


def test_default_pool_allocator(api):
    """pp_set_allocator(NULL): the library's own stream-ordered pool gives
    the same results; blocks of torch's allocator made before the switch go
    back to torch."""
    import torch
    from paper_2502_10685_amd._lib import memory_in_use
    w = W.random_circuit(31, 9, 1500, W.obs_z(9, [0, 1]))
    api.set_allocator()
    a = api.Circuit.from_workload(w)
    va = float(a.evaluate().item())
    api.reset_allocator()
    try:
        b = api.Circuit.from_workload(w)
        vb = float(b.evaluate().item())
        assert va == vb
        a.close()  # made by torch, returned to torch
        b.close()
    finally:
        api.set_allocator()
    torch.cuda.synchronize()
    assert abs(va - oracle.expval_sv(w)) <= 1e-12
    assert memory_in_use()[1] >= 0
