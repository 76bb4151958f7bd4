"""Parameter sweeps (pp_evaluate_thetas) and the parameter-shift gradient
built on them, against one-at-a-time evaluation, the adjoint gradient and the
CPU oracle."""
import math

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


@pytest.mark.parametrize("n,dtype", [(5, "f64"), (9, "f64"), (9, "f32"), (10, "f64")])
def test_sweep_equals_one_at_a_time_bitwise(api, n, dtype):
    """Every parameter set of a sweep gives the bits of pp_evaluate at that
    theta (same schedule, same maps, same reduction order)."""
    rng = np.random.default_rng(900 + n)
    wc = W.random_circuit(rng, n, 700, W.obs_tfim(n))
    thetas = rng.uniform(0, 2 * math.pi, size=(6, wc.n_params))
    c = api.Circuit.from_workload(wc, engine="dense", dtype=dtype)
    print(f"sweep n={n} {dtype}", flush=True)
    got = c.evaluate_thetas(thetas).cpu().numpy()
    for i in range(thetas.shape[0]):
        c.set_theta(thetas[i])
        solo = float(c.evaluate().item())
        assert got[i] == solo, (i, got[i], solo)
    if dtype == "f64":
        for i in (0, 5):
            assert abs(got[i] - oracle.expval_sv(wc.with_theta(thetas[i]))) <= 1e-12


def test_sweep_device_thetas_reuse_and_growth(api):
    import torch
    rng = np.random.default_rng(911)
    wc = W.random_circuit(rng, 8, 500, W.obs_z(8, [0, 3]))
    c = api.Circuit.from_workload(wc)
    t5 = rng.uniform(0, 2 * math.pi, size=(5, wc.n_params))
    a = c.evaluate_thetas(t5).cpu().numpy()
    b = c.evaluate_thetas(torch.tensor(t5, device="cuda")).cpu().numpy()
    assert np.array_equal(a, b)
    t3 = t5[[4, 0, 2]]
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    c3 = c.evaluate_thetas(t3, out=out).cpu().numpy()
    assert np.array_equal(c3, a[[4, 0, 2]])
    t9 = np.concatenate([t5, t5[:4]])
    c9 = c.evaluate_thetas(t9).cpu().numpy()
    assert np.array_equal(c9[:5], a) and np.array_equal(c9[5:], a[:4])


def test_sweep_rejects_other_engines(api):
    from paper_2502_10685_amd._lib import PauliPropError
    wc = W.config1()
    for kw in ({"engine": "sparse"}, {"track": True}):
        c = api.Circuit.from_workload(wc, **kw)
        with pytest.raises(PauliPropError):
            c.evaluate_thetas(np.zeros((2, wc.n_params)))


def test_psr_gradient_shared_parameter(api):
    # two rotations on one parameter: d/dt <Z> of RY(t) RY(t) = -2 sin 2t
    gates = (np.array([4, 4], np.uint8), np.array([0, 0], np.int32), np.array([-1, -1], np.int32),
             np.array([0, 0], np.int32))
    wc = W.make_circuit(1, gates, 1, W.obs_z(1, [0]), [0.4])
    c = api.Circuit.from_workload(wc)
    g = c.psr_gradient(wc.theta).cpu().numpy()
    assert abs(g[0] + 2 * math.sin(0.8)) <= 1e-14


def test_psr_gradient_config4_matches_adjoint_and_oracle(api):
    """n = 8, HEA-40, TFIM: the 1,920 shifted evaluations run as one sweep;
    the result matches the adjoint gradient and the oracle's parameter-shift
    gradient within 1e-10."""
    wc = W.config4()
    c = api.Circuit.from_workload(wc)
    print("psr sweep config4", flush=True)
    g_psr = c.psr_gradient(wc.theta).cpu().numpy()
    _, g_adj = c.gradient(5 * 32)
    g_adj = g_adj.cpu().numpy()
    assert np.max(np.abs(g_psr - g_adj)) <= 1e-10
    assert np.max(np.abs(g_psr - oracle.psr_gradient(wc))) <= 1e-10
