"""Adjoint gradient (pp_gradient and the autograd binding) against the
parameter-shift rule and central differences of the CPU oracle.

Bars: adjoint vs parameter-shift <= 1e-10 absolute (both analytic), vs
central differences with h = 1e-6 <= 1e-6 absolute."""
import math

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_PSR = 1e-10
TOL_FD = 1e-6


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _grad(api, wc, every=0):
    c = api.Circuit.from_workload(wc)
    ev, g = c.gradient(every)
    return float(ev.item()), g.cpu().numpy()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_adjoint_vs_psr_random(api, n):
    rng = np.random.default_rng(300 + n)
    obs = W.obs_tfim(n) if n >= 2 else W.obs_z(1, [0])
    wc = W.random_circuit(rng, n, 120, obs)
    print(f"gradient random n={n}", flush=True)
    ev, g = _grad(api, wc, every=37)
    assert abs(ev - oracle.expval_sv(wc)) <= 1e-12
    psr = oracle.psr_gradient(wc)
    assert np.max(np.abs(g - psr)) <= TOL_PSR, np.max(np.abs(g - psr))


def test_checkpoint_interval_does_not_change_the_gradient(api):
    rng = np.random.default_rng(41)
    wc = W.random_circuit(rng, 9, 200, W.obs_z(9, [0, 4]))
    print("gradient checkpoints n=9", flush=True)
    ref_ev, ref = _grad(api, wc, every=0)
    for every in (1, 13, 64, 10000):
        # segment boundaries change how single-qubit gates are folded, so
        # the rounding (not the value) of <O> may differ
        ev, g = _grad(api, wc, every=every)
        assert abs(ev - ref_ev) <= 1e-14
        assert np.max(np.abs(g - ref)) <= 1e-12
    assert np.max(np.abs(ref - oracle.psr_gradient(wc))) <= TOL_PSR


def test_shared_parameters_are_summed(api):
    # two rotations on one parameter: d/dt <Z> of RY(t) RY(t) = -2 sin 2t
    gates = (np.array([4, 4], np.uint8), np.array([0, 0], np.int32), np.array([-1, -1], np.int32),
             np.array([0, 0], np.int32))
    wc = W.make_circuit(1, gates, 1, W.obs_z(1, [0]), [0.4])
    ev, g = _grad(api, wc)
    assert abs(ev - math.cos(0.8)) <= 1e-15
    assert abs(g[0] + 2 * math.sin(0.8)) <= 1e-14


def test_config4_hea8_tfim_full(api):
    """n = 8, HEA-40 (960 parameters), TFIM, checkpoint every 5 layers (160
    gates): adjoint vs 2 x 960 parameter-shift evaluations vs central
    differences."""
    wc = W.config4()
    print("gradient config4", flush=True)
    ev, g = _grad(api, wc, every=5 * 32)
    assert abs(ev - oracle.expval_sv(wc)) <= 1e-12
    psr = oracle.psr_gradient(wc)
    e_psr = float(np.max(np.abs(g - psr)))
    fd = oracle.fd_gradient(wc, h=1e-6)
    e_fd = float(np.max(np.abs(g - fd)))
    print(f"config4: max |adjoint - psr| = {e_psr:.2e}, max |adjoint - fd| = {e_fd:.2e}", flush=True)
    assert e_psr <= TOL_PSR and e_fd <= TOL_FD


def test_autograd_binding(api):
    import torch
    wc = W.hea_circuit(17, 4, 3, W.obs_tfim(4))
    c = api.Circuit.from_workload(wc)
    theta = torch.tensor(wc.theta, device="cuda", requires_grad=True)
    f = api.expval(c, theta, 8)
    (2.0 * f).backward()
    want = 2.0 * oracle.psr_gradient(wc)
    assert abs(float(f.item()) - oracle.expval_sv(wc)) <= 1e-12
    assert np.max(np.abs(theta.grad.cpu().numpy() - want)) <= 2 * TOL_PSR
    # without requires_grad the forward is a plain evaluation
    f2 = api.expval(c, theta.detach())
    assert float(f2.item()) == pytest.approx(float(f.item()), abs=1e-12)


def test_autograd_forward_runs_no_gradient(api):
    """The forward evaluates <O> only; the adjoint sweep runs in backward
    (its forward-sweep kernels are timed as tile passes: none before
    backward).  A CPU angle tensor that requires grad gets its gradient on
    the CPU."""
    import torch
    from paper_2502_10685_amd import _lib as L
    wc = W.hea_circuit(18, 5, 3, W.obs_tfim(5))
    c = api.Circuit.from_workload(wc)
    theta = torch.tensor(wc.theta, requires_grad=True)  # CPU
    L.profile_enable(True)
    L.profile_read()
    f = api.expval(c, theta, 6)
    torch.cuda.synchronize()
    fwd = L.profile_read()
    assert "tile_pass" not in fwd and "resident" in fwd, fwd
    f.backward()
    torch.cuda.synchronize()
    bwd = L.profile_read()
    L.profile_enable(False)
    assert "tile_pass" in bwd, bwd
    assert theta.grad.device.type == "cpu"
    assert np.max(np.abs(theta.grad.numpy() - oracle.psr_gradient(wc))) <= TOL_PSR
    assert abs(float(f.item()) - oracle.expval_sv(wc)) <= 1e-12


def test_autograd_backward_uses_the_forward_angles(api):
    """Angles changed on the circuit between forward and backward do not
    change the gradient of the recorded forward."""
    import torch
    wc = W.hea_circuit(19, 4, 2, W.obs_tfim(4))
    c = api.Circuit.from_workload(wc)
    theta = torch.tensor(wc.theta, device="cuda", requires_grad=True)
    f = api.expval(c, theta)
    c.set_theta(np.zeros(wc.n_params))
    f.backward()
    assert np.max(np.abs(theta.grad.cpu().numpy() - oracle.psr_gradient(wc))) <= TOL_PSR


def test_gradient_rejects_other_engines(api):
    from paper_2502_10685_amd._lib import PauliPropError
    wc = W.config1()
    c = api.Circuit.from_workload(wc, engine="sparse")
    with pytest.raises(PauliPropError):
        c.gradient()
    c = api.Circuit.from_workload(wc, dtype="f32")
    with pytest.raises(PauliPropError):
        c.gradient()


def test_gradient_graph_replays_match_eager(api):
    """PP_OPT_USE_GRAPH captures the whole gradient launch sequence once;
    replays with new theta (set between replays, with eager work and
    synchronizations in between) give the eager results bit for bit."""
    import torch
    rng = np.random.default_rng(520)
    wc = W.random_circuit(rng, 9, 300, W.obs_tfim(9))
    eager = api.Circuit.from_workload(wc)
    graph = api.Circuit.from_workload(wc, use_graph=True)
    for rep in range(4):
        th = rng.uniform(0, 2 * math.pi, size=wc.n_params)
        eager.set_theta(th)
        ev_e, g_e = eager.gradient(64)
        if rep % 2:
            graph.set_theta(torch.tensor(th, device="cuda"))
        else:
            graph.set_theta(th)
        ev_g, g_g = graph.gradient(64)
        torch.cuda.synchronize()
        assert float(ev_g.item()) == float(ev_e.item())
        assert np.array_equal(g_g.cpu().numpy(), g_e.cpu().numpy())
        _ = eager.evaluate()  # unrelated eager work between replays
        torch.cuda.synchronize()
