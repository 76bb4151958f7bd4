"""GPU parity of pp_density_matrix (the paper's toDM task) against the CPU
oracle: rho = psi psi^dag from the FP64 state vector, and for small n also
rho = 2^-n prod_j (I + P_j) from the forward-evolved generators (eq. (2)).

Bars: every entry within 1e-12 (FP64 weights) or 1e-5 (FP32 weights);
Tr rho = 1, Tr rho^2 = 1 and rho Hermitian within the same bars.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rho_sv(wc):
    psi = oracle.statevector(wc)
    return np.outer(psi, psi.conj())


def _check(rho, want, tol):
    assert rho.shape == want.shape
    err = float(np.max(np.abs(rho - want)))
    assert err <= tol, err
    assert abs(np.trace(rho) - 1.0) <= tol
    assert abs(np.trace(rho @ rho) - 1.0) <= 10 * tol
    assert float(np.max(np.abs(rho - rho.conj().T))) <= tol
    return err


@pytest.mark.parametrize("n,m,seed", [(1, 40, 1), (2, 80, 2), (3, 120, 3), (5, 300, 5), (7, 400, 7),
                                      (8, 300, 8), (9, 300, 9)])
def test_density_matrix_matches_state_vector(api, n, m, seed):
    wc = W.random_circuit(np.random.default_rng(seed), n, m)
    _say(f"density n={n} m={m} seed={seed}")
    c = api.Circuit.from_workload(wc)
    rho = c.density_matrix().cpu().numpy()
    _check(rho, _rho_sv(wc), TOL64)
    # a second call with new theta reuses the internal circuit
    th = np.random.default_rng(seed + 100).uniform(0, 2 * np.pi, wc.n_params)
    c.set_theta(th)
    rho2 = c.density_matrix().cpu().numpy()
    _check(rho2, _rho_sv(wc.with_theta(th)), TOL64)
    c.close()


@pytest.mark.parametrize("n,seed", [(3, 11), (4, 12)])
def test_density_matrix_matches_generator_product(api, n, seed):
    """eq. (2): the product of the n evolved generators (oracle) equals the
    group-sum route the GPU takes."""
    wc = W.random_circuit(np.random.default_rng(seed), n, 60)
    _say(f"density vs generators n={n}")
    c = api.Circuit.from_workload(wc)
    rho = c.density_matrix().cpu().numpy()
    _check(rho, oracle.rho_from_generators(wc), TOL64)
    c.close()


@pytest.mark.parametrize("k", [4, 5])
def test_density_matrix_tile_sizes(api, k):
    wc = W.random_circuit(np.random.default_rng(40 + k), 8, 250)
    _say(f"density n=8 tile_qubits={k}")
    c = api.Circuit.from_workload(wc, tile_qubits=k)
    _check(c.density_matrix().cpu().numpy(), _rho_sv(wc), TOL64)
    c.close()


def test_density_matrix_fp32(api):
    wc = W.random_circuit(np.random.default_rng(31), 6, 300)
    _say("density fp32 n=6")
    c = api.Circuit.from_workload(wc, dtype="f32")
    _check(c.density_matrix().cpu().numpy(), _rho_sv(wc), TOL32)
    c.close()


def test_density_matrix_paper_chain_workload(api):
    """The paper's timing shape: n = 4, 60,200 gates (CX ring + RZ RX RZ)."""
    wc = W.chain_zxz_circuit()
    _say(f"density {wc.name} m={wc.m}")
    c = api.Circuit.from_workload(wc)
    err = _check(c.density_matrix().cpu().numpy(), _rho_sv(wc), TOL64)
    _say(f"density {wc.name}: max |rho - psi psi^dag| = {err:.2e}")
    c.close()


@pytest.mark.parametrize("n,layers,repeats", [(2, 1000, 1), (3, 100, 1), (4, 1, 1), (2, 50, 100), (3, 50, 10),
                                               (4, 50, 1)])
def test_density_matrix_paper_sweep_points(api, n, layers, repeats):
    """Points of the paper's two timing sweeps (Sec. V): W_chain+ZXZ at
    n = 2..4, #Layers up to 1000 at #Repeats = 1, #Repeats up to 100 at
    #Layers = 50."""
    wc = W.chain_zxz_circuit(seed=1000 * n + layers + repeats, n=n, layers=layers, repeats=repeats)
    _say(f"density sweep n={n} layers={layers} repeats={repeats} m={wc.m}")
    c = api.Circuit.from_workload(wc)
    err = _check(c.density_matrix().cpu().numpy(), _rho_sv(wc), TOL64)
    _say(f"density sweep n={n} layers={layers} repeats={repeats}: max error {err:.2e}")
    c.close()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_stabilizer_order_matches_forward_oracle(api, n):
    """The stabilizer order (Sec. II-B) of U_k Z_j U_k^dag after the first k
    gates of the W_chain+ZXZ ansatz: a tracked GPU run of Z_j backwards
    through the k gates reversed has exactly the size of the oracle's
    forward (Schroedinger) set."""
    wc = W.chain_zxz_circuit(seed=n, n=n, layers=2, repeats=1)
    _say(f"stabilizer order n={n} m={wc.m}")
    for k in range(0, wc.m + 1, 3):
        for j in range(n):
            fwd = W.make_circuit(n, (wc.op[:k], wc.q0[:k], wc.q1[:k], wc.param[:k]), wc.n_params,
                                 W.obs_z(n, [j]), wc.theta)
            want = len(oracle.propagate(fwd, direction=1).x)
            rev = W.make_circuit(n, (np.ascontiguousarray(wc.op[:k][::-1]), np.ascontiguousarray(wc.q0[:k][::-1]),
                                     np.ascontiguousarray(wc.q1[:k][::-1]), np.ascontiguousarray(wc.param[:k][::-1])),
                                 wc.n_params, W.obs_z(n, [j]), wc.theta)
            c = api.Circuit.from_workload(rev, track=True)
            c.evaluate()
            assert int(c.stats()["final_terms"]) == want, (k, j)
            c.close()


def test_density_matrix_clifford_state_is_a_projector(api):
    """H on every qubit: rho = |+...+><+...+|, every entry exactly 2^-n."""
    n = 5
    gates = W._arrays([W.H] * n, list(range(n)), [-1] * n, [-1] * n)
    wc = W.make_circuit(n, gates, 0, W.obs_z(n, [0]), np.zeros(0))
    c = api.Circuit.from_workload(wc)
    rho = c.density_matrix().cpu().numpy()
    assert float(np.max(np.abs(rho - 1.0 / (1 << n)))) <= TOL64
    c.close()


def test_density_matrix_rejects_large_n(api):
    import ctypes

    import torch
    from paper_2502_10685_amd import _lib as L
    wc = W.random_circuit(np.random.default_rng(1), 13, 20)
    c = api.Circuit.from_workload(wc)
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(L.PauliPropError):
        L.check(c._lib.pp_density_matrix(c._h, None, ctypes.c_void_p(out.data_ptr())))
    c.close()
