"""Host logic of the Clifford-frame SPARSE engine, checked on the CPU with
dense matrices (no GPU): the rotation axis P = D sigma D^dag the planner
gives every pass, the x rows of the final frame, the sign rule of a child
i P S, and propagation in the stored frame against the scalar propagator."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

LIB = pytest.importorskip("paper_2502_10685_amd._lib")


def _frame(w):
    try:
        return LIB.plan_sparse_frame(w.n, w.op, w.q0, w.q1, w.param, w.n_params)
    except RuntimeError as e:  # library not built
        pytest.skip(str(e))


def _pauli(n, key):
    x = int(key) & ((1 << n) - 1)
    z = int(key) >> n
    return oracle.pauli_matrix(n, x, z)


def _axis_matrix(n, op, q):
    letter = {3: (1, 0), 4: (1, 1), 5: (0, 1)}[op]
    return oracle.pauli_matrix(n, letter[0] << q, letter[1] << q)


def _all_keys(n):
    return range(4 ** n)


def _as_pauli(n, m):
    """(key, sign) with m = sign * Pauli(key), or None."""
    for key in _all_keys(n):
        p = _pauli(n, key)
        for s in (1, -1):
            if np.allclose(m, s * p, atol=1e-12):
                return key, s
    return None


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (2, 3), (3, 4), (3, 5), (4, 6)])
def test_rotation_axes_and_xrows_match_dense_conjugation(n, seed):
    rng = np.random.default_rng(900 + seed)
    w = W.random_circuit(rng, n, 60, W.obs_z(n, [0]))
    pmask, sign, rot_param, ngates, xrows = _frame(w)
    dim = 1 << n
    D = np.eye(dim, dtype=complex)
    passes = 0
    for g in range(w.m - 1, -1, -1):  # Heisenberg order: g_m first
        op = int(w.op[g])
        if op <= 2:
            D = D @ oracle.gate_unitary(n, op, int(w.q0[g]), int(w.q1[g]), 0.0)
            continue
        P = D @ _axis_matrix(n, op, int(w.q0[g])) @ D.conj().T
        want = sign[passes] * _pauli(n, pmask[passes])
        assert np.allclose(P, want, atol=1e-12), (g, passes)
        assert rot_param[passes] == w.param[g]
        passes += 1
    assert passes == int(np.sum(w.op >= 3))
    assert int(np.sum(ngates)) == w.m
    # the x part of D^dag G D for every generator G of the stored key
    for b in range(2 * n):
        img = D.conj().T @ _pauli(n, 1 << b) @ D
        key, _ = _as_pauli(n, img)
        x = key & ((1 << n) - 1)
        for j in range(n):
            assert ((x >> j) & 1) == (bin((1 << b) & int(xrows[j])).count("1") & 1)


def test_child_sign_rule():
    """i P S = sign * Pauli(key(P) ^ key(S)) for anticommuting Hermitian P,
    S, with sign = +1 iff (1 + |xP zP| + |xS zS| + 2|zP xS| - |x' z'|) = 0
    mod 4 (the rule the frame kernel uses), for every pair on two qubits."""
    n = 2
    lo = (1 << n) - 1
    for kp, ks in itertools.product(_all_keys(n), repeat=2):
        xp, zp, xs, zs = kp & lo, kp >> n, ks & lo, ks >> n
        if (bin(xs & zp).count("1") + bin(zs & xp).count("1")) % 2 == 0:
            continue
        m = 1j * _pauli(n, kp) @ _pauli(n, ks)
        key, s = _as_pauli(n, m)
        assert key == kp ^ ks
        e = (1 + bin(xp & zp).count("1") + bin(xs & zs).count("1") + 2 * bin(zp & xs).count("1")
             - bin((xs ^ xp) & (zs ^ zp)).count("1")) % 4
        assert s == (1 if e == 0 else -1)


def _pauli_coeffs(n, m):
    return {key: float(np.real(np.trace(_pauli(n, key) @ m))) / (1 << n) for key in _all_keys(n)}


@pytest.mark.parametrize("n,seed", [(2, 7), (3, 8)])
def test_stored_frame_propagation_matches_oracle(n, seed):
    """Rotate in the stored frame about P (dense exp), never applying the
    Clifford gates, then map the final operator back with D^dag . D: the
    weights equal the scalar propagator's."""
    rng = np.random.default_rng(950 + seed)
    w = W.random_circuit(rng, n, 50, W.obs_tfim(n) if n >= 2 else W.obs_z(1, [0]))
    pmask, sign, rot_param, _, _ = _frame(w)
    O = oracle.obs_matrix(n, w.obs_x, w.obs_z, w.obs_c)
    D = np.eye(1 << n, dtype=complex)
    i = 0
    for g in range(w.m - 1, -1, -1):
        op = int(w.op[g])
        if op <= 2:
            D = D @ oracle.gate_unitary(n, op, int(w.q0[g]), int(w.q1[g]), 0.0)
            continue
        th = float(w.theta[rot_param[i]])
        P = sign[i] * _pauli(n, pmask[i])
        R = math.cos(th / 2) * np.eye(1 << n) - 1j * math.sin(th / 2) * P
        O = R.conj().T @ O @ R
        i += 1
    actual = D.conj().T @ O @ D
    want = oracle.propagate(w).as_dict()
    got = _pauli_coeffs(n, actual)
    for key, v in got.items():
        x, z = key & ((1 << n) - 1), key >> n
        assert abs(v - want.get((x, z), 0.0)) < 1e-12
