"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each oracle function is checked against something other than itself: values
the paper prints (tests/golden/*, each with its citation), closed forms,
invariants, and brute force with full matrices on a few qubits.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

RNG_SEEDS = [11, 12, 13, 14, 15]


def _one_gate(n, op, q0, q1=-1, theta=None, obs=None):
    params = [0] if op >= 3 else [-1]
    th = [theta if theta is not None else 0.0]
    gates = (np.array([op], np.uint8), np.array([q0], np.int32), np.array([q1], np.int32),
             np.array(params, np.int32))
    return W.make_circuit(n, gates, 1, obs or W.obs_z(n, [0]), th)


def _letters_circ(n, seq, theta, obs_string):
    """seq: list of (op, q0, q1); every rotation uses its own parameter."""
    ops, q0s, q1s, params = [], [], [], []
    p = 0
    for op, a, b in seq:
        ops.append(op); q0s.append(a); q1s.append(b)
        if op >= 3:
            params.append(p); p += 1
        else:
            params.append(-1)
    gates = (np.array(ops, np.uint8), np.array(q0s, np.int32), np.array(q1s, np.int32),
             np.array(params, np.int32))
    obs = W.observable([W.pauli_from_string(obs_string)])
    return W.make_circuit(n, gates, p, obs, theta)


def _read(name):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        return [ln.rstrip("\n") for ln in f if ln.strip() and not ln.startswith("#")]


# ---------------------------------------------------------------- Table I
@pytest.mark.parametrize("theta", [0.0, 0.3, 1.2, math.pi / 2, 2.5, 4.0])
def test_table1_rows_forward(theta):
    """Sec. III-C Table I: the oracle's forward single-gate image of each of
    X, Y, Z equals the printed row (golden fixture)."""
    names = {"H": 0, "S": 1, "RX": 3, "RY": 4, "RZ": 5}
    c, s = math.cos(theta), math.sin(theta)
    for line in _read("table1_rows.txt"):
        gname, rest = line.split(":")
        outs = [e.strip() for e in rest.split(";")]
        op = names[gname.strip()]
        for L_in, letter in ((1, "X"), (2, "Y"), (3, "Z")):
            w = [0.0] * 4
            w[L_in] = 1.0
            env = {"w0": w[0], "w1": w[1], "w2": w[2], "w3": w[3], "c": c, "s": s}
            expect = [eval(e, {"__builtins__": {}}, env) for e in outs]
            circ = _letters_circ(1, [(op, 0, -1)], [theta], letter)
            r = oracle.propagate(circ, direction=1)
            got = [0.0] * 4
            for x, z, v in zip(r.x, r.z, r.c):
                L = {(0, 0): 0, (1, 0): 1, (1, 1): 2, (0, 1): 3}[(int(x), int(z))]
                got[L] += v
            assert np.allclose(got, expect, atol=1e-15), (gname, letter, got, expect)


@pytest.mark.parametrize("op", [0, 1, 3, 4, 5])
@pytest.mark.parametrize("theta", [0.0, 0.7, 2.2, 5.9])
def test_single_gate_images_match_dense_conjugation(op, theta):
    """Forward image g P g^dag and Heisenberg image g^dag P g of every Pauli
    on one qubit, against 2x2 matrix conjugation with R = exp(-i theta s/2)."""
    u = oracle.gate_unitary(1, op, 0, -1, theta)
    for letter in "XYZ":
        x, z, _ = W.pauli_from_string(letter)
        P = oracle.pauli_matrix(1, x, z)
        for direction, img in ((1, u @ P @ u.conj().T), (0, u.conj().T @ P @ u)):
            circ = _letters_circ(1, [(op, 0, -1)], [theta], letter)
            r = oracle.propagate(circ, direction=direction)
            got = oracle.obs_matrix(1, r.x, r.z, r.c)
            assert np.allclose(got, img, atol=1e-14), (op, letter, direction)


def test_cx_pairs_golden_and_dense():
    """Sec. III-C CX list (control = first letter, XZ <-> -YY), checked both
    against the printed list and against 4x4 matrix conjugation."""
    u = oracle.gate_unitary(2, 2, 0, 1, 0.0)
    seen = set()
    for line in _read("cx_pairs.txt"):
        a, b = line.split()
        sign = -1.0 if b.startswith("-") else 1.0
        b = b.lstrip("-")
        for src, dst in ((a, b), (b, a)):
            seen.add(src)
            circ = _letters_circ(2, [(2, 0, 1)], [], src)
            for direction in (0, 1):
                r = oracle.propagate(circ, direction=direction)
                assert len(r.c) == 1
                assert oracle.symplectic_to_string(2, r.x[0], r.z[0]) == dst
                assert r.c[0] == sign
            x, z, _ = W.pauli_from_string(src)
            P = oracle.pauli_matrix(2, x, z)
            xd, zd, _ = W.pauli_from_string(dst)
            assert np.allclose(u @ P @ u.conj().T, sign * oracle.pauli_matrix(2, xd, zd))
    assert len(seen) == 16


# ------------------------------------------------------------- worked examples
@pytest.mark.parametrize("t1,t2", [(0.4, 1.1), (2.0, -0.7), (math.pi / 3, 5.0)])
def test_example1(t1, t2):
    """Example 1 (Sec. II-B): X -> R_y(t1) -> R_x(t2)."""
    circ = _letters_circ(1, [(4, 0, -1), (3, 0, -1)], [t1, t2], "X")
    r = oracle.propagate(circ, direction=1)
    got = {oracle.symplectic_to_string(1, x, z): v for x, z, v in zip(r.x, r.z, r.c)}
    for line in _read("example1.txt"):
        letter, expr = line.split(":")
        want = eval(expr, {"__builtins__": {}, "cos": math.cos, "sin": math.sin},
                    {"t1": t1, "t2": t2})
        assert abs(got[letter.strip()] - want) < 1e-15
    assert set(got) == {"X", "Y", "Z"}


def test_example2_index():
    for line in _read("example2.txt"):
        s, idx = line.split()
        assert oracle.string_to_index(s) == int(idx)
        assert oracle.index_to_string(int(idx), len(s)) == s
    for k in range(64):
        assert oracle.string_to_index(oracle.index_to_string(k, 3)) == k


def test_example3_expand_reduce():
    lines = dict(ln.split(":", 1) for ln in _read("example3.txt"))
    w = eval(lines["weights"])
    lam = oracle.expand_reduce(w)
    ones = [int(t) for t in lines["ones_at"].split()]
    assert lam.shape == (16,)
    assert sorted(np.nonzero(lam)[0].tolist()) == ones
    assert np.all(lam[ones] == 1.0)
    assert [oracle.index_to_string(i, 2) for i in ones] == lines["strings"].split()


def test_example4_flatten_reduce():
    lines = dict(ln.split(":", 1) for ln in _read("example4.txt"))
    w = eval(lines["weights"])
    rows = oracle.flatten(w)
    row = [float(t) for t in lines["row"].split()]
    assert rows.shape == (2, 16)
    assert np.array_equal(rows[0], row) and np.array_equal(rows[1], row)
    red = oracle.flatten_reduce(w)
    assert red[0] == float(lines["reduced_first"]) and red[-1] == float(lines["reduced_last"])
    assert np.array_equal(red, 2 * np.array(row))


def test_symplectic_string_roundtrip():
    for s in ["I", "X", "Y", "Z", "XYZ", "IZXY", "YYII"]:
        x, z, _ = W.pauli_from_string(s)
        assert oracle.symplectic_to_string(len(s), x, z) == s


# ----------------------------------------------------------- state vector
@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_statevector_vs_dense_unitary(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 5))
    circ = W.random_circuit(rng, n, 40, W.obs_random_2local(rng, n) if n >= 2 else W.obs_z(n, [0]))
    psi = oracle.statevector(circ)
    u = oracle.unitary(circ)
    assert np.allclose(psi, u[:, 0], atol=1e-12)
    assert abs(np.vdot(psi, psi) - 1) < 1e-12
    assert abs(oracle.expval_sv(circ) - oracle.expval_dense(circ)) < 1e-12


@pytest.mark.parametrize("theta", [0.0, 0.5, 1.9, math.pi, 4.4])
def test_closed_forms(theta):
    """<Z> after RX(t) and RY(t) is cos t, after RZ it is 1; RY(a) then RX(b)
    gives cos a cos b; <X> after RY(t) is sin t."""
    for op, want in ((3, math.cos(theta)), (4, math.cos(theta)), (5, 1.0)):
        c = _one_gate(1, op, 0, theta=theta)
        assert abs(oracle.expval_sv(c) - want) < 1e-14
        assert abs(oracle.propagate(c).expval - want) < 1e-14
    a, b = theta, 0.37
    c = _letters_circ(1, [(4, 0, -1), (3, 0, -1)], [a, b], "Z")
    assert abs(oracle.expval_sv(c) - math.cos(a) * math.cos(b)) < 1e-14
    assert abs(oracle.propagate(c).expval - math.cos(a) * math.cos(b)) < 1e-14
    c = _letters_circ(1, [(4, 0, -1)], [theta], "X")
    assert abs(oracle.expval_sv(c) - math.sin(theta)) < 1e-14
    assert abs(oracle.propagate(c).expval - math.sin(theta)) < 1e-14


def test_product_state_factorizes():
    """Without CX the state is a product; <Z_0 Z_1 Z_2> is the product of the
    single-qubit Bloch z components."""
    rng = np.random.default_rng(3)
    seq, th = [], []
    for q in range(3):
        for op in (3, 4, 5, 3):
            seq.append((op, q, -1))
            th.append(rng.uniform(0, 2 * math.pi))
    circ = _letters_circ(3, seq, th, "ZZZ")
    want = 1.0
    for q in range(3):
        sub = _letters_circ(1, [(op, 0, -1) for op, qq, _ in seq if qq == q],
                            [t for (op, qq, _), t in zip(seq, th) if qq == q], "Z")
        want *= oracle.expval_sv(sub)
    assert abs(oracle.expval_sv(circ) - want) < 1e-13
    assert abs(oracle.propagate(circ).expval - want) < 1e-13


# ------------------------------------------------------- scalar propagation
@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_propagate_full_set_vs_ptm(seed):
    """Every coefficient of the Heisenberg-propagated set, against full Pauli
    transfer matrices 2^-n Tr(Q g^dag P g) (n <= 3)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 4))
    obs = W.obs_random_2local(rng, n) if n >= 2 else W.obs_z(1, [0])
    circ = W.random_circuit(rng, n, 25, obs)
    r = oracle.propagate(circ)
    ev_ptm, vec = oracle.ptm_propagate(circ)
    got = r.as_dict()
    for k, v in vec.items():
        assert abs(got.get(k, 0.0) - v) < 1e-12, (k, got.get(k), v)
    for k in got:
        assert k in vec
    assert abs(r.expval - ev_ptm) < 1e-12


@pytest.mark.parametrize("seed", RNG_SEEDS)
def test_propagate_vs_statevector(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    circ = W.random_circuit(rng, n, 120, W.obs_random_2local(rng, n))
    assert abs(oracle.propagate(circ).expval - oracle.expval_sv(circ)) < 1e-12


def test_propagate_hea_sum_observable():
    circ = W.hea_circuit(7, 4, 3, W.obs_tfim(4))
    assert abs(oracle.propagate(circ).expval - oracle.expval_sv(circ)) < 1e-12


def test_heisenberg_equals_schroedinger_generators():
    """eq. (1)-(2): rho from the forward-evolved generators equals |psi><psi|;
    Tr rho = 1 and Tr rho^2 = 1; and <O> = Tr(rho O) equals the Heisenberg
    result."""
    rng = np.random.default_rng(21)
    for n in (1, 2, 3, 4):
        circ = W.random_circuit(rng, n, 30, W.obs_random_2local(rng, n) if n > 1 else W.obs_z(1, [0]))
        rho = oracle.rho_from_generators(circ)
        psi = oracle.statevector(circ)
        assert np.allclose(rho, np.outer(psi, psi.conj()), atol=1e-12)
        assert abs(np.trace(rho) - 1) < 1e-12
        assert abs(np.trace(rho @ rho) - 1) < 1e-12
        o = oracle.obs_matrix(n, circ.obs_x, circ.obs_z, circ.obs_c)
        assert abs(np.real(np.trace(rho @ o)) - oracle.propagate(circ).expval) < 1e-12


def test_clifford_only_expectations_are_integers():
    rng = np.random.default_rng(5)
    for _ in range(30):
        n = int(rng.integers(1, 6))
        m = 60
        ops = rng.choice([0, 1, 2] if n > 1 else [0, 1], size=m).astype(np.uint8)
        q0 = rng.integers(0, n, size=m).astype(np.int32)
        q1 = np.full(m, -1, np.int32)
        for g in range(m):
            if ops[g] == 2:
                b = int(rng.integers(0, n - 1))
                q1[g] = b + (b >= q0[g])
        obs = W.obs_random_2local(rng, n) if n > 1 else W.obs_z(1, [0])
        circ = W.make_circuit(n, (ops, q0, q1, np.full(m, -1, np.int32)), 0, obs, [])
        r = oracle.propagate(circ)
        assert r.expval in (-1.0, 0.0, 1.0)
        assert len(r.c) == 1 and abs(r.c[0]) == 1.0
        assert abs(r.expval - oracle.expval_sv(circ)) < 1e-12


def _symp(a, b):
    return bin((a[0] & b[1]) ^ (a[1] & b[0])).count("1") & 1


def test_clifford_preserves_commutation():
    rng = np.random.default_rng(8)
    n = 4
    for _ in range(10):
        m = 40
        ops = rng.choice([0, 1, 2], size=m).astype(np.uint8)
        q0 = rng.integers(0, n, size=m).astype(np.int32)
        q1 = np.full(m, -1, np.int32)
        for g in range(m):
            if ops[g] == 2:
                b = int(rng.integers(0, n - 1))
                q1[g] = b + (b >= q0[g])
        paulis = [(int(rng.integers(0, 16)), int(rng.integers(0, 16))) for _ in range(6)]
        images = []
        for x, z in paulis:
            circ = W.make_circuit(n, (ops, q0, q1, np.full(m, -1, np.int32)), 0,
                                  W.observable([(x, z, 1.0)]), [])
            r = oracle.propagate(circ)
            images.append((int(r.x[0]), int(r.z[0])))
        for i in range(6):
            for j in range(6):
                assert _symp(paulis[i], paulis[j]) == _symp(images[i], images[j])


def test_rotation_zero_is_identity_and_half_pi_is_clifford():
    rng = np.random.default_rng(9)
    n = 3
    base = W.random_circuit(rng, n, 30, W.obs_tfim(n))
    for op, equiv in ((5, [1]), (3, [0, 1, 0]), (4, [1, 1, 0])):
        for q in range(n):
            # R(0): same coefficients, missing keys read as zero
            seq0 = W.make_circuit(n, (np.concatenate([base.op, [op]]).astype(np.uint8),
                                      np.concatenate([base.q0, [q]]).astype(np.int32),
                                      np.concatenate([base.q1, [-1]]).astype(np.int32),
                                      np.concatenate([base.param, [base.n_params]]).astype(np.int32)),
                                  base.n_params + 1, (base.obs_x, base.obs_z, base.obs_c),
                                  np.concatenate([base.theta, [0.0]]))
            a = oracle.propagate(seq0).as_dict()
            b = oracle.propagate(base).as_dict()
            for k in set(a) | set(b):
                assert abs(a.get(k, 0.0) - b.get(k, 0.0)) < 1e-13
            # R(pi/2) vs its Clifford equivalent (equal up to a global phase)
            seqh = W.make_circuit(n, (np.concatenate([base.op, [op]]).astype(np.uint8),
                                      np.concatenate([base.q0, [q]]).astype(np.int32),
                                      np.concatenate([base.q1, [-1]]).astype(np.int32),
                                      np.concatenate([base.param, [base.n_params]]).astype(np.int32)),
                                  base.n_params + 1, (base.obs_x, base.obs_z, base.obs_c),
                                  np.concatenate([base.theta, [math.pi / 2]]))
            k = len(equiv)
            seqc = W.make_circuit(n, (np.concatenate([base.op, equiv]).astype(np.uint8),
                                      np.concatenate([base.q0, [q] * k]).astype(np.int32),
                                      np.concatenate([base.q1, [-1] * k]).astype(np.int32),
                                      np.concatenate([base.param, [-1] * k]).astype(np.int32)),
                                  base.n_params, (base.obs_x, base.obs_z, base.obs_c), base.theta)
            assert abs(oracle.propagate(seqh).expval - oracle.propagate(seqc).expval) < 1e-12
            assert abs(oracle.propagate(seqh).expval - oracle.expval_sv(seqh)) < 1e-12


def test_norm_conserved_and_key_set_structural():
    """sum c^2 is conserved by every gate (orthogonal maps) and the key set
    does not depend on theta (no pruning)."""
    rng = np.random.default_rng(10)
    circ = W.random_circuit(rng, 4, 200, W.obs_tfim(4))
    r1 = oracle.propagate(circ)
    assert abs(np.sum(r1.c ** 2) - np.sum(circ.obs_c ** 2)) < 1e-12
    r2 = oracle.propagate(circ.with_theta(rng.uniform(0, 2 * math.pi, circ.n_params)))
    r3 = oracle.propagate(circ.with_theta(np.zeros(circ.n_params)))
    assert np.array_equal(r1.x, r2.x) and np.array_equal(r1.z, r2.z)
    assert np.array_equal(r1.x, r3.x) and np.array_equal(r1.z, r3.z)
    assert r1.updates == r2.updates == r3.updates
    assert len(r1.c) <= 4 ** 4


def test_theta_dependence_is_trigonometric():
    """f(theta_p) = A + B cos theta_p + C sin theta_p, period 2 pi."""
    rng = np.random.default_rng(12)
    circ = W.random_circuit(rng, 4, 80, W.obs_z(4, [0, 1]))
    p = 3
    def f(t):
        th = circ.theta.copy(); th[p] = t
        return oracle.propagate(circ.with_theta(th)).expval
    A = (f(0.0) + f(math.pi)) / 2
    B = (f(0.0) - f(math.pi)) / 2
    C = f(math.pi / 2) - A
    for t in (0.3, 1.7, 4.1):
        assert abs(f(t) - (A + B * math.cos(t) + C * math.sin(t))) < 1e-12
        assert abs(f(t) - f(t + 2 * math.pi)) < 1e-12


def test_updates_count_definition():
    """U = sum over gates of the set size entering the gate: one rotation on an
    anticommuting single string gives U = 1 then the set has 2 strings."""
    c = _letters_circ(1, [(3, 0, -1), (3, 0, -1)], [0.3, 0.4], "Z")
    r = oracle.propagate(c)
    assert r.updates == 1 + 2 and len(r.c) == 2


def test_updates_count_hand_computed_mixed_circuit():
    """U on a circuit that mixes Clifford gates and rotations, worked out by
    hand in Heisenberg order (last gate first), with O = Z on qubit 1 and the
    gates RX_0(a), CX(0->1), H_1, RY_1(b), S_0 in application order:
      S_0 sees {IZ} (1), RY_1 splits it into {IZ, IX} (1 entering),
      H_1 maps it to {IX, IZ} (2), CX maps IZ to ZZ (2), RX_0 splits ZZ into
      {ZZ, YZ} (2 entering): U = 1 + 1 + 2 + 2 + 2 = 8, final set
      {IX: cos b, ZZ: -sin b cos a, YZ: -sin b sin a}, so <O> = -sin b cos a
      (the Bloch vector of qubit 1 after H is (cos a, 0, 0), rotated by b
      about Y).  A counter that skipped the Clifford gates would give 5, one
      that counted the set leaving each gate 10."""
    a, b = 0.7, 1.1
    c = _letters_circ(2, [(3, 0, -1), (2, 0, 1), (0, 1, -1), (4, 1, -1), (1, 0, -1)], [a, b], "IZ")
    r = oracle.propagate(c)
    assert r.updates == 8 and len(r.c) == 3
    want = {(2, 0): math.cos(b), (0, 3): -math.sin(b) * math.cos(a), (1, 3): -math.sin(b) * math.sin(a)}
    got = r.as_dict()
    assert set(got) == set(want)
    for k, v in want.items():
        assert abs(got[k] - v) < 1e-15, (k, got[k], v)
    assert abs(r.expval + math.sin(b) * math.cos(a)) < 1e-15


def test_updates_count_hand_computed_with_merge():
    """Children that land on strings already in the set are merged before the
    next gate counts the set.  n = 1, O = Z, gates RX(a), RZ(c), RY(b):
    RY splits Z into {Z, X} (1 entering), RZ splits X into {X, Y} (2
    entering: {Z, X, Y}), RX splits Z and Y into each other (3 entering), and
    the children merge into the existing Z and Y, so U = 1 + 2 + 3 = 6 with 3
    strings at the end (5 without the merge).  Weights by hand:
      X: -sin b cos c,
      Z: cos b cos a - sin b sin c sin a,
      Y: sin b sin c cos a + cos b sin a."""
    a, cc, b = 0.3, 0.5, 0.9
    c = _letters_circ(1, [(3, 0, -1), (5, 0, -1), (4, 0, -1)], [a, cc, b], "Z")
    r = oracle.propagate(c)
    assert r.updates == 6 and len(r.c) == 3
    want = {(1, 0): -math.sin(b) * math.cos(cc),
            (0, 1): math.cos(b) * math.cos(a) - math.sin(b) * math.sin(cc) * math.sin(a),
            (1, 1): math.sin(b) * math.sin(cc) * math.cos(a) + math.cos(b) * math.sin(a)}
    got = r.as_dict()
    assert set(got) == set(want)
    for k, v in want.items():
        assert abs(got[k] - v) < 1e-15, (k, got[k], v)


# ----------------------------------------------------------------- gradients
def test_psr_and_fd_match_closed_form():
    for t in (0.2, 1.3, 3.0):
        c = _one_gate(1, 4, 0, theta=t)
        assert abs(oracle.psr_gradient(c)[0] + math.sin(t)) < 1e-13
        assert abs(oracle.fd_gradient(c)[0] + math.sin(t)) < 1e-8
    # two rotations sharing one parameter: d/dt cos(2t) = -2 sin(2t)
    gates = (np.array([4, 4], np.uint8), np.array([0, 0], np.int32), np.array([-1, -1], np.int32),
             np.array([0, 0], np.int32))
    c = W.make_circuit(1, gates, 1, W.obs_z(1, [0]), [0.4])
    assert abs(oracle.psr_gradient(c)[0] + 2 * math.sin(0.8)) < 1e-13


def test_psr_matches_fd_random():
    circ = W.hea_circuit(3, 3, 2, W.obs_tfim(3))
    g1 = oracle.psr_gradient(circ)
    g2 = oracle.fd_gradient(circ)
    assert np.max(np.abs(g1 - g2)) < 1e-7
