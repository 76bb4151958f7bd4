"""Seeded synthetic workloads: circuits, angles and observables.

This module only draws random numbers and lays out gate lists; it holds none
of the propagation arithmetic.  Both the CPU oracle (through the tests) and the
GPU path consume what it produces, so the two never disagree about inputs.

Gate encoding (shared by every consumer):
    op     uint8   0=H 1=S 2=CX 3=RX 4=RY 5=RZ
    q0     int32   acted-on qubit (control for CX)
    q1     int32   target qubit for CX, -1 otherwise
    param  int32   index into theta for rotations, -1 for Clifford gates
Rotation convention: R_sigma(theta) = exp(-i theta sigma / 2).  Gates are
listed in application order g_1 ... g_m (g_1 acts first on |0...0>).

Observables are weighted Pauli strings in symplectic form: bit q of x/z is
qubit q, with I=(0,0) X=(1,0) Y=(1,1) Z=(0,1) and Y Hermitian.

The paper's workloads are parameterized circuits on a few qubits with many
gates (Sec. I, Sec. V); the generators below reproduce those shapes with
seeded numpy PCG64 streams.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

H, S, CX, RX, RY, RZ = 0, 1, 2, 3, 4, 5
OP_NAMES = {H: "H", S: "S", CX: "CX", RX: "RX", RY: "RY", RZ: "RZ"}
ROTATIONS = (RX, RY, RZ)
TWO_PI = 2.0 * math.pi


@dataclass
class Circuit:
    """A gate list plus parameters and an observable (all host numpy)."""

    n: int
    op: np.ndarray
    q0: np.ndarray
    q1: np.ndarray
    param: np.ndarray
    theta: np.ndarray
    obs_x: np.ndarray
    obs_z: np.ndarray
    obs_c: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.op.shape[0])

    @property
    def n_params(self) -> int:
        return int(self.theta.shape[0])

    def with_theta(self, theta) -> "Circuit":
        theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        assert theta.shape == self.theta.shape
        return Circuit(self.n, self.op, self.q0, self.q1, self.param, theta,
                       self.obs_x, self.obs_z, self.obs_c, self.name, dict(self.meta))


def _arrays(ops, q0s, q1s, params):
    return (np.ascontiguousarray(np.asarray(ops, dtype=np.uint8)),
            np.ascontiguousarray(np.asarray(q0s, dtype=np.int32)),
            np.ascontiguousarray(np.asarray(q1s, dtype=np.int32)),
            np.ascontiguousarray(np.asarray(params, dtype=np.int32)))


# ----------------------------------------------------------------- observables
def pauli_from_string(s: str, coeff: float = 1.0):
    """'XIZ' (qubit 0 leftmost) -> (x, z, c) symplectic words."""
    x = z = 0
    for q, ch in enumerate(s):
        if ch == "X":
            x |= 1 << q
        elif ch == "Z":
            z |= 1 << q
        elif ch == "Y":
            x |= 1 << q
            z |= 1 << q
        elif ch != "I":
            raise ValueError(ch)
    return x, z, coeff


def observable(terms):
    """[(x, z, c), ...] -> three contiguous arrays."""
    xs = np.array([t[0] for t in terms], dtype=np.uint64)
    zs = np.array([t[1] for t in terms], dtype=np.uint64)
    cs = np.array([t[2] for t in terms], dtype=np.float64)
    return xs, zs, cs


def obs_z(n, qubits):
    z = 0
    for q in qubits:
        z |= 1 << q
    return observable([(0, z, 1.0)])


def obs_sum_z(n):
    return observable([(0, 1 << i, 1.0) for i in range(n)])


def obs_tfim(n, J=1.0, h=1.0):
    """Open-chain transverse-field Ising: sum Z_i Z_{i+1} + sum X_i."""
    terms = [(0, (1 << i) | (1 << (i + 1)), J) for i in range(n - 1)]
    terms += [(1 << i, 0, h) for i in range(n)]
    return observable(terms)


def obs_random_2local(rng, n):
    a, b = rng.choice(n, size=2, replace=False)
    x = z = 0
    for q in (int(a), int(b)):
        letter = int(rng.integers(1, 4))  # 1=X 2=Y 3=Z
        if letter in (1, 2):
            x |= 1 << q
        if letter in (2, 3):
            z |= 1 << q
    return observable([(x, z, 1.0)])


# -------------------------------------------------------------------- circuits
def hea_gates(n: int, layers: int):
    """Hardware-efficient ansatz: per layer RX,RY,RZ on each qubit (qubit-major)
    then a CX ring 0->1, 1->2, ..., (n-1)->0.  theta index = 3n*layer+3q+k."""
    ops, q0s, q1s, params = [], [], [], []
    for layer in range(layers):
        for q in range(n):
            for k, g in enumerate((RX, RY, RZ)):
                ops.append(g)
                q0s.append(q)
                q1s.append(-1)
                params.append(3 * n * layer + 3 * q + k)
        if n >= 2:
            for q in range(n):
                ops.append(CX)
                q0s.append(q)
                q1s.append((q + 1) % n)
                params.append(-1)
    return _arrays(ops, q0s, q1s, params), 3 * n * layers


def random_gates(rng: np.random.Generator, n: int, m: int):
    """m gates, each a Clifford (H, S, CX uniform) or a rotation (axis, qubit
    uniform) with probability 1/2; every rotation gets its own parameter."""
    ops = np.empty(m, dtype=np.uint8)
    q0 = np.empty(m, dtype=np.int32)
    q1 = np.full(m, -1, dtype=np.int32)
    param = np.full(m, -1, dtype=np.int32)
    is_rot = rng.random(m) < 0.5
    kind = rng.integers(0, 3, size=m)
    qa = rng.integers(0, n, size=m)
    qb = rng.integers(0, max(n - 1, 1), size=m)
    p = 0
    for g in range(m):
        if is_rot[g]:
            ops[g] = RX + kind[g]
            q0[g] = qa[g]
            param[g] = p
            p += 1
        else:
            c = kind[g]
            if c == 2 and n >= 2:
                a = int(qa[g])
                b = int(qb[g])
                if b >= a:
                    b += 1
                ops[g] = CX
                q0[g] = a
                q1[g] = b
            else:
                ops[g] = H if c == 0 else (S if c == 1 else H)
                q0[g] = qa[g]
    return (ops, q0, q1, param), p


def log_uniform_int(rng, lo, hi):
    return int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def make_circuit(n, gates, n_params, obs, theta, name="", meta=None):
    ops, q0, q1, param = gates
    x, z, c = obs
    return Circuit(n, ops, q0, q1, param,
                   np.ascontiguousarray(np.asarray(theta, dtype=np.float64)),
                   np.ascontiguousarray(x), np.ascontiguousarray(z),
                   np.ascontiguousarray(c), name, meta or {})


def random_circuit(seed_or_rng, n, m, obs=None, name="random"):
    rng = np.random.default_rng(seed_or_rng) if not isinstance(
        seed_or_rng, np.random.Generator) else seed_or_rng
    gates, p = random_gates(rng, n, m)
    theta = rng.uniform(0.0, TWO_PI, size=p)
    if obs is None:
        obs = obs_z(n, [0])
    return make_circuit(n, gates, p, obs, theta, name)


def hea_circuit(seed, n, layers, obs=None, name="hea"):
    rng = np.random.default_rng(seed)
    gates, p = hea_gates(n, layers)
    theta = rng.uniform(0.0, TWO_PI, size=p)
    if obs is None:
        obs = obs_z(n, [0])
    return make_circuit(n, gates, p, obs, theta, name)


def chain_zxz_gates(n: int, layers: int, repeats: int):
    """The shape of the paper's timing ansatz (Sec. V): per layer a CX chain
    closed into a ring 0->1, ..., (n-1)->0 (the topology drawing is not
    available; a ring of n CX gives the stated 60.2K gates at n = 4, 50
    layers, 100 repeats), then `repeats` blocks of RZ, RX, RZ on every qubit,
    each rotation with its own parameter."""
    ops, q0s, q1s, params = [], [], [], []
    p = 0
    for _ in range(layers):
        if n >= 2:
            for q in range(n):
                ops.append(CX)
                q0s.append(q)
                q1s.append((q + 1) % n)
                params.append(-1)
        for _ in range(repeats):
            for q in range(n):
                for g in (RZ, RX, RZ):
                    ops.append(g)
                    q0s.append(q)
                    q1s.append(-1)
                    params.append(p)
                    p += 1
    return (np.array(ops, np.uint8), np.array(q0s, np.int32), np.array(q1s, np.int32),
            np.array(params, np.int32)), p


def chain_zxz_circuit(seed=6, n=4, layers=50, repeats=100):
    """n = 4, 50 layers x (4 CX + 100 x 12 rotations) = 60,200 gates, O = Z_0."""
    rng = np.random.default_rng(seed)
    gates, p = chain_zxz_gates(n, layers, repeats)
    theta = rng.uniform(0.0, TWO_PI, size=p)
    return make_circuit(n, gates, p, obs_z(n, [0]), theta, name=f"chainzxz{n}x{layers}x{repeats}")


def spread_circuit(seed, n, k):
    """A circuit whose Heisenberg string set has a known size, for sets of
    millions of strings.  In application order: H on every even qubit, S on
    every qubit divisible by 3, a CX chain 0->1, ..., (n-2)->(n-1); then RY on
    qubits 0..k-1; then RX on every qubit.  O = Z^n.

    Propagated backward, the RX layer turns Z^n into all 2^n strings over
    {Z, Y}; each RY sends Z to {Z, X} and keeps Y, giving 2^(n-k) 3^k strings;
    the Clifford prefix maps strings one to one.  meta["final_terms"] holds
    that count."""
    rng = np.random.default_rng(seed)
    ops, q0s, q1s, params = [], [], [], []
    for q in range(0, n, 2):
        ops.append(H); q0s.append(q); q1s.append(-1); params.append(-1)
    for q in range(0, n, 3):
        ops.append(S); q0s.append(q); q1s.append(-1); params.append(-1)
    for q in range(n - 1):
        ops.append(CX); q0s.append(q); q1s.append(q + 1); params.append(-1)
    p = 0
    for q in range(k):
        ops.append(RY); q0s.append(q); q1s.append(-1); params.append(p)
        p += 1
    for q in range(n):
        ops.append(RX); q0s.append(q); q1s.append(-1); params.append(p)
        p += 1
    theta = rng.uniform(0.0, TWO_PI, size=p)
    obs = observable([(0, (1 << n) - 1, 1.0)])
    return make_circuit(n, _arrays(ops, q0s, q1s, params), p, obs, theta, name=f"spread{n}k{k}",
                        meta={"final_terms": (2 ** (n - k)) * (3 ** k)})


# ---------------------------------------------------------- the five workloads
def config1(seed=1):
    """n=4, HEA-10 (160 gates), O = Z_0, FP64."""
    return hea_circuit(seed, 4, 10, obs_z(4, [0]), name="hea4x10_Z0")


def config2(seed=2, m=60000):
    """n=6, 60,000 random gates, O = sum_i Z_i."""
    return random_circuit(seed, 6, m, obs_sum_z(6), name="rand6x60000_sumZ")


def config3(seed=3, count=512, n_lo=4, n_hi=10, m_lo=1000, m_hi=20000):
    """512 uneven circuits, n ~ U{4..10}, m log-uniform in [1k, 20k], O = Z0 Z1."""
    ss = np.random.SeedSequence(seed)
    out = []
    for i, child in enumerate(ss.spawn(count)):
        rng = np.random.default_rng(child)
        n = int(rng.integers(n_lo, n_hi + 1))
        m = log_uniform_int(rng, m_lo, m_hi)
        out.append(random_circuit(rng, n, m, obs_z(n, [0, 1]), name=f"batch{i}_n{n}_m{m}"))
    return out


def config4(seed=4, n=8, layers=40):
    """n=8, HEA-40 (1,280 gates, 960 parameters), TFIM observable."""
    return hea_circuit(seed, n, layers, obs_tfim(n), name="hea8x40_tfim")


def config5_requests(seed=5, lam=100.0, count=256, n_lo=4, n_hi=12, m_lo=1000, m_hi=60000):
    """Poisson arrivals (rate lam per second) of random circuits."""
    ss = np.random.SeedSequence([seed, int(lam)])
    arr_rng = np.random.default_rng(ss.spawn(1)[0])
    gaps = arr_rng.exponential(1.0 / lam, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i, child in enumerate(ss.spawn(count + 1)[1:]):
        rng = np.random.default_rng(child)
        n = int(rng.integers(n_lo, n_hi + 1))
        m = log_uniform_int(rng, m_lo, m_hi)
        obs = obs_z(n, [0]) if rng.random() < 0.5 else obs_random_2local(rng, n)
        reqs.append((float(arrivals[i]), random_circuit(rng, n, m, obs, name=f"req{i}_n{n}_m{m}")))
    return reqs
