"""CPU oracle for Pauli propagation -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library; the two meet only in the
seeded inputs of ``paper_2502_10685_amd.workloads`` (which hold no arithmetic of
the method).

Contents (all FP64):
  * ``statevector`` / ``expval_sv``: dense state vector (C), the plain
    definition <0|U^dag O U|0> (Sec. I, Sec. II-A).
  * ``propagate``: scalar Pauli propagation (C), Table I and the CX list of
    Sec. III-C, merge after every gate (Sec. III-B, Examples 3-4, eq. (7)).
  * ``unitary`` / ``expval_dense`` / ``ptm_propagate``: brute force with full
    matrices for a few qubits (textbook linear algebra, used as pins).
  * ``rho_from_generators``: density matrix from the n evolved generators,
    eq. (1) then eq. (2) (read with the product over all n generators).
  * ``psr_gradient`` / ``fd_gradient``: parameter-shift rule (Sec. I) and
    central differences on the state vector.
  * ``string_to_index`` / ``index_to_string`` / ``expand_reduce`` /
    ``flatten_reduce``: the paper's base-4 encoding (Sec. III-B, Example 2,
    Example 3, eq. (7) and Example 4).

Every function here is pinned by tests against values the paper prints, closed
forms, invariants or brute force; see tests/test_oracle_pins.py.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_sv_run.restype = ctypes.c_int
        lib.orc_sv_run.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P]
        lib.orc_sv_expval.restype = ctypes.c_double
        lib.orc_sv_expval.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, P]
        lib.orc_propagate.restype = ctypes.c_double
        lib.orc_propagate.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, ctypes.c_int,
                                      ctypes.c_int64, P, P, P, ctypes.c_int64, P, P, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _gate_arrays(circ):
    op = np.ascontiguousarray(circ.op, dtype=np.uint8)
    q0 = np.ascontiguousarray(circ.q0, dtype=np.int32)
    q1 = np.ascontiguousarray(circ.q1, dtype=np.int32)
    pa = np.ascontiguousarray(circ.param, dtype=np.int32)
    th = np.ascontiguousarray(circ.theta, dtype=np.float64)
    if th.size == 0:
        th = np.zeros(1)
    return op, q0, q1, pa, th


# ------------------------------------------------------------ state vector (C)
def statevector(circ) -> np.ndarray:
    lib = _load()
    op, q0, q1, pa, th = _gate_arrays(circ)
    out = np.zeros(2 * (1 << circ.n), dtype=np.float64)
    rc = lib.orc_sv_run(circ.n, circ.m, _p(op), _p(q0), _p(q1), _p(pa), _p(th), _p(out))
    if rc != 0:
        raise RuntimeError(f"orc_sv_run failed ({rc})")
    return out[0::2] + 1j * out[1::2]


def expval_psi(n, psi, x, z, c) -> float:
    lib = _load()
    buf = np.empty(2 * psi.size, dtype=np.float64)
    buf[0::2] = psi.real
    buf[1::2] = psi.imag
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return float(lib.orc_sv_expval(n, _p(buf), x.size, _p(x), _p(z), _p(c)))


def expval_sv(circ) -> float:
    return expval_psi(circ.n, statevector(circ), circ.obs_x, circ.obs_z, circ.obs_c)


# ------------------------------------------------------- Pauli propagation (C)
class PropResult:
    def __init__(self, expval, x, z, c, updates):
        self.expval = expval
        self.x, self.z, self.c = x, z, c
        self.updates = updates

    def as_dict(self):
        return {(int(a), int(b)): float(v) for a, b, v in zip(self.x, self.z, self.c)}


def propagate(circ, direction: int = 0, x=None, z=None, c=None, cap=None) -> PropResult:
    """direction 0 = Heisenberg (observable, g_m first); 1 = Schroedinger."""
    lib = _load()
    op, q0, q1, pa, th = _gate_arrays(circ)
    x = np.ascontiguousarray(circ.obs_x if x is None else x, dtype=np.uint64)
    z = np.ascontiguousarray(circ.obs_z if z is None else z, dtype=np.uint64)
    c = np.ascontiguousarray(circ.obs_c if c is None else c, dtype=np.float64)
    if cap is None:
        cap = min(4 ** circ.n, 1 << 24)
    xo = np.zeros(cap, dtype=np.uint64)
    zo = np.zeros(cap, dtype=np.uint64)
    co = np.zeros(cap, dtype=np.float64)
    nout = np.zeros(1, dtype=np.int64)
    upd = np.zeros(1, dtype=np.int64)
    ev = lib.orc_propagate(circ.n, circ.m, _p(op), _p(q0), _p(q1), _p(pa), _p(th), direction,
                           x.size, _p(x), _p(z), _p(c), cap, _p(xo), _p(zo), _p(co),
                           _p(nout), _p(upd))
    k = int(nout[0])
    if k < 0:
        raise MemoryError("oracle propagation ran out of memory")
    if k > cap:
        raise ValueError(f"output capacity {cap} < {k}")
    return PropResult(float(ev), xo[:k].copy(), zo[:k].copy(), co[:k].copy(), int(upd[0]))


# ------------------------------------------------- dense-matrix brute force
_I2 = np.eye(2, dtype=complex)
_X2 = np.array([[0, 1], [1, 0]], dtype=complex)
_Y2 = np.array([[0, -1j], [1j, 0]], dtype=complex)
_Z2 = np.array([[1, 0], [0, -1]], dtype=complex)


def pauli_matrix(n, x, z) -> np.ndarray:
    """Full 2^n matrix of P(x, z); qubit q is bit q of the basis index."""
    m = np.ones((1, 1), dtype=complex)
    for q in range(n - 1, -1, -1):
        xb, zb = (int(x) >> q) & 1, (int(z) >> q) & 1
        p = _I2 if not xb and not zb else _X2 if xb and not zb else _Y2 if xb else _Z2
        m = np.kron(m, p)
    return m


def _one_qubit(op, th):
    c, s = math.cos(th / 2), math.sin(th / 2)
    if op == 0:
        return np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2)
    if op == 1:
        return np.array([[1, 0], [0, 1j]], dtype=complex)
    if op == 3:
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=complex)
    if op == 4:
        return np.array([[c, -s], [s, c]], dtype=complex)
    return np.array([[np.exp(-0.5j * th), 0], [0, np.exp(0.5j * th)]], dtype=complex)


def gate_unitary(n, op, q0, q1, th) -> np.ndarray:
    dim = 1 << n
    if op == 2:
        u = np.zeros((dim, dim), dtype=complex)
        for b in range(dim):
            bb = b ^ (1 << q1) if (b >> q0) & 1 else b
            u[bb, b] = 1
        return u
    m = np.ones((1, 1), dtype=complex)
    for q in range(n - 1, -1, -1):
        m = np.kron(m, _one_qubit(op, th) if q == q0 else _I2)
    return m


def _gate_theta(circ, g):
    return float(circ.theta[circ.param[g]]) if circ.op[g] >= 3 else 0.0


def unitary(circ) -> np.ndarray:
    u = np.eye(1 << circ.n, dtype=complex)
    for g in range(circ.m):
        u = gate_unitary(circ.n, int(circ.op[g]), int(circ.q0[g]), int(circ.q1[g]),
                         _gate_theta(circ, g)) @ u
    return u


def obs_matrix(n, x, z, c) -> np.ndarray:
    o = np.zeros((1 << n, 1 << n), dtype=complex)
    for a, b, v in zip(x, z, c):
        o += float(v) * pauli_matrix(n, a, b)
    return o


def expval_dense(circ) -> float:
    u = unitary(circ)
    psi = u[:, 0]
    o = obs_matrix(circ.n, circ.obs_x, circ.obs_z, circ.obs_c)
    return float(np.real(np.vdot(psi, o @ psi)))


def ptm_propagate(circ):
    """Heisenberg propagation with full Pauli transfer matrices (n <= 3):
    R_g[Q, P] = 2^-n Tr(Q g^dag P g).  Returns (expval, {(x, z): coeff})."""
    n = circ.n
    keys = [(x, z) for z in range(1 << n) for x in range(1 << n)]
    mats = [pauli_matrix(n, x, z) for x, z in keys]
    vec = np.zeros(len(keys))
    for a, b, v in zip(circ.obs_x, circ.obs_z, circ.obs_c):
        vec[keys.index((int(a), int(b)))] += float(v)
    for g in range(circ.m - 1, -1, -1):
        u = gate_unitary(n, int(circ.op[g]), int(circ.q0[g]), int(circ.q1[g]), _gate_theta(circ, g))
        R = np.zeros((len(keys), len(keys)))
        for j, P in enumerate(mats):
            img = u.conj().T @ P @ u
            for i, Q in enumerate(mats):
                R[i, j] = np.real(np.trace(Q @ img)) / (1 << n)
        vec = R @ vec
    ev = sum(vec[i] for i, (x, z) in enumerate(keys) if x == 0)
    return float(ev), {k: float(v) for k, v in zip(keys, vec)}


def rho_from_generators(circ) -> np.ndarray:
    """eq. (1) then eq. (2): evolve Z_j forward through the circuit and form
    rho = 2^-n prod_j (I + P_j) over all n generators."""
    n = circ.n
    rho = np.eye(1 << n, dtype=complex)
    for j in range(n):
        r = propagate(circ, direction=1, x=np.zeros(1, np.uint64),
                      z=np.array([1 << j], np.uint64), c=np.ones(1))
        pj = obs_matrix(n, r.x, r.z, r.c)
        rho = rho @ (np.eye(1 << n) + pj)
    return rho / (1 << n)


# -------------------------------------------------------------- gradients
def _with_shift(circ, g, delta):
    th = np.concatenate([circ.theta, [circ.theta[circ.param[g]] + delta]])
    pa = circ.param.copy()
    pa[g] = len(circ.theta)
    c2 = circ.with_theta(circ.theta)
    c2.theta = th
    c2.param = pa
    return c2


def psr_gradient(circ, expval=expval_sv) -> np.ndarray:
    """Parameter-shift rule (Sec. I): d<O>/d theta_g = [f(+pi/2) - f(-pi/2)] / 2
    per rotation gate, summed into its parameter."""
    grad = np.zeros(circ.n_params)
    for g in range(circ.m):
        if circ.op[g] < 3:
            continue
        fp = expval(_with_shift(circ, g, math.pi / 2))
        fm = expval(_with_shift(circ, g, -math.pi / 2))
        grad[circ.param[g]] += 0.5 * (fp - fm)
    return grad


def fd_gradient(circ, h=1e-6, expval=expval_sv) -> np.ndarray:
    grad = np.zeros(circ.n_params)
    for p in range(circ.n_params):
        tp = circ.theta.copy(); tp[p] += h
        tm = circ.theta.copy(); tm[p] -= h
        grad[p] = (expval(circ.with_theta(tp)) - expval(circ.with_theta(tm))) / (2 * h)
    return grad


# ------------------------------------------------- the paper's base-4 encoding
_LETTER_DIGIT = {"I": 0, "X": 1, "Y": 2, "Z": 3}
_DIGIT_LETTER = "IXYZ"


def string_to_index(s: str) -> int:
    """Sec. III-B: base-4 digits I=0 X=1 Y=2 Z=3, qubit 0 most significant."""
    idx = 0
    for ch in s:
        idx = idx * 4 + _LETTER_DIGIT[ch]
    return idx


def index_to_string(idx: int, n: int) -> str:
    out = []
    for _ in range(n):
        out.append(_DIGIT_LETTER[idx % 4])
        idx //= 4
    return "".join(reversed(out))


def expand_reduce(weights) -> np.ndarray:
    """weights: n' x n x 4 (one weight vector per qubit per product).  Each
    product of sums is expanded by the Kronecker product over qubits (qubit 0
    most significant) and the products are summed: lambda in R^{4^n}."""
    w = np.asarray(weights, dtype=np.float64)
    lam = np.zeros(4 ** w.shape[1])
    for row in w:
        k = np.ones(1)
        for q in range(w.shape[1]):
            k = np.kron(k, row[q])
        lam += k
    return lam


def flatten(weights) -> np.ndarray:
    """eq. (7) before the reduction: one row of 4^n products per term."""
    w = np.asarray(weights, dtype=np.float64)
    rows = []
    for row in w:
        k = np.ones(1)
        for q in range(w.shape[1]):
            k = np.kron(k, row[q])
        rows.append(k)
    return np.array(rows)


def flatten_reduce(weights) -> np.ndarray:
    return flatten(weights).sum(axis=0)


def symplectic_to_string(n, x, z) -> str:
    s = []
    for q in range(n):
        xb, zb = (int(x) >> q) & 1, (int(z) >> q) & 1
        s.append("I" if not xb and not zb else "X" if not zb else "Y" if xb else "Z")
    return "".join(s)
