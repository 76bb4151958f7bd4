"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (FP64): string sets bit-identical, every weight and <O> within 1e-12
absolute, term-update counts equal; FP32 storage within 1e-5 absolute.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

_CFG3 = []


def _config3():
    if not _CFG3:
        _CFG3.extend(W.config3())
    return _CFG3

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


def _check_set(c, want, tol=TOL64, check_updates=True):
    x, z, v = c.terms()
    assert len(x) == len(want.x), (len(x), len(want.x))
    assert np.array_equal(x, want.x) and np.array_equal(z, want.z), "string sets differ"
    err = float(np.max(np.abs(v - want.c))) if len(v) else 0.0
    assert err <= tol, err
    if check_updates:
        assert c.stats()["term_updates"] == want.updates
    return err


def _run(api, wc, **kw):
    c = api.Circuit.from_workload(wc, **kw)
    ev = float(c.evaluate().item())
    return c, ev


# ----------------------------------------------------------------- config 1
@pytest.mark.parametrize("engine", ["dense", "sparse"])
def test_config1_hea4(api, engine):
    wc = W.config1()
    _say(f"config1 engine={engine}")
    want = oracle.propagate(wc)
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc, engine=engine, track=True)
    assert abs(ev - want.expval) <= TOL64 and abs(ev - sv) <= TOL64
    _check_set(c, want)
    assert len(want.x) == 255
    c2, ev2 = _run(api, wc, engine=engine)
    assert abs(ev2 - want.expval) <= TOL64


# ------------------------------------------------- random circuits, n = 1..7
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("engine", ["dense", "sparse"])
def test_random_resident_sizes(api, n, engine):
    rng = np.random.default_rng(1000 + n)
    m = 400 if n <= 5 else 250
    obs = W.obs_random_2local(rng, n) if n >= 2 else W.obs_z(1, [0])
    wc = W.random_circuit(rng, n, m, obs)
    _say(f"random n={n} m={m} engine={engine}")
    want = oracle.propagate(wc)
    for track in (True, False):
        c, ev = _run(api, wc, engine=engine, track=track)
        assert abs(ev - want.expval) <= TOL64, (track, ev, want.expval)
        if track or engine == "sparse":
            _check_set(c, want)
        c.close()


@pytest.mark.parametrize("n,k", [(8, 5), (8, 4), (9, 5), (9, 6)])
def test_tiled_dense_vs_oracle(api, n, k):
    rng = np.random.default_rng(2000 + 10 * n + k)
    wc = W.random_circuit(rng, n, 160, W.obs_tfim(n))
    _say(f"tiled n={n} k={k}")
    want = oracle.propagate(wc)
    for track in (True, False):
        c, ev = _run(api, wc, engine="dense", track=track, tile_qubits=k)
        assert abs(ev - want.expval) <= TOL64
        st = c.stats()
        assert st["tile_qubits"] == k and st["passes"] >= 2
        if track:
            _check_set(c, want)
        c.close()


@pytest.mark.parametrize("k", [5, 6, 7])
def test_tiled_dense_n11(api, k):
    """n = 11 (4^11 slots, past the batch workload's n <= 10): 2,500 random
    gates against the FP64 state vector for every tile size, solo and
    batched with smaller circuits; the last 175 gates, tracked, against the
    scalar propagator string for string (tens of thousands to half a million
    strings)."""
    rng = np.random.default_rng(1100 + k)
    wc = W.random_circuit(rng, 11, 2500, W.obs_random_2local(rng, 11))
    _say(f"tiled n=11 k={k} m={wc.m}")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc, engine="dense", tile_qubits=k)
    st = c.stats()
    assert st["tile_qubits"] == k and st["passes"] >= 2
    assert abs(ev - sv) <= TOL64, (ev, sv)
    others = [W.random_circuit(rng, n, 700, W.obs_z(n, [0, 1])) for n in (8, 10, 11)]
    cs = [c] + [api.Circuit.from_workload(w, tile_qubits=k) for w in others]
    out = api.evaluate_batch(cs).cpu().numpy()
    assert out[0] == ev
    for w, v in zip(others, out[1:]):
        assert abs(v - oracle.expval_sv(w)) <= TOL64
    pre = W.make_circuit(11, (wc.op[-175:], wc.q0[-175:], wc.q1[-175:], wc.param[-175:]), wc.n_params,
                         (wc.obs_x, wc.obs_z, wc.obs_c), wc.theta)
    want = oracle.propagate(pre)
    ct, evt = _run(api, pre, engine="dense", track=True, tile_qubits=k)
    assert abs(evt - want.expval) <= TOL64
    _check_set(ct, want)
    for o in cs + [ct]:
        o.close()


def test_sparse_n8_ragged(api):
    rng = np.random.default_rng(77)
    wc = W.random_circuit(rng, 8, 120, W.obs_z(8, [0, 3]))
    _say("sparse n=8")
    want = oracle.propagate(wc)
    c, ev = _run(api, wc, engine="sparse")
    assert abs(ev - want.expval) <= TOL64
    _check_set(c, want)
    assert len(want.x) % 2048 != 0


def test_sparse_beyond_dense_range(api):
    """n = 20: the dense engine cannot hold 4^n slots; a shallow circuit keeps
    the set small and the sparse engine runs it (state-vector check)."""
    rng = np.random.default_rng(5)
    n = 20
    wc = W.random_circuit(rng, n, 60, W.obs_z(n, [0, 1]))
    _say("sparse n=20")
    want_sv = oracle.expval_sv(wc)
    want = oracle.propagate(wc, cap=1 << 16)
    c, ev = _run(api, wc, engine="auto", max_terms=1 << 16)
    assert c.stats()["engine"] == 2
    assert abs(ev - want_sv) <= TOL64 and abs(ev - want.expval) <= TOL64
    x, z, v = c.terms(capacity=1 << 16)
    assert np.array_equal(x, want.x) and np.array_equal(z, want.z)
    assert np.max(np.abs(v - want.c)) <= TOL64


# ------------------------------------------------------------- full sizes
def test_config2_full_size_fp64(api):
    wc = W.config2()
    _say("config2 fp64 full size")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc, engine="dense")
    assert abs(ev - sv) <= TOL64, (ev, sv)


def test_config2_full_size_fp32(api):
    wc = W.config2()
    _say("config2 fp32 full size")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc, engine="dense", dtype="f32")
    err = abs(ev - sv)
    _say(f"config2 fp32 |err| = {err:.3e}")
    assert err <= TOL32, err


def test_config2_prefix_sets_match(api):
    """The first 3,000 gates of config 2: whole string set and U."""
    full = W.config2()
    m = 3000
    wc = W.make_circuit(full.n, (full.op[:m], full.q0[:m], full.q1[:m], full.param[:m]), full.n_params,
                        (full.obs_x, full.obs_z, full.obs_c), full.theta)
    _say("config2 prefix 3000")
    want = oracle.propagate(wc)
    c, ev = _run(api, wc, engine="dense", track=True)
    assert abs(ev - want.expval) <= TOL64
    _check_set(c, want)


def test_config4_hea8(api):
    wc = W.config4()
    _say("config4 n=8 HEA-40 TFIM")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc, engine="dense")
    assert abs(ev - sv) <= TOL64
    c, ev = _run(api, wc, engine="dense", track=True)
    assert abs(ev - sv) <= TOL64
    st = c.stats()
    assert st["term_updates"] == 80086509 and st["final_terms"] == 65535


@pytest.mark.parametrize("idx", [0, 5, 17, 101, 260, 511])
def test_config3_sampled_circuits(api, idx):
    wc = _config3()[idx]
    _say(f"config3 circuit {idx} n={wc.n} m={wc.m}")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc)
    assert abs(ev - sv) <= TOL64, (ev, sv)


@pytest.mark.parametrize("dtype,tol", [("f64", TOL64), ("f32", TOL32)])
def test_config3_full_batch_every_output(api, dtype, tol):
    """The 512-circuit batch in the launch configuration the benchmark times
    (one pp_evaluate_batch, default kernels): every output against the
    oracle's state vector."""
    import torch
    circs = _config3()
    _say(f"config3 full batch {dtype}")
    objs = [api.Circuit.from_workload(w, dtype=dtype) for w in circs]
    out = api.evaluate_batch(objs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = np.array([oracle.expval_sv(w) for w in circs])
    err = np.abs(got - want)
    assert float(err.max()) <= tol, (int(err.argmax()), float(err.max()))
    for o in objs:
        o.close()


def test_n12_sampled(api):
    rng = np.random.default_rng(12)
    wc = W.random_circuit(rng, 12, 1500, W.obs_z(12, [0]))
    _say("n=12 m=1500")
    sv = oracle.expval_sv(wc)
    c, ev = _run(api, wc)
    assert abs(ev - sv) <= TOL64, (ev, sv)


# ----------------------------------------------------------------- batching
def test_batch_equals_solo_bitwise(api):
    import torch
    circs = W.config3(count=24, m_lo=200, m_hi=1500)
    _say("batch of 24")
    objs = [api.Circuit.from_workload(w) for w in circs]
    solo = [float(o.evaluate().item()) for o in objs]
    out = api.evaluate_batch(objs)
    torch.cuda.synchronize()
    got = out.cpu().numpy().tolist()
    assert got == solo
    out2 = api.evaluate_batch(objs)  # cached descriptors
    assert out2.cpu().numpy().tolist() == solo
    for w, v in zip(circs[:6], solo):
        assert abs(v - oracle.expval_sv(w)) <= TOL64


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_full_batch_equals_solo_bitwise(api, dtype):
    """The 512-circuit batch: its launches walk several rounds of tiles per
    workgroup (next-tile prefetch, half of it in FP64; circuits ordered by
    their pass's op count), while one circuit at a time fits one round.
    Every output must be identical bit for bit."""
    import torch
    circs = _config3()
    _say(f"config3 batch vs solo {dtype}")
    objs = [api.Circuit.from_workload(w, dtype=dtype) for w in circs]
    out = api.evaluate_batch(objs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    solo = np.array([float(o.evaluate().item()) for o in objs])
    assert np.array_equal(got.view(np.uint64), solo.view(np.uint64)), int(np.argmax(got != solo))
    for o in objs:
        o.close()


# ---------------------------------------------------------------- edge cases
def test_empty_circuit_and_clifford_only(api):
    wc = W.make_circuit(3, (np.zeros(0, np.uint8), np.zeros(0, np.int32), np.zeros(0, np.int32),
                            np.zeros(0, np.int32)), 0, W.obs_tfim(3), [])
    c, ev = _run(api, wc, track=True)
    assert ev == 0.0 + 2.0  # Z0Z1 + Z1Z2 on |000> = 2, X terms 0
    rng = np.random.default_rng(3)
    for eng in ("dense", "sparse"):
        for _ in range(5):
            n = 5
            m = 80
            ops = rng.choice([0, 1, 2], size=m).astype(np.uint8)
            q0 = rng.integers(0, n, size=m).astype(np.int32)
            q1 = np.full(m, -1, np.int32)
            for g in range(m):
                if ops[g] == 2:
                    b = int(rng.integers(0, n - 1))
                    q1[g] = b + (b >= q0[g])
            wc = W.make_circuit(n, (ops, q0, q1, np.full(m, -1, np.int32)), 0,
                                W.obs_random_2local(rng, n), [])
            c, ev = _run(api, wc, engine=eng, track=True)
            want = oracle.propagate(wc)
            assert ev == want.expval and ev in (-1.0, 0.0, 1.0)
            x, z, v = c.terms()
            assert np.array_equal(v, want.c)


def test_rotation_zero_and_theta_reuse(api):
    import torch
    rng = np.random.default_rng(8)
    wc = W.random_circuit(rng, 5, 300, W.obs_tfim(5))
    c = api.Circuit.from_workload(wc, track=True)
    for th in (wc.theta, np.zeros(wc.n_params), rng.uniform(0, 2 * math.pi, wc.n_params)):
        w2 = wc.with_theta(th)
        c.set_theta(torch.tensor(th, device="cuda"))
        ev = float(c.evaluate().item())
        want = oracle.propagate(w2)
        assert abs(ev - want.expval) <= TOL64
        _check_set(c, want)


def test_graph_replay_matches_eager(api):
    import torch
    rng = np.random.default_rng(9)
    wc = W.random_circuit(rng, 9, 400, W.obs_z(9, [0, 1]))
    eager = api.Circuit.from_workload(wc, engine="dense", tile_qubits=5)
    graph = api.Circuit.from_workload(wc, engine="dense", tile_qubits=5, use_graph=True)
    for r in range(4):
        th = rng.uniform(0, 2 * math.pi, wc.n_params)
        eager.set_theta(th)
        graph.set_theta(th)
        a = float(eager.evaluate().item())
        b = float(graph.evaluate().item())
        torch.cuda.synchronize()
        assert a == b, (r, a, b)
        assert abs(a - oracle.expval_sv(wc.with_theta(th))) <= TOL64


def test_sparse_capacity_overflow_is_reported(api):
    rng = np.random.default_rng(10)
    wc = W.random_circuit(rng, 6, 200, W.obs_z(6, [0]))
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=64)
    ev = float(c.evaluate().item())
    assert math.isnan(ev)
    assert c.stats()["overflow"] == 1
    from paper_2502_10685_amd._lib import PauliPropError
    with pytest.raises(PauliPropError):
        c.terms()


def test_invalid_inputs(api):
    from paper_2502_10685_amd._lib import PauliPropError
    wc = W.config1()
    bad_q = wc.q0.copy()
    bad_q[3] = 9
    with pytest.raises(PauliPropError):
        api.Circuit(wc.n, wc.op, bad_q, wc.q1, wc.param, wc.n_params, wc.obs_x, wc.obs_z, wc.obs_c)
    bad_p = wc.param.copy()
    bad_p[0] = wc.n_params
    with pytest.raises(PauliPropError):
        api.Circuit(wc.n, wc.op, wc.q0, wc.q1, bad_p, wc.n_params, wc.obs_x, wc.obs_z, wc.obs_c)
    with pytest.raises(PauliPropError):
        api.Circuit(wc.n, wc.op, wc.q0, wc.q1, wc.param, wc.n_params, np.array([1 << 5], np.uint64),
                    np.array([0], np.uint64), np.array([1.0]))
    c = api.Circuit(wc.n, wc.op, wc.q0, wc.q1, wc.param, wc.n_params, wc.obs_x, wc.obs_z, wc.obs_c)
    with pytest.raises(PauliPropError):
        c.evaluate()  # theta never set


@pytest.mark.parametrize("k", [4, 5, 6, 7])
def test_tile_kernel_variants_bitwise(api, k):
    """The three tile-pass kernels (one 256-thread workgroup per tile,
    persistent prefetching workgroups, one wave per tile) run the same ops in
    the same order on every tile, so results are identical bit for bit."""
    from paper_2502_10685_amd import _lib as L
    rng = np.random.default_rng(600 + k)
    n = k + 3
    wc = W.random_circuit(rng, n, 900, W.obs_tfim(n))
    sv = oracle.expval_sv(wc)
    vals = []
    old = L.tune_get(L.PP_TUNE_TILE_KERNEL, k)
    try:
        for variant in ((0, 1, 2) if k <= 6 else (0, 1)):
            L.tune_set(L.PP_TUNE_TILE_KERNEL, k, variant)
            c = api.Circuit.from_workload(wc, engine="dense", tile_qubits=k)
            vals.append(float(c.evaluate().item()))
            c.close()
    finally:
        L.tune_set(L.PP_TUNE_TILE_KERNEL, k, old)
    assert all(v == vals[0] for v in vals), vals
    assert abs(vals[0] - sv) <= TOL64


@pytest.mark.parametrize("n", [5, 6, 7])
def test_resident_block_sizes_agree(api, n):
    """The LDS-resident kernel at 256, 512 and 1024 threads: the ops run in the
    same order on every slot, only the readout sum order differs."""
    from paper_2502_10685_amd import _lib as L
    rng = np.random.default_rng(640 + n)
    wc = W.random_circuit(rng, n, 700, W.obs_tfim(n))
    sv = oracle.expval_sv(wc)
    old = L.tune_get(L.PP_TUNE_RESIDENT_BLOCK, n)
    try:
        for b in (256, 512, 1024):
            L.tune_set(L.PP_TUNE_RESIDENT_BLOCK, n, b)
            c = api.Circuit.from_workload(wc)
            assert abs(float(c.evaluate().item()) - sv) <= TOL64, b
            c.close()
    finally:
        L.tune_set(L.PP_TUNE_RESIDENT_BLOCK, n, old)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [8, 9, 10])
def test_register_tile_kernel_bitwise(api, n, dtype):
    """The register-tile kernel (one wave per 4^6-slot tile, the tile held in
    registers, LDS only between digit-triple segments), persistent or not,
    against the 256-thread LDS kernel.  Selecting it re-plans the circuit
    with its ops ordered into segments; its two forms run the same ops in the
    same order with the same FP32 rounding points, so their weights are
    identical bit for bit.  The LDS kernel's plan packs commuting ops in
    another order (other rounding): its weights agree within the tolerance;
    all match the state vector."""
    from paper_2502_10685_amd import _lib as L
    rng = np.random.default_rng(660 + n)
    wc = W.random_circuit(rng, n, 1500, W.obs_tfim(n))
    sv = oracle.expval_sv(wc)
    tol = TOL64 if dtype == "f64" else TOL32
    old = L.tune_get(L.PP_TUNE_TILE_KERNEL, 6)
    res = []
    try:
        for variant in (0, 3, 4):
            L.tune_set(L.PP_TUNE_TILE_KERNEL, 6, variant)
            print(f"register tile n={n} {dtype} variant={variant}", flush=True)
            c = api.Circuit.from_workload(wc, engine="dense", tile_qubits=6, dtype=dtype)
            ev = float(c.evaluate().item())
            x, z, cf = c.terms()
            res.append((ev, x, z, cf))
            c.close()
    finally:
        L.tune_set(L.PP_TUNE_TILE_KERNEL, 6, old)
    e0, x0, z0, c0 = res[0]
    e3, x3, z3, c3 = res[1]
    e4, x4, z4, c4 = res[2]
    assert e3 == e4
    assert np.array_equal(x3, x4) and np.array_equal(z3, z4)
    assert np.array_equal(c3.view(np.uint64), c4.view(np.uint64))
    # the same weights up to rounding (a string whose weight cancels to
    # exactly zero in one order may be reported by the other only)
    w0 = {(int(a), int(b)): float(w) for a, b, w in zip(x0, z0, c0)}
    w3 = {(int(a), int(b)): float(w) for a, b, w in zip(x3, z3, c3)}
    assert max(abs(w0.get(key, 0.0) - w3.get(key, 0.0)) for key in set(w0) | set(w3)) <= tol
    for e in (e0, e3):
        assert abs(e - sv) <= tol


@pytest.mark.parametrize("n", [14, 15])
def test_register_tile_kernel_largest_registers(api, n):
    """n = 14 is the largest register the register-tile kernel takes (its
    buffer offsets reach 2^31 bytes at FP64); at n = 15 the launcher runs the
    LDS kernel instead.  Its two forms agree bit for bit, the LDS kernel's
    plan (another op order) within the tolerance; all match the state
    vector."""
    from paper_2502_10685_amd import _lib as L
    rng = np.random.default_rng(657 + n)
    wc = W.random_circuit(rng, n, 90, W.obs_z(n, [0, n - 1]))
    sv = oracle.expval_sv(wc)
    old = L.tune_get(L.PP_TUNE_TILE_KERNEL, 6)
    vals = []
    try:
        for variant in (0, 3, 4):
            L.tune_set(L.PP_TUNE_TILE_KERNEL, 6, variant)
            print(f"register tile n={n} variant={variant}", flush=True)
            c = api.Circuit.from_workload(wc, engine="dense", tile_qubits=6)
            vals.append(float(c.evaluate().item()))
            c.close()
    finally:
        L.tune_set(L.PP_TUNE_TILE_KERNEL, 6, old)
    assert vals[1] == vals[2], vals
    for v in vals:
        assert abs(v - sv) <= TOL64, vals
    assert abs(vals[1] - sv) <= TOL64


def test_untracked_dense_terms_are_the_nonzero_weights(api):
    """Without term tracking a tiled DENSE evaluation reports the strings of
    nonzero final weight: they match the tracked structural set up to the
    exact zeros, weight by weight; an untracked LDS-resident run refuses."""
    from paper_2502_10685_amd._lib import PauliPropError
    rng = np.random.default_rng(680)
    wc = W.random_circuit(rng, 8, 600, W.obs_tfim(8))
    ct = api.Circuit.from_workload(wc, engine="dense", track=True)
    ct.evaluate()
    xt, zt, cft = ct.terms()
    cu = api.Circuit.from_workload(wc, engine="dense")
    cu.evaluate()
    xu, zu, cfu = cu.terms()
    assert np.all(cfu != 0.0)
    tr = {(int(a), int(b)): float(w) for a, b, w in zip(xt, zt, cft)}
    un = {(int(a), int(b)): float(w) for a, b, w in zip(xu, zu, cfu)}
    assert set(un) <= set(tr)
    assert all(key in un for key, w in tr.items() if abs(w) > 1e-9)
    assert max(abs(tr[key] - un.get(key, 0.0)) for key in tr) <= TOL64
    small = api.Circuit.from_workload(W.config1())
    small.evaluate()
    with pytest.raises(PauliPropError):
        small.terms()


def test_chain_zxz_paper_shape(api):
    """The 60,200-gate n = 4 circuit of the paper's timing ansatz shape."""
    wc = W.chain_zxz_circuit()
    c = api.Circuit.from_workload(wc)
    print("chain zxz n=4 60200 gates", flush=True)
    assert abs(float(c.evaluate().item()) - oracle.expval_sv(wc)) <= TOL64
