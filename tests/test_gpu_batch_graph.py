"""The batch step captured as one hipGraph (PP_OPT_USE_GRAPH on every
circuit of a pp_evaluate_batch call) against the eager step: every replay
equal bit for bit, with the program's own eager work and synchronizations
between replays, new theta picked up at replay, a new output array or a
changed set of circuits recaptured, and batches that cannot be captured
(a SPARSE member) run eagerly."""
import sys

import numpy as np
import pytest

import oracle
from paper_2502_10685_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def api():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible HIP device"
    from paper_2502_10685_amd import api as A
    return A


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def _use_graph(objs, on):
    from paper_2502_10685_amd import _lib as L
    for o in objs:
        o.set_option(L.PP_OPT_USE_GRAPH, 1 if on else 0)


def test_batch_graph_replays_equal_eager(api):
    import torch
    circs = W.config3(count=24, m_lo=200, m_hi=1500)  # LDS-resident and tiled circuits
    objs = [api.Circuit.from_workload(w) for w in circs]
    out_e = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    _say("eager batch of 24")
    api.evaluate_batch(objs, out_e)
    torch.cuda.synchronize()
    want = out_e.cpu().numpy().copy()
    _use_graph(objs, True)
    out_g = torch.empty_like(out_e)
    for rep in range(4):
        _say(f"graph replay {rep}")
        out_g.fill_(float("nan"))
        api.evaluate_batch(objs, out_g)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(out_g.cpu().numpy()), _bits(want)), rep
        # eager work of the program between replays
        solo = float(objs[rep].evaluate().item())
        assert _bits([solo])[0] == _bits([want[rep]])[0]
    for w, v in zip(circs[:5], want[:5]):
        assert abs(v - oracle.expval_sv(w)) <= TOL64
    for o in objs:
        o.close()


def test_batch_graph_reads_new_theta(api):
    import torch
    circs = W.config3(count=12, m_lo=300, m_hi=1200)
    objs = [api.Circuit.from_workload(w) for w in circs]
    _use_graph(objs, True)
    out = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    api.evaluate_batch(objs, out)  # captures
    torch.cuda.synchronize()
    rng = np.random.default_rng(77)
    for rep in range(3):
        thetas = [rng.uniform(0, 2 * np.pi, size=w.n_params) for w in circs]
        for o, th in zip(objs, thetas):
            o.set_theta(th)
        _say(f"graph replay with new theta {rep}")
        api.evaluate_batch(objs, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        _use_graph(objs, False)
        solo = np.array([float(o.evaluate().item()) for o in objs])
        _use_graph(objs, True)
        assert np.array_equal(_bits(got), _bits(solo)), rep
        w = circs[rep]
        wt = W.make_circuit(w.n, (w.op, w.q0, w.q1, w.param), w.n_params, (w.obs_x, w.obs_z, w.obs_c), thetas[rep])
        assert abs(got[rep] - oracle.expval_sv(wt)) <= TOL64
    for o in objs:
        o.close()


def test_batch_graph_recaptures_on_change(api):
    import torch
    circs = W.config3(count=10, m_lo=300, m_hi=1000)
    objs = [api.Circuit.from_workload(w) for w in circs]
    solo = np.array([float(o.evaluate().item()) for o in objs])
    _use_graph(objs, True)
    a = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    b = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    _say("graph: output array A, B, then a smaller set")
    api.evaluate_batch(objs, a)
    api.evaluate_batch(objs, b)  # new output array: recaptured
    torch.cuda.synchronize()
    assert np.array_equal(_bits(a.cpu().numpy()), _bits(solo))
    assert np.array_equal(_bits(b.cpu().numpy()), _bits(solo))
    api.evaluate_batch(objs[:6], a[:6])  # another set of circuits
    torch.cuda.synchronize()
    assert np.array_equal(_bits(a[:6].cpu().numpy()), _bits(solo[:6]))
    for o in objs:
        o.close()


def test_batch_with_sparse_member_runs_eagerly(api):
    import torch
    circs = W.config3(count=6, m_lo=200, m_hi=600)
    objs = [api.Circuit.from_workload(w) for w in circs]
    wsp = W.random_circuit(np.random.default_rng(5), 14, 120, W.obs_z(14, [0]))
    objs.append(api.Circuit.from_workload(wsp, engine="sparse"))
    _use_graph(objs, True)
    out = torch.empty(len(objs), dtype=torch.float64, device="cuda")
    _say("graph option with a SPARSE member")
    for _ in range(2):
        api.evaluate_batch(objs, out)
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    for w, v in zip(circs + [wsp], got):
        assert abs(v - oracle.expval_sv(w)) <= TOL64
    for o in objs:
        o.close()
