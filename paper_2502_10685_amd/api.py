"""Python binding of libpauliprop: device memory and streams come from torch;
every step of the propagation runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

_DTYPES = {"f64": L.PP_F64, "fp64": L.PP_F64, "float64": L.PP_F64,
           "f32": L.PP_F32, "fp32": L.PP_F32, "float32": L.PP_F32}
_ENGINES = {"auto": L.PP_ENGINE_AUTO, "dense": L.PP_ENGINE_DENSE, "sparse": L.PP_ENGINE_SPARSE}


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("pauliprop needs a HIP device (MI355X); none is visible")


class Circuit:
    """One parameterized circuit with an observable, owned by the library."""

    def __init__(self, n, op, q0, q1, param, n_params, obs_x, obs_z, obs_c, *, theta=None,
                 dtype="f64", engine="auto", track=False, tile_qubits=0, use_graph=False,
                 max_terms=0):
        _require_gpu()
        self._lib = L.load()
        self.n = int(n)
        self.n_params = int(n_params)
        self.dtype = dtype
        h = ctypes.c_void_p()
        L.check(self._lib.pp_circuit_create(self.n, _DTYPES[dtype], _ENGINES[engine], ctypes.byref(h)))
        self._h = h
        self.load_gates(op, q0, q1, param, n_params)
        self.set_observable(obs_x, obs_z, obs_c)
        if track:
            self.set_option(L.PP_OPT_TRACK_TERMS, 1)
        if tile_qubits:
            self.set_option(L.PP_OPT_TILE_QUBITS, tile_qubits)
        if use_graph:
            self.set_option(L.PP_OPT_USE_GRAPH, 1)
        if max_terms:
            self.set_option(L.PP_OPT_MAX_TERMS, max_terms)
        if theta is not None:
            self.set_theta(theta)

    @classmethod
    def from_workload(cls, wc, **kw):
        return cls(wc.n, wc.op, wc.q0, wc.q1, wc.param, wc.n_params, wc.obs_x, wc.obs_z, wc.obs_c,
                   theta=wc.theta, **kw)

    # -------------------------------------------------------------- setup
    def load_gates(self, op, q0, q1, param, n_params):
        op = np.ascontiguousarray(op, dtype=np.uint8)
        q0 = np.ascontiguousarray(q0, dtype=np.int32)
        q1 = np.ascontiguousarray(q1, dtype=np.int32)
        param = np.ascontiguousarray(param, dtype=np.int32)
        self._op, self._q0, self._q1, self._param = op, q0, q1, param
        self._psr = None
        self.m = int(op.shape[0])
        L.check(self._lib.pp_circuit_load_gates(self._h, self.m, _ptr(op), _ptr(q0), _ptr(q1),
                                                _ptr(param), int(n_params)))
        self.n_params = int(n_params)

    def set_observable(self, x, z, c):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        self._obs = (x, z, c)
        self._psr = None
        L.check(self._lib.pp_circuit_set_observable(self._h, int(x.shape[0]), _ptr(x), _ptr(z), _ptr(c)))

    def set_theta(self, theta, stream=None):
        if isinstance(theta, torch.Tensor) and theta.is_cuda:
            t = theta.detach().to(torch.float64).contiguous()
            L.check(self._lib.pp_circuit_set_theta(self._h, ctypes.c_void_p(t.data_ptr()), 1,
                                                   _stream(stream)))
            self._theta_keep = t
        else:
            a = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
            if a.size == 0:
                a = np.zeros(1)
            L.check(self._lib.pp_circuit_set_theta(self._h, _ptr(a), 0, _stream(stream)))

    def set_option(self, key, value):
        L.check(self._lib.pp_circuit_set_option(self._h, int(key), int(value)))

    # ---------------------------------------------------------- evaluation
    def evaluate(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty((), dtype=torch.float64, device="cuda")
        L.check(self._lib.pp_evaluate(self._h, _stream(stream), ctypes.c_void_p(out.data_ptr())))
        return out

    def evaluate_thetas(self, thetas, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """<O> at every row of thetas (count x n_params), one set of shared
        launches; a CUDA tensor is read in place, anything else is copied."""
        if isinstance(thetas, torch.Tensor) and thetas.is_cuda:
            t = thetas.detach().to(torch.float64).contiguous()
            count = int(t.shape[0]) if t.dim() > 1 else 1
            ptr, on_dev = ctypes.c_void_p(t.data_ptr()), 1
            keep = t
        else:
            t = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64))
            count = int(t.shape[0]) if t.ndim > 1 else 1
            if t.size == 0:
                t = np.zeros(max(count, 1))
            ptr, on_dev = _ptr(t), 0
            keep = t
        if out is None:
            out = torch.empty(count, dtype=torch.float64, device="cuda")
        L.check(self._lib.pp_evaluate_thetas(self._h, count, ptr, on_dev, _stream(stream),
                                             ctypes.c_void_p(out.data_ptr())))
        self._sweep_keep = keep
        return out

    def psr_gradient(self, theta, stream=None):
        """Parameter-shift gradient of <O> from 2 x (rotation gates) shifted
        evaluations in one sweep: each rotation gate gets its own copy of its
        parameter, shifted by +-pi/2, and the halves of the differences are
        summed per parameter.  Uses a private circuit with one parameter per
        rotation gate (built on first use)."""
        import math
        theta = np.asarray(theta.detach().cpu().numpy() if isinstance(theta, torch.Tensor) else theta,
                           dtype=np.float64)
        if getattr(self, "_psr", None) is None:
            rot = np.nonzero(self._op >= 3)[0]
            pexp = np.full(self.m, -1, np.int32)
            pexp[rot] = np.arange(rot.size, dtype=np.int32)
            c = Circuit(self.n, self._op, self._q0, self._q1, np.where(pexp >= 0, pexp, 0), max(rot.size, 1),
                        self._obs[0], self._obs[1], self._obs[2], dtype=self.dtype, engine="dense")
            self._psr = (c, rot)
        c, rot = self._psr
        base = theta[self._param[rot]] if rot.size else np.zeros(1)
        R = rot.size
        thetas = np.repeat(base[None, :], 2 * max(R, 1), axis=0)
        for j in range(R):
            thetas[2 * j, j] += math.pi / 2
            thetas[2 * j + 1, j] -= math.pi / 2
        vals = c.evaluate_thetas(thetas, stream=stream).cpu().numpy()
        gexp = 0.5 * (vals[0::2] - vals[1::2])[:R]
        grad = np.zeros(self.n_params)
        np.add.at(grad, self._param[rot], gexp)
        return torch.tensor(grad, dtype=torch.float64)

    def gradient(self, checkpoint_every=0, stream=None):
        ev = torch.empty((), dtype=torch.float64, device="cuda")
        grad = torch.zeros(max(self.n_params, 1), dtype=torch.float64, device="cuda")
        L.check(self._lib.pp_gradient(self._h, _stream(stream), int(checkpoint_every),
                                      ctypes.c_void_p(ev.data_ptr()), ctypes.c_void_p(grad.data_ptr())))
        return ev, grad[: self.n_params]

    def density_matrix(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """rho = U|0><0|U^dag as a complex128 (2^n, 2^n) CUDA tensor (n <= 12);
        basis bit q is qubit q.  `out`, if given, is a float64 CUDA tensor of
        shape (2^n, 2^n, 2) that receives (real, imaginary) pairs."""
        N = 1 << self.n
        if out is None:
            out = torch.empty((N, N, 2), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous() and out.numel() == 2 * N * N
        L.check(self._lib.pp_density_matrix(self._h, _stream(stream), ctypes.c_void_p(out.data_ptr())))
        return torch.view_as_complex(out.view(N, N, 2))

    def set_truncation(self, min_abs_coeff=0.0, max_weight=64):
        """Approximate SPARSE propagation: drop strings heavier than max_weight
        letters or lighter than min_abs_coeff (defaults: exact)."""
        L.check(self._lib.pp_circuit_set_truncation(self._h, float(min_abs_coeff), int(max_weight)))

    def truncation_dropped(self, stream=None) -> float:
        """Summed |weight| dropped by truncation in the last evaluation; it
        bounds the error of <O>."""
        v = ctypes.c_double(0.0)
        L.check(self._lib.pp_get_truncation(self._h, _stream(stream), ctypes.byref(v)))
        return v.value

    def terms(self, capacity=None, stream=None):
        """Final string set of the last evaluation, canonical order (z, then x)."""
        if capacity is None:
            capacity = min(4 ** self.n, 1 << 26)
        x = np.zeros(capacity, np.uint64)
        z = np.zeros(capacity, np.uint64)
        c = np.zeros(capacity, np.float64)
        nout = ctypes.c_int64(0)
        L.check(self._lib.pp_get_terms(self._h, _stream(stream), capacity, _ptr(x), _ptr(z), _ptr(c),
                                       ctypes.byref(nout)))
        k = nout.value
        return x[:k], z[:k], c[:k]

    def stats(self) -> dict:
        s = L.PPStats()
        L.check(self._lib.pp_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_psr", None) is not None:
            self._psr[0].close()
            self._psr = None
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pp_circuit_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evaluate_batch(circuits, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    lib = L.load()
    n = len(circuits)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
    arr = (ctypes.c_void_p * max(n, 1))(*[c._h.value for c in circuits])
    L.check(lib.pp_evaluate_batch(ctypes.cast(arr, ctypes.c_void_p), n, _stream(stream),
                                  ctypes.c_void_p(out.data_ptr())))
    return out


class Server:
    """Continuous-batching serving loop of the library (its own host thread
    and streams).  submit() takes a prepared Circuit and returns a ticket;
    poll() returns None until done, then (expval, latency_us)."""

    def __init__(self, mem_budget_bytes=64 << 30, max_active=256):
        _require_gpu()
        self._lib = L.load()
        h = ctypes.c_void_p()
        L.check(self._lib.pp_server_create(int(mem_budget_bytes), int(max_active), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, circ: Circuit) -> int:
        t = ctypes.c_int64(0)
        L.check(self._lib.pp_server_submit(self._h, circ._h, ctypes.byref(t)))
        self._keep[t.value] = circ
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32(0)
        ev = ctypes.c_double(0.0)
        lat = ctypes.c_double(0.0)
        L.check(self._lib.pp_server_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(ev),
                                         ctypes.byref(lat)))
        if not done.value:
            return None
        self._keep.pop(int(ticket), None)
        return ev.value, lat.value

    def drain(self):
        L.check(self._lib.pp_server_drain(self._h))

    def counters(self):
        a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        L.check(self._lib.pp_server_counters(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"iterations": a.value, "tile_launches": b.value, "max_in_flight": c.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pp_server_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _ExpvalFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, circ, checkpoint_every):
        circ.set_theta(theta)
        if theta.requires_grad:
            ev, grad = circ.gradient(checkpoint_every)
            ctx.save_for_backward(grad)
        else:
            ev = circ.evaluate()
            ctx.save_for_backward(torch.zeros(0, dtype=torch.float64, device=ev.device))
        return ev.clone()

    @staticmethod
    def backward(ctx, grad_out):
        (grad,) = ctx.saved_tensors
        return (grad_out * grad).to(grad.dtype), None, None


def expval(circ: Circuit, theta: torch.Tensor, checkpoint_every: int = 0) -> torch.Tensor:
    """<O>(theta) with an adjoint gradient behind torch.autograd."""
    return _ExpvalFn.apply(theta, circ, checkpoint_every)
