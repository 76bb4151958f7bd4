"""Python binding of libpauliprop: device memory and streams come from torch;
every step of the propagation runs in the library's HIP kernels."""
from __future__ import annotations

import atexit
import ctypes
import weakref

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


# ------------------------------------------------------------ device memory
# The library's device buffers come from torch's caching allocator (installed
# on first use), so torch owns the device memory of the whole process.  The
# callbacks may run on the library's own threads (serving loop, preparation
# threads); ctypes takes the GIL for them.
_LIVE = weakref.WeakSet()  # circuits and servers not yet closed
_HOOK = {"struct": None, "kind": None}
# every allocator ever installed stays alive: a block goes back to the hook
# that made it, even after another allocator was installed
_HOOKS_KEPT = []


def _torch_alloc(nbytes, stream, user):
    try:
        return int(torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0)))
    except Exception:  # out of memory: the library reports PP_ERR_NOMEM
        return None


def _torch_free(ptr, nbytes, stream, user):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


def set_allocator(alloc=None, free=None):
    """Installs the library's device allocator.  With no arguments: torch's
    caching allocator.  Otherwise alloc(nbytes) -> device pointer (int) or
    None, and free(ptr).  Blocks go back to the allocator that made them."""
    lib = L.load()
    if alloc is None:
        a, f, kind = _torch_alloc, _torch_free, "torch"
    else:
        a = lambda nbytes, stream, user: alloc(int(nbytes))  # noqa: E731
        f = lambda ptr, nbytes, stream, user: free(int(ptr))  # noqa: E731
        kind = "custom"
    st = L.PPAllocator(L.ALLOC_FN(a), L.FREE_FN(f), None)
    L.check(lib.pp_set_allocator(ctypes.byref(st)))
    _HOOK["struct"], _HOOK["kind"] = st, kind
    _HOOKS_KEPT.append(st)


def reset_allocator():
    """Back to the library's default device allocator (its stream-ordered
    pool)."""
    L.check(L.load().pp_set_allocator(None))
    _HOOK["kind"] = "default"


def memory_in_use():
    """(bytes, blocks) of device memory the library holds."""
    return L.memory_in_use()


@atexit.register
def _release_at_exit():
    # close what is still open while torch (and its allocator) is alive
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass
    if _HOOK["kind"] is not None and L._lib is not None:
        L._lib.pp_set_allocator(None)


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("pauliprop needs a HIP device (MI355X); none is visible")
    if _HOOK["kind"] is None:
        set_allocator()


class Circuit:
    """One parameterized circuit with an observable, owned by the library."""

    def __init__(self, n, op, q0, q1, param, n_params, obs_x, obs_z, obs_c, *, theta=None,
                 dtype="f64", engine="auto", track=False, tile_qubits=0, use_graph=False,
                 max_terms=0, frame_ramp=0):
        _require_gpu()
        self._lib = L.load()
        self.n = int(n)
        self.n_params = int(n_params)
        self.dtype = dtype
        h = ctypes.c_void_p()
        L.check(self._lib.pp_circuit_create(self.n, _DTYPES[dtype], _ENGINES[engine], ctypes.byref(h)))
        self._h = h
        _LIVE.add(self)
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
        if frame_ramp:
            self.set_option(L.PP_OPT_FRAME_RAMP, frame_ramp)
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
        self.m = int(op.shape[0])
        L.check(self._lib.pp_circuit_load_gates(self._h, self.m, _ptr(op), _ptr(q0), _ptr(q1),
                                                _ptr(param), int(n_params)))
        self.n_params = int(n_params)

    def set_observable(self, x, z, c):
        x = np.ascontiguousarray(x, dtype=np.uint64)
        z = np.ascontiguousarray(z, dtype=np.uint64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        self._obs = (x, z, c)
        L.check(self._lib.pp_circuit_set_observable(self._h, int(x.shape[0]), _ptr(x), _ptr(z), _ptr(c)))

    def set_theta(self, theta, stream=None):
        if isinstance(theta, torch.Tensor):
            theta = theta.detach()
        if isinstance(theta, torch.Tensor) and theta.is_cuda:
            t = theta.to(torch.float64).contiguous()
            L.check(self._lib.pp_circuit_set_theta(self._h, ctypes.c_void_p(t.data_ptr()), 1,
                                                   _stream(stream)))
            self._theta_keep = t
        else:
            if isinstance(theta, torch.Tensor):
                theta = theta.cpu().numpy()
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

    def psr_gradient(self, theta=None, stream=None) -> torch.Tensor:
        """Parameter-shift gradient of <O> (a CUDA tensor of n_params
        doubles): the library evaluates the 2 x (rotation gates) shifted
        angle sets as one parameter sweep and sums the halved differences
        per parameter on the device.  theta, if given, is set first."""
        if theta is not None:
            self.set_theta(theta, stream)
        grad = torch.zeros(max(self.n_params, 1), dtype=torch.float64, device="cuda")
        L.check(self._lib.pp_psr_gradient(self._h, _stream(stream), ctypes.c_void_p(grad.data_ptr())))
        return grad[: self.n_params]

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
        _LIVE.add(self)

    def set_queue_limit(self, max_queued):
        """With max_queued > 0, submit() raises PauliPropError(PP_ERR_BUSY)
        while that many requests wait for admission (0: no limit)."""
        L.check(self._lib.pp_server_set_queue_limit(self._h, int(max_queued)))

    def pool_bytes(self):
        """(held, peak) bytes of the server's weight pool."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        L.check(self._lib.pp_server_pool_bytes(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

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
    """Forward evaluates <O> only; backward runs the adjoint gradient
    (pp_gradient) at the angles the forward saw."""

    @staticmethod
    def forward(ctx, theta, circ, checkpoint_every):
        circ.set_theta(theta)
        ev = circ.evaluate()
        ctx.circ = circ
        ctx.checkpoint_every = checkpoint_every
        ctx.save_for_backward(theta)
        return ev.clone()

    @staticmethod
    def backward(ctx, grad_out):
        (theta,) = ctx.saved_tensors
        if not ctx.needs_input_grad[0]:
            return None, None, None
        circ = ctx.circ
        circ.set_theta(theta)
        _, grad = circ.gradient(ctx.checkpoint_every)
        g = grad_out.to(grad.device, torch.float64) * grad
        return g.to(device=theta.device, dtype=theta.dtype), None, None


def expval(circ: Circuit, theta: torch.Tensor, checkpoint_every: int = 0) -> torch.Tensor:
    """<O>(theta) with an adjoint gradient behind torch.autograd (computed
    in backward only)."""
    return _ExpvalFn.apply(theta, circ, checkpoint_every)
