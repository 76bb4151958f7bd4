"""pauliprop: Heisenberg-picture Pauli propagation on MI355X (gfx950).

The compute path is libpauliprop.so (hand-written HIP kernels behind the C ABI
of include/pauliprop.h); this package only marshals arguments to it.  The
binding is imported lazily so that ``workloads`` can be used without a GPU.
"""

__all__ = ["Circuit", "Server", "evaluate_batch", "expval", "workloads"]


def __getattr__(name):
    if name in ("Circuit", "Server", "evaluate_batch", "expval"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
