"""MI355X (gfx950) reverse-mode path for pointful, index-set-typed loops.

The HIP kernels and the C ABI live in libdexmi.so (sources in csrc/, header in
include/dex.h); `dex` is its ctypes binding and `autograd` wraps it as
torch.autograd.Functions. Importing the package does not load the library;
the first call does, and raises if it is not built.
"""
from . import dex  # noqa: F401

__all__ = ["dex", "autograd"]


def __getattr__(name):
    if name == "autograd":
        import importlib
        return importlib.import_module(__name__ + ".autograd")
    raise AttributeError(name)
