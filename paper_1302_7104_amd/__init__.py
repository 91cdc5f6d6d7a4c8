"""MI355X-native polar-coordinate FDLB step (Lin, Xu, Zhang, Li, Succi,
arXiv:1302.7104): HIP kernels behind the C ABI of include/pclb.h, a ctypes
binding, and torch-owned device memory.

``workloads`` (seeded inputs) imports without the native library; ``Sim``
and the autograd Functions load libpclb.so on first use and raise if it is
missing.
"""
import importlib

__all__ = ["Sim", "InitState", "Evolve"]


def __getattr__(name):
    if name in ("Sim", "InitState", "Evolve"):
        return getattr(importlib.import_module(".sim", __name__), name)
    raise AttributeError(name)
