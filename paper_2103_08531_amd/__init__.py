"""MI355X-native VGF / Hockney-Eastwood free-space Poisson solver.

The compute path is the HIP library csrc/ -> libvgf.so behind the C ABI
declared in include/vgf.h; `vgf` is its thin ctypes binding (torch is used
only for device memory and streams). `workloads` holds the seeded synthetic
charge densities.
"""
import importlib

__all__ = ["vgf", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
