"""MI355X-native matrix-product-state gate update (arXiv:1111.3124, Section 3.1).

The device path lives in ``csrc/`` (HIP kernels for gfx950 behind a C ABI declared
in ``include/mps.h``); ``binding`` is its thin ctypes wrapper.  ``workloads`` draws
seeded synthetic inputs.  Importing the package does not load the device library;
``paper_1111_3124_amd.binding`` does, and raises if it has not been built.
"""
import importlib

__all__ = ["binding", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
