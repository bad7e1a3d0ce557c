"""MI355X-native particles-on-demand (PonD) f+g step, DDF-BGK, total-energy split, D2Q16.

The compute path is the HIP library ``libpond.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/pond.h``; ``pond`` is its thin ctypes binding.
``workloads`` draws seeded initial fields.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "pond"]


def __getattr__(name):
    if name == "pond":
        import importlib
        return importlib.import_module(__name__ + ".pond")
    raise AttributeError(name)
