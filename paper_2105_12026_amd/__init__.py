"""MI355X-native exemplar-based clustering (EBC) hot path.

The compute lives in ``libebc.so`` (hand-written HIP for gfx950, C ABI declared
in include/ebc.h). This package holds the thin ctypes binding (``ebc``), the
build step (``build``) and the seeded input generators (``workloads``).
Submodules load lazily so that importing the generators never touches a GPU.
"""
import importlib

__all__ = ["ebc", "workloads", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
