"""MI355X-native pass-through connectivity counting (FastCod, Section 2 "Method", Alg. 2).

The counting runs in hand-written HIP kernels for gfx950 behind the C-ABI library
``libfastcod.so`` (declared in ``include/fastcod.h``); ``fastcod`` is its thin ctypes
binding.  ``synth`` draws seeded synthetic workloads.  Submodules load lazily so that
``synth`` is usable without the built library.
"""
import importlib

__all__ = ["fastcod", "synth", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
