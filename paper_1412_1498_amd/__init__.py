"""MI355X-native overrelaxation gauge fixing of SU(3) lattice fields.

Submodules are imported lazily: ``synth`` (seeded synthetic inputs) needs no
GPU library, while ``gf`` loads the HIP shared library ``libgf.so``.
"""
import importlib

__all__ = ["gf", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
