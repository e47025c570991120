"""MI355X (gfx950) restarted-PDHCG solver for linear Fisher markets.

``paper_2506_06258_amd.pdhcg`` is the ctypes binding of the HIP library
(``libpdhcg.so``, C ABI in ``include/pdhcg.h``); ``synth`` draws seeded
synthetic markets.  Submodules are imported on first use so that the
generators work without loading the GPU library.
"""
import importlib

__all__ = ["pdhcg", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
