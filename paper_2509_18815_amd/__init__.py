"""MI355X-native GMM rANS entropy coder (FlashGMM hot path) for gfx950.

The compute path is hand-written HIP behind the C ABI of ``libflashgmm.so``
(declared in ``include/flashgmm.h``); :mod:`.api` is a thin ctypes binding
over it. Importing the package itself loads nothing native, so that the
input generator (:mod:`.synth`) can be used on machines without a GPU.
"""
import importlib

__all__ = ["api", "synth"]


def __getattr__(name):
    if name in ("api", "synth", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
