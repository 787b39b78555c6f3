"""Big-means on one AMD Instinct MI355X (gfx950).

The clustering runs in hand-written HIP kernels behind a C ABI
(``include/bigmeans.h``, built into ``libbigmeans.so``); ``bigmeans`` is the
thin ctypes binding over it and ``synth`` makes seeded synthetic inputs.
"""
import importlib

__all__ = ["bigmeans", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
