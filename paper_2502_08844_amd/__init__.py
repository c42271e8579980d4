"""mjh: a batched rigid-body physics step for AMD MI355X (gfx950).

The GPU binding lives in :mod:`paper_2502_08844_amd.mjh` and is imported on first use,
so that importing :mod:`paper_2502_08844_amd.synth` never loads the native library.
"""
import importlib

__all__ = ["mjh", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
