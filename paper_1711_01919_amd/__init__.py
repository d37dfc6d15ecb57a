"""Exact uint32 integral histograms of uint8 frames on AMD MI355X (gfx950).

The computation lives in ``libih.so`` (hand-written HIP kernels behind the C
ABI declared in ``include/ih.h``).  This package is the thin Python binding
used by the tests and the benchmark: it marshals arguments (torch tensors for
device memory, torch streams) and calls the library.  It never computes a
result itself and has no CPU fallback: importing ``binding`` raises when the
library is missing.

``synth`` draws the seeded synthetic inputs and holds none of the method.
"""
import importlib

__all__ = ["binding", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
