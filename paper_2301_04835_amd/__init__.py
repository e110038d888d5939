"""sampx: the biasing-force path of CV-based enhanced sampling (PySAGES,
arXiv 2301.04835) as hand-written HIP for MI355X behind a C ABI.

Importing the package loads nothing; :class:`Sampler` loads libsampx.so on
first use and raises if it is not built (there is no CPU fallback).
"""

__all__ = ["Sampler", "CVFunction"]


def __getattr__(name):
    if name == "Sampler":
        from .api import Sampler
        return Sampler
    if name == "CVFunction":
        from .autograd import CVFunction
        return CVFunction
    raise AttributeError(name)
