"""MI355X (gfx950) implementation of the matrix-free Lippmann-Schwinger displacement solver of
arXiv 2301.12836: HIP kernels behind the C ABI of include/ls.h, a ctypes binding (``lsvie``) and
seeded synthetic inputs shaped like the paper's models (``models``)."""

import importlib

from . import models  # noqa: F401

__all__ = ["models", "lsvie"]


def __getattr__(name):
    if name == "lsvie":
        return importlib.import_module(__name__ + ".lsvie")
    raise AttributeError(name)
