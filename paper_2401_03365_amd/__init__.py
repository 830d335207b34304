"""MI355X-native moving-least-squares (MLS) projection of point clouds.

The hot path -- exact k-nearest neighbours on a Morton-sorted grid hash,
Gaussian-weighted reference plane, weighted quadratic height fit and
projection, plus its adjoint -- runs in hand-written HIP kernels for gfx950
inside ``lib/libmls.so`` behind the C ABI of ``include/mls.h``. This package
is the thin PyTorch binding (``api``) and the seeded input generators
(``synth``). Importing it does not load the library; the first call does, and
fails loudly if the library has not been built.
"""
import importlib

__all__ = ["Grid", "build_grid", "project", "mls_project", "MLSProject", "autotune_cell_factor"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".api"), name)
    raise AttributeError("module %r has no attribute %r" % (__name__, name))
