"""MI355X (gfx950) implementation of the per-step sweep of the third-order
discrete unified gas kinetic scheme (T3S3-DUGKS), Wu, Shu, Shi & Chen,
arXiv 1709.05458.

- ``cases``: velocity sets, grids and initial fields (inputs).
- ``dugks``: ctypes binding of the C-ABI library ``libdugks.so`` (HIP kernels).
"""
from . import cases  # noqa: F401

__all__ = ["cases", "dugks"]


def __getattr__(name):
    if name == "dugks":
        import importlib
        return importlib.import_module(__name__ + ".dugks")
    raise AttributeError(name)
