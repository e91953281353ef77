"""MI355X (gfx950) hot path of the vectorized primal hybrid FEM of arXiv 2509.11133.

The work runs in libphfem.so (hand-written HIP kernels behind the C-ABI of
include/phfem.h).  ``_binding`` exposes the C entry points under their C names,
``pipeline`` wraps them with tensor allocation, ``meshes`` holds the seeded synthetic
inputs.  Importing the package does not load the library; the first call does, and fails
loudly when it was not built.
"""
from . import meshes  # noqa: F401

__all__ = ["meshes", "pipeline", "_binding"]


def __getattr__(name):
    if name in ("pipeline", "_binding"):
        import importlib

        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
