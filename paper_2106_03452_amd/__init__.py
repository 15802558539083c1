"""MI355X-native differentiable Poisson solver (Shape As Points, Peng et al. 2021).

The compute lives in ``libpsr.so`` (hand-written HIP for gfx950, C ABI in
``include/psr.h``); this package is its thin Python binding:

  * ``solve(points, normals, res, sigma)`` -- differentiable indicator grid;
  * ``forward`` / ``backward`` -- the two ABI calls with explicit buffers;
  * ``batched`` -- many independent solves per launch sequence;
  * ``serve`` -- continuous-batching request engine.
"""
from ._lib import PSRError, Context, context, lib, workspace_bytes, saved_bytes  # noqa: F401

__all__ = ["PSRError", "Context", "context", "lib", "workspace_bytes", "saved_bytes",
           "solve", "forward", "backward"]


def __getattr__(name):
    # the torch-facing helpers import torch lazily so that the ABI checks run without it
    if name in ("solve", "forward", "backward", "status", "scalars", "debug_spectral", "debug_splat",
                "PSRFunction"):
        from . import function
        return getattr(function, name)
    raise AttributeError(name)
