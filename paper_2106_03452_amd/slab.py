"""Slab-decomposed forward solve for large grids (16^3 to 1024^3), the
large-scene form of the solver (main Sec. 5: the dense grid's memory is cubic
in the resolution).

``forward(points, normals, res, sigma, slabs)`` returns the same indicator
grid as :func:`function.forward` (main Eqs. 2-4) computed slab by slab along
j0: every pass of ``libpsr.so`` runs per slab of res/slabs planes (or per
pencil owner for the transform along j0), and the spectrum moves between them
in equal exchange blocks. This module only allocates buffers and marshals
arguments.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .function import _check_points, _ptr, _stream


class SlabResult(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("cscale", ctypes.c_double), ("scale", ctypes.c_double),
                ("chi0", ctypes.c_double), ("status", ctypes.c_int32), ("flags", ctypes.c_int32)]


def workspace_bytes(res: int, npoints: int, slabs: int) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().psr_slab_workspace_bytes(int(res), int(npoints), int(slabs), ctypes.byref(out)),
               "psr_slab_workspace_bytes")
    return int(out.value)


def _ctx(dev, ctx):
    return ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())


def forward_raw(points: torch.Tensor, normals: torch.Tensor, res: int, sigma: float, slabs: int,
                chi: torch.Tensor, result: torch.Tensor, workspace: torch.Tensor,
                ctx: _lib.Context | None = None) -> None:
    """Enqueue ``psr_slab_forward`` into caller-owned buffers (no allocation,
    no synchronisation): chi [res]^3 float32, result a 48-byte uint8 tensor."""
    dev = points.device
    _lib.check(_lib.lib().psr_slab_forward(_ctx(dev, ctx).handle, _ptr(points), _ptr(normals),
                                           int(points.shape[0]), int(res), float(sigma), int(slabs), _ptr(chi),
                                           _ptr(result), _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                                           _stream(dev)), "psr_slab_forward")


def forward(points: torch.Tensor, normals: torch.Tensor, res: int, sigma: float = 2.0, slabs: int = 8,
            ctx: _lib.Context | None = None, workspace: torch.Tensor | None = None):
    """Run the slab forward. Returns (chi [res,res,res] float32, scalars dict
    with mu, cscale, scale, chi0, status, flags; reading the scalars
    synchronises the stream)."""
    _check_points(points, normals)
    points, normals = points.contiguous(), normals.contiguous()
    dev = points.device
    nbytes = workspace_bytes(res, int(points.shape[0]), slabs)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    chi = torch.empty((res, res, res), dtype=torch.float32, device=dev)
    result = torch.zeros(ctypes.sizeof(SlabResult), dtype=torch.uint8, device=dev)
    forward_raw(points, normals, res, sigma, slabs, chi, result, workspace, ctx)
    return chi, read_result(result)


def read_result(result: torch.Tensor) -> dict:
    r = SlabResult.from_buffer_copy(bytes(result.cpu().numpy()))
    return {"mu": r.mu, "cscale": r.cscale, "scale": r.scale, "chi0": r.chi0, "status": int(r.status),
            "flags": int(r.flags)}


def debug_spectral(v: torch.Tensor, sigma: float = 2.0, slabs: int = 8,
                   ctx: _lib.Context | None = None) -> torch.Tensor:
    """The slab passes on a given field v [3, r, r, r] -> unnormalised chi'."""
    if not v.is_cuda or v.dtype != torch.float32 or v.dim() != 4 or v.shape[0] != 3:
        raise ValueError("v must be a CUDA float32 tensor of shape (3, r, r, r)")
    v = v.contiguous()
    res = int(v.shape[-1])
    dev = v.device
    ws = torch.empty(workspace_bytes(res, 0, slabs), dtype=torch.uint8, device=dev)
    out = torch.empty((res, res, res), dtype=torch.float32, device=dev)
    _lib.check(_lib.lib().psr_slab_debug_spectral(_ctx(dev, ctx).handle, _ptr(v), res, float(sigma), int(slabs),
                                                  _ptr(out), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(dev)),
               "psr_slab_debug_spectral")
    return out
