"""PyTorch front end: device buffers and streams come from torch, all compute from libpsr.

``solve(points, normals, res, sigma)`` is differentiable with respect to the
points and the normals (main Sec. 3.1: the solver must pass gradients from a
loss on the indicator grid back to the oriented point cloud).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_points(points: torch.Tensor, normals: torch.Tensor):
    for name, t in (("points", points), ("normals", normals)):
        if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3:
            raise ValueError(f"{name} must be a CUDA float32 tensor of shape (P, 3), got "
                             f"{tuple(t.shape)} {t.dtype} on {t.device}")
    if points.shape != normals.shape or points.device != normals.device:
        raise ValueError("points and normals must have the same shape and device")


def forward(points: torch.Tensor, normals: torch.Tensor, res: int, sigma: float = 2.0,
            ctx: _lib.Context | None = None, workspace: torch.Tensor | None = None):
    """Run ``psr_forward``. Returns (chi [res,res,res] float32, saved uint8 tensor)."""
    _check_points(points, normals)
    points = points.contiguous()
    normals = normals.contiguous()
    dev = points.device
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    P = int(points.shape[0])
    ws_bytes = _lib.workspace_bytes(res, P)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    saved = torch.empty(_lib.saved_bytes(res, P), dtype=torch.uint8, device=dev)
    chi = torch.empty((res, res, res), dtype=torch.float32, device=dev)
    rc = _lib.lib().psr_forward(ctx.handle, _ptr(points), _ptr(normals), P, int(res), float(sigma),
                                _ptr(chi), _ptr(saved), _ptr(workspace), ctypes.c_size_t(workspace.numel()),
                                _stream(dev))
    _lib.check(rc, "psr_forward")
    # the resolution and point count this state was made for; backward checks them
    saved.psr_meta = (int(res), P)
    return chi, saved


def _check_saved(chi: torch.Tensor, saved: torch.Tensor, npoints: int, res: int) -> None:
    """Raise before any launch if (res, npoints) cannot be the forward's: the
    kernels would index the saved state with the wrong layout."""
    if tuple(chi.shape) != (res, res, res) or chi.dtype != torch.float32 or not chi.is_cuda:
        raise ValueError(f"chi must be a CUDA float32 ({res},{res},{res}) tensor, got {tuple(chi.shape)} {chi.dtype}")
    if saved.dtype != torch.uint8 or not saved.is_cuda or saved.numel() < _lib.saved_bytes(res, npoints):
        raise ValueError(f"saved must be the uint8 state of a forward with res={res}, npoints={npoints}")
    meta = getattr(saved, "psr_meta", None)
    if meta is not None and meta != (int(res), int(npoints)):
        raise ValueError(f"saved comes from a forward with (res, npoints) = {meta}, backward got "
                         f"({res}, {npoints})")


def backward(chi: torch.Tensor, saved: torch.Tensor, dchi: torch.Tensor, npoints: int, res: int,
             sigma: float = 2.0, need_points: bool = True, need_normals: bool = True,
             ctx: _lib.Context | None = None, workspace: torch.Tensor | None = None):
    """Run ``psr_backward``. Returns (dpoints or None, dnormals or None), each (P, 3)."""
    dev = chi.device
    _check_saved(chi, saved, npoints, res)
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    dchi = dchi.contiguous().to(torch.float32)
    if dchi.shape != chi.shape:
        raise ValueError("dchi must have the shape of chi")
    ws_bytes = _lib.workspace_bytes(res, npoints)
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    dp = torch.empty((npoints, 3), dtype=torch.float32, device=dev) if need_points else None
    dn = torch.empty((npoints, 3), dtype=torch.float32, device=dev) if need_normals else None
    rc = _lib.lib().psr_backward(ctx.handle, int(npoints), int(res), float(sigma), _ptr(chi), _ptr(saved),
                                 _ptr(dchi), _ptr(dp), _ptr(dn), _ptr(workspace),
                                 ctypes.c_size_t(workspace.numel()), _stream(dev))
    _lib.check(rc, "psr_backward")
    return dp, dn


def status(saved: torch.Tensor) -> int:
    """Synchronise the current stream and return the forward's status code."""
    out = ctypes.c_int(0)
    _lib.check(_lib.lib().psr_saved_status(_ptr(saved), _stream(saved.device), ctypes.byref(out)),
               "psr_saved_status")
    return int(out.value)


def scalars(saved: torch.Tensor) -> dict:
    """Synchronise and return the forward's FP64 scalars (mean, cscale, scale, chi0)."""
    vals = [ctypes.c_double(0.0) for _ in range(4)]
    _lib.check(_lib.lib().psr_saved_scalars(_ptr(saved), _stream(saved.device), *[ctypes.byref(v) for v in vals]),
               "psr_saved_scalars")
    return dict(zip(("mean", "cscale", "scale", "chi0"), (v.value for v in vals)))


def debug_spectral(v: torch.Tensor, sigma: float = 2.0, ctx: _lib.Context | None = None) -> torch.Tensor:
    """Spectral solve only (main Eq. 3) of a given field v [3, r, r, r] -> unnormalised chi'."""
    if not v.is_cuda or v.dtype != torch.float32 or v.dim() != 4 or v.shape[0] != 3:
        raise ValueError("v must be a CUDA float32 tensor of shape (3, r, r, r)")
    v = v.contiguous()
    res = int(v.shape[-1])
    dev = v.device
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    ws = torch.empty(_lib.workspace_bytes(res, 1), dtype=torch.uint8, device=dev)
    out = torch.empty((res, res, res), dtype=torch.float32, device=dev)
    _lib.check(_lib.lib().psr_debug_spectral(ctx.handle, _ptr(v), res, float(sigma), _ptr(out), _ptr(ws),
                                             ctypes.c_size_t(ws.numel()), _stream(dev)), "psr_debug_spectral")
    return out


def debug_splat(points: torch.Tensor, normals: torch.Tensor, res: int,
                ctx: _lib.Context | None = None) -> torch.Tensor:
    """Rasterised normal field v [3, r, r, r] (supplement Sec. A.1)."""
    _check_points(points, normals)
    points, normals = points.contiguous(), normals.contiguous()
    dev = points.device
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    P = int(points.shape[0])
    ws = torch.empty(_lib.workspace_bytes(res, P), dtype=torch.uint8, device=dev)
    saved = torch.empty(_lib.saved_bytes(res, P), dtype=torch.uint8, device=dev)
    v = torch.empty((3, res, res, res), dtype=torch.float32, device=dev)
    _lib.check(_lib.lib().psr_debug_splat(ctx.handle, _ptr(points), _ptr(normals), P, int(res), _ptr(v),
                                          _ptr(saved), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream(dev)),
               "psr_debug_splat")
    return v


class PSRFunction(torch.autograd.Function):
    """chi = DPSR(points, normals); backward is the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, points, normals, res, sigma):
        chi, saved = forward(points, normals, res, sigma)
        ctx.res, ctx.sigma, ctx.P = int(res), float(sigma), int(points.shape[0])
        ctx.save_for_backward(chi, saved)
        return chi

    @staticmethod
    def backward(ctx, dchi):
        chi, saved = ctx.saved_tensors
        dp, dn = backward(chi, saved, dchi, ctx.P, ctx.res, ctx.sigma,
                          need_points=ctx.needs_input_grad[0], need_normals=ctx.needs_input_grad[1])
        return dp, dn, None, None


def solve(points: torch.Tensor, normals: torch.Tensor, res: int, sigma: float = 2.0) -> torch.Tensor:
    """Differentiable indicator grid chi [res, res, res] of an oriented point cloud."""
    return PSRFunction.apply(points, normals, res, sigma)
