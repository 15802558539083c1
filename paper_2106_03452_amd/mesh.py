"""Marching Cubes on the indicator grid, differentiable with respect to the
grid through the inverse surface normal (main Sec. 3.2, Eq. 6).

Every step runs in ``libpsr.so`` (``psr_marching_cubes`` and
``psr_marching_cubes_backward``); this module allocates buffers through
PyTorch, reads the mesh size, and wraps the two calls in an autograd Function.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def state_bytes(res: int) -> int:
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().psr_mc_state_bytes(int(res), ctypes.byref(out)), "psr_mc_state_bytes")
    return int(out.value)


@dataclass
class Mesh:
    verts: torch.Tensor    # (V, 3) float32, positions in [0, 1]^3
    faces: torch.Tensor    # (F, 3) int32 vertex indices, counter-clockwise seen from outside
    normals: torch.Tensor  # (V, 3) float32 unit normals (towards chi > iso)
    edges: torch.Tensor    # (V,) int32 global edge id 3 * j + axis of each vertex
    state: torch.Tensor    # uint8 state for the backward
    res: int
    iso: float


def marching_cubes(chi: torch.Tensor, iso: float = 0.0, ctx: _lib.Context | None = None,
                   capacity: tuple[int, int] | None = None) -> Mesh:
    """Mesh of the level chi = iso of a (res, res, res) float32 CUDA grid.

    Runs the library call with a capacity guess and, if the mesh is larger,
    once more with the exact sizes (the call synchronises the stream to read
    the mesh size)."""
    if not chi.is_cuda or chi.dtype != torch.float32 or chi.dim() != 3 or len(set(chi.shape)) != 1:
        raise ValueError("chi must be a cubic CUDA float32 grid")
    chi = chi.detach().contiguous()
    res = int(chi.shape[0])
    dev = chi.device
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    L = _lib.lib()
    state = torch.empty(state_bytes(res), dtype=torch.uint8, device=dev)
    vcap, tcap = capacity or (max(4096, 8 * res * res), max(8192, 16 * res * res))
    for _ in range(2):
        verts = torch.empty((vcap, 3), dtype=torch.float32, device=dev)
        normals = torch.empty((vcap, 3), dtype=torch.float32, device=dev)
        edges = torch.empty((vcap,), dtype=torch.int32, device=dev)
        tris = torch.empty((tcap, 3), dtype=torch.int32, device=dev)
        _lib.check(L.psr_marching_cubes(ctx.handle, _ptr(chi), res, float(iso), _ptr(verts), _ptr(normals),
                                        _ptr(edges), vcap, _ptr(tris), tcap, _ptr(state), _stream(dev)),
                   "psr_marching_cubes")
        nv, nt, st = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int(0)
        _lib.check(L.psr_mc_counts(_ptr(state), _stream(dev), ctypes.byref(nv), ctypes.byref(nt), ctypes.byref(st)),
                   "psr_mc_counts")
        _lib.check(st.value, "psr_marching_cubes")
        if nv.value <= vcap and nt.value <= tcap:
            n, m = int(nv.value), int(nt.value)
            return Mesh(verts[:n], tris[:m], normals[:n], edges[:n], state, res, float(iso))
        vcap, tcap = max(int(nv.value), 1), max(int(nt.value), 1)
    raise RuntimeError("marching cubes: mesh size changed between two runs on the same grid")


def marching_cubes_backward(chi: torch.Tensor, mesh: Mesh, dverts: torch.Tensor,
                            ctx: _lib.Context | None = None) -> torch.Tensor:
    """dL/dchi (res^3) from dL/dverts through dp/dchi = -n (main Eq. 6)."""
    chi = chi.detach().contiguous()
    dev = chi.device
    if tuple(chi.shape) != (mesh.res,) * 3:
        raise ValueError("chi must be the grid the mesh was made from")
    dverts = dverts.contiguous().to(torch.float32)
    if dverts.shape != mesh.verts.shape:
        raise ValueError("dverts must have the shape of the mesh vertices")
    ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
    dchi = torch.empty_like(chi)
    nv = int(mesh.verts.shape[0])
    _lib.check(_lib.lib().psr_marching_cubes_backward(ctx.handle, _ptr(chi), mesh.res, float(mesh.iso),
                                                      _ptr(mesh.state), _ptr(mesh.normals) if nv else None,
                                                      _ptr(dverts) if nv else None, nv, _ptr(dchi), _stream(dev)),
               "psr_marching_cubes_backward")
    return dchi


class MarchingCubesFunction(torch.autograd.Function):
    """verts = MC(chi); the backward is main Eq. 6 (dp/dchi = -n)."""

    @staticmethod
    def forward(ctx, chi, iso):
        mesh = marching_cubes(chi, iso)
        ctx.mesh = mesh
        ctx.save_for_backward(chi)
        ctx.mark_non_differentiable(mesh.faces, mesh.normals)
        return mesh.verts, mesh.faces, mesh.normals

    @staticmethod
    def backward(ctx, dverts, dfaces, dnormals):
        (chi,) = ctx.saved_tensors
        return marching_cubes_backward(chi, ctx.mesh, dverts), None


def mesh(chi: torch.Tensor, iso: float = 0.0):
    """(verts, faces, normals) of the level chi = iso; verts carry gradients to chi."""
    return MarchingCubesFunction.apply(chi, iso)
