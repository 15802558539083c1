"""Optimisation-based surface reconstruction with the differentiable solver
(main Sec. 3.2): an oriented point cloud (positions and normals, the only
parameters) is solved into the indicator grid, meshed by Marching Cubes,
sampled uniformly by area, and pulled towards a target point cloud by the
bidirectional Chamfer loss; the gradient flows back through the samples, the
mesh (main Eq. 6) and the solver's adjoint (main Eq. 5).

The schedule follows main Sec. 3.2 and supp Sec. B: the cloud starts as a
sphere, is replaced every 200 iterations by points and normals resampled
from the largest mesh component, and the grid grows coarse to fine (32^3,
64^3, 128^3, 256^3 with sigma 2, 2, 3, 3 and 1000, 1000, 1000, 200
iterations; Adam, learning rate 2e-3 decayed by 0.7 at every new grid size).

Every step (solve, Marching Cubes, sampling, Chamfer, components and all
backwards) runs in ``libpsr.so``; this module draws the random numbers with
PyTorch's generator and marshals buffers. By default an iteration is one
library call (``psr_opt_step``, Adam included); the same loop also runs
through autograd Functions around the separate calls with PyTorch's Adam.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field

import torch

from . import _lib
from . import function as F
from . import mesh as M


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _st(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ctx(dev):
    return _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())


def _size(fn, *args):
    out = ctypes.c_size_t(0)
    _lib.check(fn(*args, ctypes.byref(out)), "workspace size")
    return int(out.value)


def sample_raw(verts, faces, u, vnormals=None, face_weight=None):
    """(points, normals or None, face, bary) of the samples drawn with u [M, 3]."""
    dev = verts.device
    L = _lib.lib()
    nv, nf, m = int(verts.shape[0]), int(faces.shape[0]), int(u.shape[0])
    ws = torch.empty(_size(L.psr_mesh_sample_workspace_bytes, nf), dtype=torch.uint8, device=dev)
    pts = torch.empty((m, 3), dtype=torch.float32, device=dev)
    nrm = torch.empty((m, 3), dtype=torch.float32, device=dev) if vnormals is not None else None
    face = torch.empty((m,), dtype=torch.int32, device=dev)
    bary = torch.empty((m, 3), dtype=torch.float32, device=dev)
    _lib.check(L.psr_mesh_sample(_ctx(dev).handle, _p(verts.detach().contiguous()),
                                 _p(vnormals.contiguous()) if vnormals is not None else None, nv,
                                 _p(faces.contiguous()), nf,
                                 _p(face_weight.contiguous()) if face_weight is not None else None,
                                 _p(u.contiguous()), m, _p(pts), _p(nrm), _p(face), _p(bary), _p(ws),
                                 ctypes.c_size_t(ws.numel()), _st(dev)), "psr_mesh_sample")
    return pts, nrm, face, bary


class SampleFunction(torch.autograd.Function):
    """Points on the mesh; differentiable with respect to the vertices."""

    @staticmethod
    def forward(ctx, verts, faces, u):
        pts, _, face, bary = sample_raw(verts, faces, u)
        ctx.save_for_backward(faces, face, bary)
        ctx.nv = int(verts.shape[0])
        return pts

    @staticmethod
    def backward(ctx, dp):
        faces, face, bary = ctx.saved_tensors
        dev = faces.device
        dv = torch.empty((ctx.nv, 3), dtype=torch.float32, device=dev)
        _lib.check(_lib.lib().psr_mesh_sample_backward(_ctx(dev).handle, _p(faces), ctx.nv, _p(face), _p(bary),
                                                       _p(dp.contiguous()), int(face.shape[0]), _p(dv), _st(dev)),
                   "psr_mesh_sample_backward")
        return dv, None, None


def chamfer_raw(x, y):
    """(loss as a 0-d double tensor, nn_x, d_x, nn_y, d_y)."""
    dev = x.device
    L = _lib.lib()
    nx, ny = int(x.shape[0]), int(y.shape[0])
    ws = torch.empty(_size(L.psr_chamfer_workspace_bytes, nx, ny), dtype=torch.uint8, device=dev)
    nnx = torch.empty((nx,), dtype=torch.int32, device=dev)
    dx = torch.empty((nx,), dtype=torch.float32, device=dev)
    nny = torch.empty((ny,), dtype=torch.int32, device=dev)
    dy = torch.empty((ny,), dtype=torch.float32, device=dev)
    loss = torch.empty((), dtype=torch.float64, device=dev)
    _lib.check(L.psr_chamfer(_ctx(dev).handle, _p(x.detach().contiguous()), nx, _p(y.contiguous()), ny, _p(nnx),
                             _p(dx), _p(nny), _p(dy), _p(loss), _p(ws), ctypes.c_size_t(ws.numel()), _st(dev)),
               "psr_chamfer")
    return loss, nnx, dx, nny, dy


class ChamferFunction(torch.autograd.Function):
    """Bidirectional L2 Chamfer distance (main Eq. 5) of x to the fixed cloud y."""

    @staticmethod
    def forward(ctx, x, y):
        x = x.contiguous()
        loss, nnx, _, nny, _ = chamfer_raw(x, y)
        ctx.save_for_backward(x, y, nnx, nny)
        return loss.to(torch.float32)

    @staticmethod
    def backward(ctx, g):
        x, y, nnx, nny = ctx.saved_tensors
        dev = x.device
        gx = torch.empty_like(x)
        _lib.check(_lib.lib().psr_chamfer_backward(_ctx(dev).handle, _p(x), int(x.shape[0]), _p(y.contiguous()),
                                                   int(y.shape[0]), _p(nnx), _p(nny), _p(gx), _st(dev)),
                   "psr_chamfer_backward")
        return gx * g, None


def components(verts, faces, largest: bool = True):
    """(labels [V] int32, face mask [F] float32 of the largest component or None)."""
    dev = verts.device
    L = _lib.lib()
    nv, nf = int(verts.shape[0]), int(faces.shape[0])
    ws = torch.empty(_size(L.psr_mesh_components_workspace_bytes, nv, nf), dtype=torch.uint8, device=dev)
    lab = torch.empty((nv,), dtype=torch.int32, device=dev)
    w = torch.empty((nf,), dtype=torch.float32, device=dev) if largest else None
    _lib.check(L.psr_mesh_components(_ctx(dev).handle, _p(verts.detach().contiguous()), nv, _p(faces.contiguous()),
                                     nf, _p(lab), _p(w), _p(ws), ctypes.c_size_t(ws.numel()), _st(dev)),
               "psr_mesh_components")
    return lab, w


def resample(verts, faces, vnormals, n: int, gen: torch.Generator):
    """n points and normals uniformly by area on the largest mesh component
    (main Sec. 3.2, "Resampling")."""
    _, w = components(verts, faces)
    u = torch.rand((n, 3), generator=gen, device=verts.device, dtype=torch.float32)
    pts, nrm, _, _ = sample_raw(verts, faces, u, vnormals, w)
    return pts, nrm


def sphere_cloud(n: int, radius: float, gen: torch.Generator, dev) -> tuple[torch.Tensor, torch.Tensor]:
    """The generic initial shape of main Sec. 3.2: n points on a sphere at the
    centre of the domain, with outward normals."""
    d = torch.randn((n, 3), generator=gen, device=dev)
    d = d / d.norm(dim=1, keepdim=True)
    return (0.5 + radius * d).contiguous(), d.contiguous()


@dataclass
class Level:
    res: int
    sigma: float
    iters: int


PAPER_SCHEDULE = [Level(32, 2.0, 1000), Level(64, 2.0, 1000), Level(128, 3.0, 1000), Level(256, 3.0, 200)]


@dataclass
class Result:
    points: torch.Tensor
    normals: torch.Tensor
    verts: torch.Tensor
    faces: torch.Tensor
    history: list = field(default_factory=list)  # (level, iteration, res, Chamfer loss)
    ms_per_iter: dict = field(default_factory=dict)


def step_loss(points, normals, target, res, sigma, u):
    """Chamfer loss of one iteration: solve -> mesh -> samples -> Chamfer."""
    chi = F.solve(points, normals, res, sigma)
    verts, faces, _ = M.mesh(chi)
    x = SampleFunction.apply(verts, faces, u)
    return ChamferFunction.apply(x, target), (verts, faces)


class NativeStep:
    """One iteration in one library call (``psr_opt_step``): solve, Marching
    Cubes, sampling, Chamfer loss, the backward chain and the Adam step run
    in libpsr, so the host issues one call per iteration instead of
    PyTorch's per-operation dispatch and autograd bookkeeping. Holds the
    workspace, sized for a mesh cap that grows when a mesh exceeds it."""

    def __init__(self, dev, npoints: int, ntarget: int, nsamples: int, res: int):
        self.dev, self.P, self.T, self.S, self.res = dev, int(npoints), int(ntarget), int(nsamples), int(res)
        self.vcap, self.tcap = max(4096, 8 * res * res), max(8192, 16 * res * res)
        self.counts = (ctypes.c_int64 * 2)()
        self.loss = torch.zeros((), dtype=torch.float64, device=dev)
        self._alloc()

    def _alloc(self):
        L = _lib.lib()
        nbytes = _size(L.psr_opt_step_workspace_bytes, self.res, self.P, self.T, self.S, self.vcap, self.tcap)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.dev)

    def __call__(self, p, n, moments, t: int, lr: float, target, u, sigma: float,
                 betas=(0.9, 0.999), eps: float = 1e-8) -> torch.Tensor:
        """Update p, n and moments = (m_p, v_p, m_n, v_n) in place; returns the
        Chamfer loss (0-d float64 device tensor, valid until the next call)."""
        L = _lib.lib()
        mp, vp, mn, vn = moments
        for _ in range(3):
            rc = L.psr_opt_step(_ctx(self.dev).handle, _p(p), _p(n), self.P, _p(mp), _p(vp), _p(mn), _p(vn), int(t),
                                float(lr), float(betas[0]), float(betas[1]), float(eps), _p(target), self.T, _p(u),
                                self.S, self.res, float(sigma), self.vcap, self.tcap, _p(self.loss), self.counts,
                                _p(self.ws), ctypes.c_size_t(self.ws.numel()), _st(self.dev))
            if rc == _lib.PSR_ETOOBIG:  # nothing was updated: grow the mesh cap and run the step again
                self.vcap = max(self.vcap, int(self.counts[0]))
                self.tcap = max(self.tcap, int(self.counts[1]))
                self._alloc()
                continue
            _lib.check(rc, "psr_opt_step")
            return self.loss
        raise RuntimeError("psr_opt_step: mesh cap did not settle")


def optimise(target: torch.Tensor, schedule=PAPER_SCHEDULE, npoints: int = 20000, nsamples: int | None = None,
             lr: float = 2e-3, decay: float = 0.7, resample_every: int = 200, seed: int = 0,
             init_radius: float = 0.3, log_every: int = 50, native: bool = True) -> Result:
    """Fit an oriented point cloud to `target` ([T, 3] float32 CUDA points in
    [0, 1)^3) by the coarse-to-fine schedule; returns the final cloud and mesh.

    native: each iteration is one ``psr_opt_step`` call (NativeStep; the
    returned mesh is that of the final cloud); else the same steps through
    the autograd Functions and PyTorch's Adam (the returned mesh is the last
    iteration's)."""
    if native:
        return _optimise_native(target, schedule, npoints, nsamples, lr, decay, resample_every, seed, init_radius,
                                log_every)
    dev = target.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    nsamples = nsamples or int(target.shape[0])
    p, n = sphere_cloud(npoints, init_radius, gen, dev)
    res_hist, ms = [], {}
    verts = faces = None
    for li, lev in enumerate(schedule):
        if li > 0:
            # sample the coarse mesh to start the finer grid
            chi = F.solve(p.detach(), n.detach(), schedule[li - 1].res, schedule[li - 1].sigma)
            mm = M.marching_cubes(chi)
            p, n = resample(mm.verts, mm.faces, mm.normals, npoints, gen)
        p = p.clone().requires_grad_(True)
        n = n.clone().requires_grad_(True)
        opt = torch.optim.Adam([p, n], lr=lr * decay ** li, fused=True)  # one kernel per step
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(lev.iters):
            if it > 0 and it % resample_every == 0:
                with torch.no_grad():
                    chi = F.solve(p, n, lev.res, lev.sigma)
                    mm = M.marching_cubes(chi)
                    pn, nn = resample(mm.verts, mm.faces, mm.normals, npoints, gen)
                p = pn.clone().requires_grad_(True)
                n = nn.clone().requires_grad_(True)
                opt = torch.optim.Adam([p, n], lr=lr * decay ** li, fused=True)  # one kernel per step
            u = torch.rand((nsamples, 3), generator=gen, device=dev, dtype=torch.float32)
            opt.zero_grad(set_to_none=True)
            loss, (verts, faces) = step_loss(p, n, target, lev.res, lev.sigma, u)
            loss.backward()
            opt.step()
            with torch.no_grad():
                p.remainder_(1.0)  # the periodic domain of the solver
            if log_every and (it % log_every == 0 or it == lev.iters - 1):
                res_hist.append((li, it, lev.res, float(loss)))
        torch.cuda.synchronize()
        ms[lev.res] = (time.perf_counter() - t0) / max(1, lev.iters) * 1e3
    return Result(p.detach(), n.detach(), verts.detach(), faces, res_hist, ms)


def _optimise_native(target, schedule, npoints, nsamples, lr, decay, resample_every, seed, init_radius, log_every):
    dev = target.device
    target = target.contiguous()
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    nsamples = nsamples or int(target.shape[0])
    p, n = sphere_cloud(npoints, init_radius, gen, dev)
    res_hist, ms = [], {}
    for li, lev in enumerate(schedule):
        if li > 0:
            # sample the coarse mesh to start the finer grid
            chi = F.solve(p, n, schedule[li - 1].res, schedule[li - 1].sigma)
            mm = M.marching_cubes(chi)
            p, n = resample(mm.verts, mm.faces, mm.normals, npoints, gen)
        p, n = p.detach().clone().contiguous(), n.detach().clone().contiguous()
        step = NativeStep(dev, npoints, int(target.shape[0]), nsamples, lev.res)
        moments = [torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(n), torch.zeros_like(n)]
        t = 0
        lr_l = lr * decay ** li
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(lev.iters):
            if it > 0 and it % resample_every == 0:
                chi = F.solve(p, n, lev.res, lev.sigma)
                mm = M.marching_cubes(chi)
                pn, nn = resample(mm.verts, mm.faces, mm.normals, npoints, gen)
                p, n = pn.contiguous(), nn.contiguous()
                for m in moments:
                    m.zero_()
                t = 0  # a fresh optimiser for the resampled cloud
            u = torch.rand((nsamples, 3), generator=gen, device=dev, dtype=torch.float32)
            t += 1
            loss = step(p, n, moments, t, lr_l, target, u, lev.sigma)
            if log_every and (it % log_every == 0 or it == lev.iters - 1):
                res_hist.append((li, it, lev.res, float(loss)))
        torch.cuda.synchronize()
        ms[lev.res] = (time.perf_counter() - t0) / max(1, lev.iters) * 1e3
    chi = F.solve(p, n, schedule[-1].res, schedule[-1].sigma)
    mm = M.marching_cubes(chi)
    return Result(p, n, mm.verts, mm.faces, res_hist, ms)
