"""Batched solves through ``psr_run_batched``: many independent oriented point
clouds (mixed resolutions and point counts), one launch per pipeline stage
and resolution for the whole batch.

A :class:`BatchPlan` owns every job's device buffers (chi, saved state,
workspace, gradients), so a batch can be re-run without allocating.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib


@dataclass
class Job:
    points: torch.Tensor           # (P, 3) float32, cuda
    normals: torch.Tensor          # (P, 3) float32, cuda
    res: int
    sigma: float = 2.0
    dchi: torch.Tensor | None = None  # (res, res, res) float32: run the backward too


class BatchPlan:
    """Device buffers for a list of jobs and the ABI job table that points at them."""

    def __init__(self, jobs: list[Job], device: torch.device | None = None):
        if not jobs:
            raise ValueError("empty batch")
        self.jobs = jobs
        dev = device or jobs[0].points.device
        self.device = dev
        self.chi, self.saved, self.ws, self.dp, self.dn = [], [], [], [], []
        self.table = (_lib.PsrJob * len(jobs))()
        for i, j in enumerate(jobs):
            for name, t in (("points", j.points), ("normals", j.normals)):
                if not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3 \
                        or not t.is_contiguous():
                    raise ValueError(f"job {i}: {name} must be a contiguous CUDA float32 (P, 3) tensor")
            P = int(j.points.shape[0])
            r = int(j.res)
            self.chi.append(torch.empty((r, r, r), dtype=torch.float32, device=dev))
            self.saved.append(torch.empty(_lib.saved_bytes(r, P), dtype=torch.uint8, device=dev))
            self.ws.append(torch.empty(_lib.workspace_bytes(r, P), dtype=torch.uint8, device=dev))
            bwd = j.dchi is not None
            if bwd and (j.dchi.shape != (r, r, r) or j.dchi.dtype != torch.float32 or not j.dchi.is_contiguous()):
                raise ValueError(f"job {i}: dchi must be a contiguous float32 ({r},{r},{r}) tensor")
            self.dp.append(torch.empty((P, 3), dtype=torch.float32, device=dev) if bwd else None)
            self.dn.append(torch.empty((P, 3), dtype=torch.float32, device=dev) if bwd else None)
            e = self.table[i]
            e.points = j.points.data_ptr()
            e.normals = j.normals.data_ptr()
            e.npoints = P
            e.res = r
            e.sigma = float(j.sigma)
            e.chi = self.chi[i].data_ptr()
            e.saved = self.saved[i].data_ptr()
            e.dchi = j.dchi.data_ptr() if bwd else None
            e.dpoints = self.dp[i].data_ptr() if bwd else None
            e.dnormals = self.dn[i].data_ptr() if bwd else None
            e.workspace = self.ws[i].data_ptr()
            e.workspace_bytes = self.ws[i].numel()

    def run(self, ctx: _lib.Context | None = None) -> None:
        """Enqueue the whole batch on the current stream (asynchronous)."""
        dev = self.device
        ctx = ctx or _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
        stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _lib.check(_lib.lib().psr_run_batched(ctx.handle, len(self.jobs), self.table, stream), "psr_run_batched")

    def results(self):
        """[(chi, dpoints or None, dnormals or None)] per job."""
        return list(zip(self.chi, self.dp, self.dn))


def run_batched(jobs: list[Job]):
    """Allocate, run once and return [(chi, dpoints, dnormals)] per job."""
    plan = BatchPlan(jobs)
    plan.run()
    return plan.results()
