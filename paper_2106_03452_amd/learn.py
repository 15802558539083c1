"""Learning-based reconstruction with the DPSR loss (main Sec. 3.3, Eqs. 7-9),
in miniature: a point network predicts k offsets per input point and a normal
for every displaced point, the library solves for the indicator grid, and the
loss is the mean squared error against a ground-truth grid.

The network (PyTorch modules, trained with PyTorch's optimiser) is the model
around the solver, not the hot path: every step of the solve and of its
adjoint runs in ``libpsr.so`` through :func:`function.solve`, and a batch of
shapes is solved with one launch per pipeline stage through
:func:`solve_batch`.

Architecture, after main Sec. 3.3 with the convolutional point encoder cut
down to one layer: per-point features (an MLP of the coordinates) are averaged
into a feature grid, each cell mixes its features with the mean of its 3^3
neighbourhood through one learned linear map (local context; a full 3D
convolution's weight gradient cost 80 % of the step in MIOpen), the grid is read
back at any point by trilinear interpolation (phi), an MLP f predicts the k
offsets of each input point from (c, phi(c)) (Eq. 7), and a second MLP g
predicts the normal of each displaced point from (c^, phi(c^)) (Eq. 8); f and
g share no weights; the predicted normal is added to the direction from the
input cloud's centroid (a geometric initialisation in the spirit of the
paper's, which starts from the input points: untrained random normals would
give a badly conditioned first solve). The ground-truth grid comes from the
same solver on a dense clean sample of the shape (main Sec. 3.3, "Training
and Inference").
"""
from __future__ import annotations

import ctypes

import torch
import torch.nn.functional as Fn

from . import _lib
from . import function as F


def _mlp(d_in, hidden, d_out, layers):
    mods, d = [], d_in
    for _ in range(layers):
        mods += [torch.nn.Linear(d, hidden), torch.nn.ReLU()]
        d = hidden
    mods.append(torch.nn.Linear(d, d_out))
    return torch.nn.Sequential(*mods)


class OffsetNormalNet(torch.nn.Module):
    """Predicts (c^, n^): k displaced copies of every input point and their normals."""

    def __init__(self, k: int = 7, feat: int = 32, grid: int = 32, hidden: int = 32, layers: int = 3,
                 max_offset: float = 0.05, radial_prior: bool = True):
        super().__init__()
        self.k, self.feat, self.grid, self.max_offset = k, feat, grid, max_offset
        self.radial_prior = radial_prior
        self.enc = _mlp(3, hidden, feat, 2)
        self.mix = torch.nn.Linear(2 * feat, feat)
        self.f = _mlp(3 + feat, hidden, 3 * k, layers)
        self.g = _mlp(3 + feat, hidden, 3, layers)

    def feature_grid(self, c):
        """c [B, N, 3] in [0, 1) -> feature grid [B, F, G, G, G] (mean of the point features per cell)."""
        B, N, _ = c.shape
        G = self.grid
        h = self.enc(c)  # [B, N, F]
        cell = torch.clamp((c.detach() * G).floor().long(), 0, G - 1)
        idx = (cell[..., 0] * G + cell[..., 1]) * G + cell[..., 2]  # [B, N]
        idx = idx + (torch.arange(B, device=c.device) * G ** 3)[:, None]
        flat = h.reshape(B * N, self.feat)
        acc = torch.zeros(B * G ** 3, self.feat, device=c.device, dtype=c.dtype).index_add_(0, idx.reshape(-1), flat)
        cnt = torch.zeros(B * G ** 3, device=c.device, dtype=c.dtype).index_add_(
            0, idx.reshape(-1), torch.ones(B * N, device=c.device, dtype=c.dtype))
        grid = (acc / cnt.clamp(min=1.0)[:, None]).reshape(B, G, G, G, self.feat)
        # local context: each cell mixes its features with the mean over its
        # 3^3 neighbourhood (one learned linear map per cell)
        nb = Fn.avg_pool3d(grid.permute(0, 4, 1, 2, 3), 3, stride=1, padding=1, count_include_pad=False)
        out = torch.relu(self.mix(torch.cat([grid, nb.permute(0, 2, 3, 4, 1)], -1)))
        return out.permute(0, 4, 1, 2, 3).contiguous()

    def sample(self, grid, x):
        """Trilinear interpolation of the feature grid at x [B, M, 3] (cell centres at (i + 0.5)/G)."""
        B, M, _ = x.shape
        # grid_sample's last coordinate indexes the last grid axis: reverse (x0, x1, x2)
        g = (x * 2.0 - 1.0).flip(-1).reshape(B, M, 1, 1, 3)
        out = Fn.grid_sample(grid, g, mode="bilinear", padding_mode="border", align_corners=False)
        return out.reshape(B, self.feat, M).transpose(1, 2)

    def forward(self, c):
        grid = self.feature_grid(c)
        phi = self.sample(grid, c)
        B, N, _ = c.shape
        d = torch.tanh(self.f(torch.cat([c, phi], -1))) * self.max_offset  # Eq. 7
        chat = (c[:, :, None, :] + d.reshape(B, N, self.k, 3)).reshape(B, N * self.k, 3)
        phi2 = self.sample(grid, chat)
        nhat = self.g(torch.cat([chat, phi2], -1))  # Eq. 8
        if self.radial_prior:
            # geometric initialisation: before training, normals point away from
            # the cloud's centroid, so the first solves are well conditioned
            nhat = nhat + (chat - c.mean(1, keepdim=True))
        return chat, nhat


class SolveBatch(torch.autograd.Function):
    """chi of every shape of a batch (one psr_run_batched call per direction:
    the forwards of the whole batch, later the backwards)."""

    @staticmethod
    def forward(ctx, res, sigma, *tensors):
        n = len(tensors) // 2
        pts = [t.detach().contiguous() for t in tensors[:n]]
        nrm = [t.detach().contiguous() for t in tensors[n:]]
        dev = pts[0].device
        lc = _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
        chis, saveds, wss = [], [], []
        table = (_lib.PsrJob * n)()
        for i, (p, q) in enumerate(zip(pts, nrm)):
            P = int(p.shape[0])
            chis.append(torch.empty((res, res, res), dtype=torch.float32, device=dev))
            saveds.append(torch.empty(_lib.saved_bytes(res, P), dtype=torch.uint8, device=dev))
            wss.append(torch.empty(_lib.workspace_bytes(res, P), dtype=torch.uint8, device=dev))
            e = table[i]
            e.points, e.normals, e.npoints, e.res, e.sigma = p.data_ptr(), q.data_ptr(), P, res, float(sigma)
            e.chi, e.saved, e.workspace = chis[i].data_ptr(), saveds[i].data_ptr(), wss[i].data_ptr()
            e.workspace_bytes = wss[i].numel()
        st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _lib.check(_lib.lib().psr_run_batched(lc.handle, n, table, st), "psr_run_batched")
        ctx.res, ctx.sigma, ctx.n = res, sigma, n
        ctx.P = [int(p.shape[0]) for p in pts]
        ctx.wss = wss
        ctx.save_for_backward(*chis, *saveds)
        return tuple(chis)

    @staticmethod
    def backward(ctx, *dchis):
        n = ctx.n
        chis, saveds = ctx.saved_tensors[:n], ctx.saved_tensors[n:]
        dev = chis[0].device
        lc = _lib.context(dev.index if dev.index is not None else torch.cuda.current_device())
        table = (_lib.PsrJob * n)()
        dps, dns, keep = [], [], []
        for i in range(n):
            g = (dchis[i] if dchis[i] is not None else torch.zeros_like(chis[i])).contiguous()
            keep.append(g)
            dps.append(torch.empty((ctx.P[i], 3), dtype=torch.float32, device=dev))
            dns.append(torch.empty((ctx.P[i], 3), dtype=torch.float32, device=dev))
            e = table[i]
            e.npoints, e.res, e.sigma = ctx.P[i], ctx.res, float(ctx.sigma)
            e.chi, e.saved, e.dchi = chis[i].data_ptr(), saveds[i].data_ptr(), g.data_ptr()
            e.dpoints, e.dnormals = dps[i].data_ptr(), dns[i].data_ptr()
            e.workspace, e.workspace_bytes = ctx.wss[i].data_ptr(), ctx.wss[i].numel()
            e.stages = _lib.PSR_JOB_BACKWARD
        st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _lib.check(_lib.lib().psr_run_batched(lc.handle, n, table, st), "psr_run_batched")
        return (None, None, *dps, *dns)


def solve_batch(points: list, normals: list, res: int, sigma: float = 2.0) -> list:
    """Differentiable chi of each (points, normals) pair, solved as one batch."""
    return list(SolveBatch.apply(int(res), float(sigma), *points, *normals))


def dpsr_loss(chat, nhat, chi_gt, res: int, sigma: float = 2.0, batched: bool = True):
    """main Eq. 9: the mean over the batch of the mean squared error between the
    solved grid of each predicted oriented cloud and its ground-truth grid."""
    B = chat.shape[0]
    pts = [chat[b].contiguous() for b in range(B)]
    nrm = [nhat[b].contiguous() for b in range(B)]
    if batched:
        chis = solve_batch(pts, nrm, res, sigma)
    else:
        chis = [F.solve(p, q, res, sigma) for p, q in zip(pts, nrm)]
    return sum(((c - g) ** 2).mean() for c, g in zip(chis, chi_gt)) / B


def train_step(model, opt, c_in, chi_gt, res: int, sigma: float = 2.0):
    """One optimisation step of the network on a batch: (loss value, tensor)."""
    opt.zero_grad(set_to_none=True)
    chat, nhat = model(c_in)
    loss = dpsr_loss(chat, nhat, chi_gt, res, sigma)
    loss.backward()
    opt.step()
    return loss.detach()
