"""Serving engine on the GPU: every request's chi and gradients, computed in a
mix of overlapping batches on several streams, equal the same request solved
alone (1e-6 relative: only the splat's LDS-atomic summation order differs)."""
import numpy as np
import pytest

import psr_synth as S
from gpu_common import announce, host, l2_rel, max_rel, require_gpu, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.mark.parametrize("n,res_choices,pmax,streams", [(48, (16, 32, 64), 6000, 3),
                                                         (16, (64, 128, 256), 200000, 4)])
def test_results_same_alone_and_in_the_mix(dev, n, res_choices, pmax, streams):
    """Small grids with many requests per batch, and the serving stream's own
    grid sizes and point counts (64/128/256, up to 200k points: the plane and
    row passes of every size overlap on several streams)."""
    announce(f"serve: {n} requests res {res_choices}, {streams} streams, vs solo")
    from paper_2106_03452_amd import function as F
    from paper_2106_03452_amd.serve import Engine, GpuBackend, Request, drive
    rng = np.random.Generator(np.random.PCG64(5))
    reqs, inputs = [], []
    for i in range(n):
        res = int(rng.choice(res_choices))
        P = int(round(np.exp(rng.uniform(np.log(100), np.log(pmax)))))
        sh = S.random_shape(rng, res, P)
        bwd = bool(rng.uniform() < 0.5)
        pts, nrm = to_dev(sh.points, dev), to_dev(sh.normals, dev)
        G = to_dev(rng.standard_normal((res, res, res)), dev) if bwd else None
        r = Request(i, res, P, bwd, arrival=float(i) * 2e-5, points=pts, normals=nrm, dchi=G,
                    out_chi=torch.empty((res, res, res), device=dev),
                    out_dpoints=torch.empty((P, 3), device=dev) if bwd else None,
                    out_dnormals=torch.empty((P, 3), device=dev) if bwd else None)
        reqs.append(r)
    be = GpuBackend(0, num_streams=streams)
    eng = Engine(be, {r: pmax for r in res_choices}, hbm_budget=(2 << 30) if pmax <= 6000 else (24 << 30),
                 max_batch=8)
    drive(eng, reqs)
    torch.cuda.synchronize()
    assert len(eng.finished) == n and not eng.rejected
    assert all(r.error is None and r.latency >= 0 for r in eng.finished)
    for r in reqs:
        chi, saved = F.forward(r.points, r.normals, r.res, 2.0)
        assert max_rel(host(r.out_chi), host(chi)) < 1e-6, r.rid
        if r.backward:
            dp, dn = F.backward(chi, saved, r.dchi, r.npoints, r.res, 2.0)
            assert l2_rel(host(r.out_dpoints), host(dp)) < 1e-6, r.rid
            assert l2_rel(host(r.out_dnormals), host(dn)) < 1e-6, r.rid
