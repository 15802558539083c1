"""Batched solves (psr_run_batched): every job's chi and gradients equal the
same job solved alone (1e-6 relative: only the LDS-atomic summation order of
the splat may differ), and a few jobs against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, host, l2_rel, max_rel, require_gpu, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _mixed_jobs(dev, n, seed, with_bwd=True, res_choices=(16, 32, 64), pmax=4000):
    from paper_2106_03452_amd.batch import Job
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs, shapes = [], []
    for i in range(n):
        res = int(rng.choice(res_choices))
        P = int(round(np.exp(rng.uniform(np.log(50), np.log(pmax)))))
        sh = S.random_shape(rng, res, P)
        G = rng.standard_normal((res, res, res)).astype(np.float32) if (with_bwd and i % 3 != 1) else None
        jobs.append(Job(to_dev(sh.points, dev), to_dev(sh.normals, dev), res, 2.0,
                        to_dev(G, dev) if G is not None else None))
        shapes.append((sh, G))
    return jobs, shapes


@pytest.mark.parametrize("n,res_choices", [(30, (16, 32, 64)), (29, (32,)), (12, (64, 128)), (3, (256,))])
def test_batch_equals_solo(dev, n, res_choices):
    announce(f"batch of {n} jobs res {res_choices} vs solo")
    from paper_2106_03452_amd import function as F
    from paper_2106_03452_amd.batch import BatchPlan
    # 29 jobs of one resolution span two launch chunks (24 + 5)
    jobs, shapes = _mixed_jobs(dev, n, n, res_choices=res_choices)
    plan = BatchPlan(jobs)
    plan.run()
    torch.cuda.synchronize()
    for i, (j, (chi_b, dp_b, dn_b)) in enumerate(zip(jobs, plan.results())):
        chi_s, saved = F.forward(j.points, j.normals, j.res, j.sigma)
        assert max_rel(host(chi_b), host(chi_s)) < 1e-6, i
        if j.dchi is not None:
            dp_s, dn_s = F.backward(chi_s, saved, j.dchi, j.points.shape[0], j.res, j.sigma)
            assert l2_rel(host(dp_b), host(dp_s)) < 1e-6, i
            assert l2_rel(host(dn_b), host(dn_s)) < 1e-6, i
        else:
            assert dp_b is None and dn_b is None


@pytest.mark.parametrize("n,res_choices,pmax", [(6, (16, 32, 64), 4000), (6, (64, 128), 50000)])
def test_batch_against_oracle(dev, n, res_choices, pmax):
    announce(f"batch of {n} jobs res {res_choices} vs oracle")
    from paper_2106_03452_amd.batch import BatchPlan
    jobs, shapes = _mixed_jobs(dev, n, 1, res_choices=res_choices, pmax=pmax)
    plan = BatchPlan(jobs)
    plan.run()
    torch.cuda.synchronize()
    for (sh, G), (chi_b, dp_b, dn_b) in zip(shapes, plan.results()):
        ref, aux = oracle.forward(sh.points, sh.normals, sh.res, sh.sigma)
        assert max_rel(host(chi_b), ref) < 1e-5
        if G is not None:
            dc, dn = oracle.backward(aux, G.astype(np.float64))
            assert l2_rel(host(dp_b), dc) < 1e-4 and l2_rel(host(dn_b), dn) < 1e-4


def test_batch_rerun_is_stable(dev):
    from paper_2106_03452_amd.batch import BatchPlan
    jobs, _ = _mixed_jobs(dev, 10, 2)
    plan = BatchPlan(jobs)
    plan.run()
    first = [host(c) for c in plan.chi]
    plan.run()
    torch.cuda.synchronize()
    for a, c in zip(first, plan.chi):
        assert max_rel(host(c), a) < 1e-6
