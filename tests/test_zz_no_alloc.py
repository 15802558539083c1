"""psr_forward_static (the forward that allocates nothing, its workspace and
saved state in a static device array) against psr_forward through the C ABI:
two calls in a row, the second smaller, each equal to the allocating entry
point's result (the same kernels, so within the 1e-5 chi bar and in practice
bit for bit), and a problem beyond the array's size refused before any launch."""
import ctypes

import numpy as np
import pytest

import psr_synth as S
from gpu_common import announce, host, max_rel, require_gpu, to_dev, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _static(L, ctx, pts, nrm, res, sigma, chi, dev):
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    return L.psr_forward_static(ctx.handle, p(pts), p(nrm), int(pts.shape[0]), res, float(sigma), p(chi), st)


def test_static_forward_equals_forward_twice(dev):
    from paper_2106_03452_amd import _lib
    from paper_2106_03452_amd import function as F
    L, ctx = _lib.lib(), _lib.context(0)
    cases = [S.config_c2(), S.tiny_case(11, 64, 3000, kind="torus")]  # 128^3 / 20k, then 64^3 / 3k
    for sh in cases:
        announce(f"static forward res={sh.res} P={sh.P}")
        pts, nrm = to_dev(sh.points, dev), to_dev(sh.normals, dev)
        chi_s = torch.full((sh.res,) * 3, float("nan"), dtype=torch.float32, device=dev)
        assert _static(L, ctx, pts, nrm, sh.res, sh.sigma, chi_s, dev) == 0
        chi_f, saved = F.forward(pts, nrm, sh.res, sh.sigma)
        assert F.status(saved) == 0
        e = max_rel(host(chi_s), host(chi_f))
        print(f"static vs allocating forward res={sh.res} P={sh.P}: max rel diff {e:.2e}, "
              f"bitwise equal {torch.equal(chi_s, chi_f)}")
        assert e <= 1e-5


def test_static_forward_refuses_too_large(dev):
    from paper_2106_03452_amd import _lib
    L, ctx = _lib.lib(), _lib.context(0)
    announce("static forward beyond the static scratch")
    sh = S.tiny_case(12, 256, 1000, kind="sphere")
    pts, nrm = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    chi = torch.zeros((256,) * 3, dtype=torch.float32, device=dev)
    assert _static(L, ctx, pts, nrm, 256, 2.0, chi, dev) == _lib.PSR_ETOOBIG
    torch.cuda.synchronize()
    assert not chi.any()  # nothing was launched
    # at 128^3 the limit falls at 57,036 points
    assert _lib.workspace_bytes(128, 57036) + _lib.saved_bytes(128, 57036) <= (64 << 20)
    assert _lib.workspace_bytes(128, 57037) + _lib.saved_bytes(128, 57037) > (64 << 20)
    big = S.tiny_case(13, 128, 57037, kind="sphere")
    p2, n2 = to_dev(big.points, dev), to_dev(big.normals, dev)
    chi2 = torch.zeros((128,) * 3, dtype=torch.float32, device=dev)
    assert _static(L, ctx, p2, n2, 128, 2.0, chi2, dev) == _lib.PSR_ETOOBIG
