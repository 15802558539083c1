"""Parity at the benchmark workloads, through the C ABI, at full size.

C2: 128^3, 20,000 points (torus U sphere, jittered), loss mean((chi - chi_t)^2)
    with chi_t from the clean points; chi, dL/dpoints, dL/dnormals against the
    FP64 oracle, and 64 + 64 gradient entries against FP64 central finite
    differences of the oracle (tests/golden/c2_fd.json).
C3: 256^3, 100,000 points on a superellipsoid with noisy normals, the same
    loss with chi_t from the clean normals; everything against the oracle.
    The same cloud on 512^3 (the largest grid) against stored oracle samples.
Each side computes its own target chi_t and loss gradient G.
"""
import json
import os

import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, host, l2_rel, max_rel, require_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _run_gpu(sh, dev, G_given=None):
    """GPU forward + backward. The loss gradient is the GPU's own G = 2(chi - chi_t)/N,
    or, when G_given is passed, that array (to isolate the adjoint's own error)."""
    from paper_2106_03452_amd import function as F
    chi_t, _ = F.forward(to_dev(sh.points_clean, dev), to_dev(sh.normals_clean, dev), sh.res, sh.sigma)
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), sh.res, sh.sigma)
    assert F.status(saved) == 0
    G = 2.0 * (chi - chi_t) / chi.numel() if G_given is None else to_dev(G_given, dev)
    dp, dn = F.backward(chi, saved, G, sh.P, sh.res, sh.sigma)
    torch.cuda.synchronize()
    return host(chi), host(dp), host(dn)


def _run_oracle(sh, G_f32=False):
    chi_t, _ = oracle.forward(sh.points_clean, sh.normals_clean, sh.res, sh.sigma)
    chi, aux = oracle.forward(sh.points, sh.normals, sh.res, sh.sigma)
    G = 2.0 * (chi - chi_t) / chi.size
    if G_f32:
        G = G.astype(np.float32).astype(np.float64)
    dc, dn = oracle.backward(aux, G)
    return chi, dc, dn, G


def _fd_check(fd, dp_g, dn_g):
    """Gradient entries against FP64 central differences of the oracle: per
    kind, the relative L2 error over the sampled entries and the worst entry
    relative to max(|g_FD|, 1e-3 |g|_inf)."""
    out = {}
    for kind, g_all in (("points", dp_g), ("normals", dn_g)):
        ent = [e for e in fd["entries"] if e["which"] == kind]
        g = np.array([g_all[e["i"], e["a"]] for e in ent])
        f = np.array([e["fd"] for e in ent])
        inf = fd["grad_inf_" + kind]
        l2 = float(np.linalg.norm(g - f) / np.linalg.norm(f))
        worst = float(np.max(np.abs(g - f) / np.maximum(np.abs(f), 1e-3 * inf)))
        out[kind] = (l2, worst)
    return out


def test_c2_forward_backward_and_fd(dev):
    announce("C2 128^3 20k fwd+bwd")
    sh = S.config_c2()
    chi_g, dp_g, dn_g = _run_gpu(sh, dev)
    chi_r, dc_r, dn_r, G_r = _run_oracle(sh, G_f32=True)
    e_chi, e_dc, e_dn = max_rel(chi_g, chi_r), l2_rel(dp_g, dc_r), l2_rel(dn_g, dn_r)
    print(f"C2 end-to-end e_chi={e_chi:.3e} e_dpoints={e_dc:.3e} e_dnormals={e_dn:.3e}")
    assert e_chi < 1e-5 and e_dc < 1e-4 and e_dn < 1e-4
    _, dp_o, dn_o = _run_gpu(sh, dev, G_given=G_r)
    a_dc, a_dn = l2_rel(dp_o, dc_r), l2_rel(dn_o, dn_r)
    print(f"C2 adjoint alone (oracle G as input) e_dpoints={a_dc:.3e} e_dnormals={a_dn:.3e}")
    assert a_dc < 1e-4 and a_dn < 1e-4
    fd = json.load(open(os.path.join(GOLDEN, "c2_fd.json")))
    # end to end (the GPU's own FP32 loss gradient G): the sampled entries as a set
    for kind, (l2, worst) in _fd_check(fd, dp_g, dn_g).items():
        print(f"C2 FD end to end, {kind}: L2 rel {l2:.3e} over 64 entries; worst entry {worst:.3e}")
        assert l2 <= 1e-4
    # the adjoint alone (the oracle's G rounded to FP32 as input): every sampled
    # entry within 1e-4 max(|g_FD|, 1e-3 |g|_inf)
    for kind, (l2, worst) in _fd_check(fd, dp_o, dn_o).items():
        print(f"C2 FD adjoint alone, {kind}: L2 rel {l2:.3e}; worst entry {worst:.3e}")
        assert l2 <= 1e-4 and worst <= 1e-4


@pytest.mark.timeout(900)
def test_c3_forward_backward_vs_oracle(dev):
    announce("C3 256^3 100k fwd+bwd")
    sh = S.config_c3()
    chi_g, dp_g, dn_g = _run_gpu(sh, dev)
    chi_r, dc_r, dn_r, _ = _run_oracle(sh)
    e_chi, e_dc, e_dn = max_rel(chi_g, chi_r), l2_rel(dp_g, dc_r), l2_rel(dn_g, dn_r)
    print(f"C3 e_chi={e_chi:.3e} e_dpoints={e_dc:.3e} e_dnormals={e_dn:.3e}")
    assert e_chi < 1e-5 and e_dc < 1e-4 and e_dn < 1e-4


def test_c2_with_half_outliers(dev):
    """C2 with 50 % of the points replaced by uniform outliers with short random
    normals: the worst locality for the binning and the splat; chi and both
    gradients against the oracle (dense random loss gradient)."""
    from paper_2106_03452_amd import function as F
    announce("C2 with 50% outliers 128^3 fwd+bwd")
    sh = S.config_c2_outliers()
    G = S.loss_gradient(128, 128)
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 128, sh.sigma)
    assert F.status(saved) == 0
    dp, dn = F.backward(chi, saved, to_dev(G, dev), sh.P, 128, sh.sigma)
    ref, aux = oracle.forward(sh.points, sh.normals, 128, sh.sigma)
    dc_r, dn_r = oracle.backward(aux, G)
    e_chi, e_dc, e_dn = max_rel(host(chi), ref), l2_rel(host(dp), dc_r), l2_rel(host(dn), dn_r)
    print(f"C2 + outliers e_chi={e_chi:.3e} e_dpoints={e_dc:.3e} e_dnormals={e_dn:.3e}")
    assert e_chi < 1e-5 and e_dc < 1e-4 and e_dn < 1e-4


def test_c3_cloud_at_512_vs_stored_oracle(dev):
    """The largest grid: the C3 cloud (100k points) on 512^3 against FP64 oracle
    samples written by tests/golden/make_c3_512.py (chi at 8192 voxels over
    max|chi| of the whole grid, mu and c, both gradients at 4096 points; the
    loss gradient is psr_synth.loss_gradient(512, 512) on both sides)."""
    from paper_2106_03452_amd import function as F
    g = np.load(os.path.join(GOLDEN, "c3_512_samples.npz"))
    sh = S.config_c3()
    announce("C3 cloud at 512^3 vs stored oracle samples")
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 512, sh.sigma)
    assert F.status(saved) == 0
    G = to_dev(S.loss_gradient(512, 512), dev)
    dp, dn = F.backward(chi, saved, G, sh.P, 512, sh.sigma)
    torch.cuda.synchronize()
    del G
    sc = F.scalars(saved)
    c = abs(float(g["cscale"]))
    chi_s = host(chi.reshape(-1)[torch.as_tensor(g["vox"], device=dev)])
    e_chi = float(np.abs(chi_s.astype(np.float64) - g["chi"]).max() / float(g["chi_max"]))
    pts = torch.as_tensor(g["pts"], device=dev)
    e_dc, e_dn = l2_rel(host(dp[pts]), g["dpoints"]), l2_rel(host(dn[pts]), g["dnormals"])
    print(f"C3 cloud at 512^3: e_chi={e_chi:.3e} (8192 voxels) e_dpoints={e_dc:.3e} e_dnormals={e_dn:.3e} (4096 points)")
    assert e_chi < 1e-5
    assert abs(sc["mean"] - float(g["mu"])) <= 1e-5 * c
    assert abs(sc["cscale"] - float(g["cscale"])) <= 1e-5 * c
    assert e_dc < 1e-4 and e_dn < 1e-4


def test_c1_sphere_is_an_indicator(dev):
    """C1 at 32^3: inside the sphere chi is flat near -0.58, outside +0.5 (loose sanity, not parity)."""
    from paper_2106_03452_amd import function as F
    sh = S.config_c1()
    chi, _ = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 32, 2.0)
    chi = host(chi).ravel()
    x = np.indices((32, 32, 32)).reshape(3, -1).T / 32
    d = np.linalg.norm(x - 0.5, axis=1)
    inside, outside = chi[d < 0.3 - 3 / 32], chi[d > 0.3 + 3 / 32]
    assert -0.65 <= inside.mean() <= -0.50 and inside.std() < 0.03
    assert abs(outside.mean() - 0.5) < 0.01


@pytest.mark.parametrize("res,which", [(128, "c4_sphere"), (64, "c4_torus"), (256, "c3")])
def test_loss_correlated_with_chi(dev, res, which):
    """Loss mean(chi^2), so G = 2 chi / N: the derivative through chi'(0,0,0)
    (Eq. 4) puts a point source -Q delta_0 with Q = sum(G chi)/c into the
    cotangent, about sqrt(N) times the rest of it in L2. Its response is
    read at the points from the FP64-built table, so the gradients keep the
    1e-4 bar (an FP32 transform of the spike gave 1.4e-4 at 128^3)."""
    from paper_2106_03452_amd import function as F
    if which == "c3":
        sh = S.config_c3()
    else:
        kind = which.split("_")[1]
        sh = next(s for s in S.config_c4() if s.res == res and s.kind == kind and s.P > 10000)
    announce(f"loss mean(chi^2) res={res} {which} P={sh.P}")
    chi, saved = F.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), res, sh.sigma)
    dp, dn = F.backward(chi, saved, (2.0 * chi / chi.numel()).contiguous(), sh.P, res, sh.sigma)
    ref, aux = oracle.forward(sh.points, sh.normals, res, sh.sigma)
    dc_r, dn_r = oracle.backward(aux, 2.0 * ref / ref.size)
    e_chi, e_dc, e_dn = max_rel(host(chi), ref), l2_rel(host(dp), dc_r), l2_rel(host(dn), dn_r)
    print(f"mean(chi^2) {which} {res}^3: e_chi={e_chi:.3e} e_dpoints={e_dc:.3e} e_dnormals={e_dn:.3e}")
    assert e_chi < 1e-5 and e_dc < 1e-4 and e_dn < 1e-4
