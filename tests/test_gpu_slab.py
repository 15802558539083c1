"""GPU parity of the slab-decomposed forward (psr_slab_forward, through its C
ABI) against the FP64 oracle, and its properties at 1024^3, where the oracle
does not fit in memory.

Bars as for the single-grid forward: chi' and c within 1e-5 of max|chi'|, chi
within 1e-5 times the normalisation's amplification max|chi|/m (>= 1).
At 1024^3: the slab passes on a single Fourier mode against its closed form
(main Eq. 3), chi bitwise the same for 1, 8 and 64 slabs, and the two
constraints of main Eq. 2 (|chi(0)| = m, mean of chi at the points = 0).
"""
import os

import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, host, max_rel, require_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

E_CHI = 1e-5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


@pytest.fixture(scope="module")
def slab(dev):
    import paper_2106_03452_amd as p
    from paper_2106_03452_amd import slab as sl
    p.context(0)
    return sl


def _case(seed, res, P, kind, sigma):
    return S.tiny_case(seed, res, P, sigma, kind=kind)


# (res, P, kind, sigma, slabs): every slab count from one plane per slab
# (res 16 with 16 slabs) to one slab
CASES = [(16, 300, "sphere", 2.0, 2), (16, 513, "uniform", 1.0, 16), (32, 2049, "torus", 2.0, 4),
         (32, 700, "small", 2.0, 1), (64, 4000, "sphere", 3.0, 8), (64, 10007, "uniform", 2.0, 64),
         (128, 3000, "torus", 2.0, 4), (128, 20000, "sphere", 2.0, 16), (256, 20000, "torus", 2.0, 8)]


@pytest.mark.parametrize("res,P,kind,sigma,slabs", CASES)
def test_slab_forward_matches_oracle(slab, dev, res, P, kind, sigma, slabs):
    announce(f"slab forward res={res} P={P} kind={kind} sigma={sigma} slabs={slabs}")
    sh = _case(res * 7 + P, res, P, kind, sigma)
    chi, sc = slab.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), res, sigma, slabs)
    ref, aux = oracle.forward(sh.points, sh.normals, res, sigma)
    assert sc["status"] == 0 and aux["status"] == "ok"
    chi_g = host(chi)
    chip_g = chi_g / sc["scale"] + sc["mu"]
    span = np.abs(aux["chi_prime"]).max()
    amp = max(1.0, np.abs(ref).max() / aux["m"])
    e_p, e_c = max_rel(chip_g, aux["chi_prime"]), max_rel(chi_g, ref)
    print(f"slab res={res} slabs={slabs}: e_chi'={e_p:.2e} e_chi={e_c:.2e} (amplification {amp:.2f})")
    assert e_p < E_CHI
    assert abs(sc["cscale"] - aux["cscale"]) < E_CHI * span
    assert abs(sc["mu"] - aux["mu"]) < E_CHI * span
    assert e_c < E_CHI * amp


def test_slab_count_does_not_change_the_result(slab, dev):
    announce("slab counts 1..64 at 128^3, bitwise")
    sh = S.tiny_case(31, 128, 30000, 2.0, kind="torus")
    p, n = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    chi1, sc1 = slab.forward(p, n, 128, 2.0, 1)
    for g in (2, 4, 8, 16, 32, 64):
        chi, sc = slab.forward(p, n, 128, 2.0, g)
        assert torch.equal(chi, chi1), g
        assert sc == sc1, g


def test_slab_matches_single_grid_solver(slab, dev):
    from paper_2106_03452_amd import function as F
    announce("slab vs single-grid solver, C3 cloud at 256^3")
    sh = S.config_c3()
    p, n = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    chi_s, sc = slab.forward(p, n, 256, sh.sigma, 8)
    chi_f, saved = F.forward(p, n, 256, sh.sigma)
    e = float((chi_s - chi_f).abs().max() / chi_f.abs().max())
    print(f"slab vs single grid at 256^3: {e:.2e}")
    assert e < E_CHI
    assert abs(sc["mu"] - F.scalars(saved)["mean"]) < E_CHI * abs(sc["cscale"])


def test_slab_c3_cloud_at_512_vs_stored_oracle(slab, dev):
    """The C3 cloud on 512^3 in 4 slabs against the FP64 oracle samples that
    tests/golden/make_c3_512.py wrote (chi at 8192 voxels, mu, c)."""
    g = np.load(os.path.join(GOLDEN, "c3_512_samples.npz"))
    sh = S.config_c3()
    announce("slab C3 cloud at 512^3 vs stored oracle samples")
    chi, sc = slab.forward(to_dev(sh.points, dev), to_dev(sh.normals, dev), 512, sh.sigma, 4)
    assert sc["status"] == 0
    c = abs(float(g["cscale"]))
    chi_s = host(chi.reshape(-1)[torch.as_tensor(g["vox"], device=dev)])
    e_chi = float(np.abs(chi_s - g["chi"]).max() / float(g["chi_max"]))
    print(f"slab C3 at 512^3: e_chi={e_chi:.3e} (8192 voxels)")
    assert e_chi < E_CHI
    assert abs(sc["mu"] - float(g["mu"])) <= 1e-5 * c
    assert abs(sc["cscale"] - float(g["cscale"])) <= 1e-5 * c


def test_slab_single_mode_closed_form_at_1024(slab, dev):
    """v_d = cos(2 pi k.j / r) on 1024^3 through the slab passes: chi' =
    g(k) k_d sin(2 pi k.j / r) / (2 pi |k|^2) (main Eq. 3 on one mode). The
    FP32 rounding noise of the transforms is amplified by 1/|k'|^2 at low
    wavenumbers, so the bar holds for a mode whose own factor k_d / |k|^2 is
    not much smaller than that (k_d = 201 here, as at 512^3)."""
    res, sigma, k, d = 1024, 2.0, (100, -3, 201), 2
    announce(f"slab closed form res={res} k={k} d={d} slabs=8")
    j = torch.arange(res, device=dev, dtype=torch.float64) * (2 * np.pi / res)
    th = k[0] * j[:, None, None] + k[1] * j[None, :, None] + k[2] * j[None, None, :]
    v = torch.zeros((3, res, res, res), dtype=torch.float32, device=dev)
    v[d] = torch.cos(th).float()
    K2 = float(np.dot(k, k))
    expect = torch.sin(th)
    del th
    expect *= np.exp(-2 * sigma ** 2 * K2 / res ** 2) * k[d] / (2 * np.pi * K2)
    out = slab.debug_spectral(v, sigma, 8)
    del v
    e = float((out.double() - expect).abs().max() / expect.abs().max())
    print(f"slab closed form at 1024^3: e={e:.2e}")
    assert e < E_CHI


def test_slab_scene_at_1024(slab, dev):
    """A 1M-point scene on 1024^3: the same chi bit for bit for 1, 8 and 64
    slabs; |chi(0,0,0)| = m and the mean of chi at the points is 0 (main
    Eq. 2, reading B), the latter by trilinear interpolation in FP64."""
    sh = S.config_scene()
    res = sh.res
    announce(f"slab scene res={res} P={sh.P} slabs 8 / 1 / 64")
    p, n = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    chi, sc = slab.forward(p, n, res, sh.sigma, 8)
    assert sc["status"] == 0
    m = 0.5
    assert abs(abs(float(chi[0, 0, 0])) - m) < 1e-6
    u = (p.double() % 1.0) * res
    b = torch.floor(u).long().clamp_(0, res - 1)
    f = u - b
    acc = torch.zeros(sh.P, dtype=torch.float64, device=dev)
    for o0 in (0, 1):
        for o1 in (0, 1):
            for o2 in (0, 1):
                w = ((f[:, 0] if o0 else 1 - f[:, 0]) * (f[:, 1] if o1 else 1 - f[:, 1])
                     * (f[:, 2] if o2 else 1 - f[:, 2]))
                acc += w * chi[(b[:, 0] + o0) % res, (b[:, 1] + o1) % res, (b[:, 2] + o2) % res].double()
    mean = float(acc.mean())
    print(f"scene at 1024^3: chi(0)={float(chi[0, 0, 0]):.7f} mean at points={mean:.2e} max|chi|="
          f"{float(chi.abs().max()):.4f}")
    assert abs(mean) < 1e-6
    for g in (1, 64):
        chi_g, sc_g = slab.forward(p, n, res, sh.sigma, g)
        assert torch.equal(chi_g, chi), g
        assert sc_g == sc, g
        del chi_g


def test_slab_status_and_arguments(slab, dev):
    announce("slab status codes and argument errors")
    from paper_2106_03452_amd import _lib
    sh = S.tiny_case(3, 32, 500, 2.0)
    p, n = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    _, sc = slab.forward(p, n, 32, 2.0, 4)
    assert sc["status"] == 0
    _, sc = slab.forward(p, torch.zeros_like(n), 32, 2.0, 4)
    assert sc["status"] == -3  # PSR_EDEGENERATE: all normals zero
    bad = p.clone()
    bad[7, 1] = float("nan")
    chi, sc = slab.forward(bad, n, 32, 2.0, 4)
    assert sc["status"] == -6 and sc["flags"] & 1  # PSR_ENONFINITE
    assert torch.isnan(chi).all()
    for res, g in ((8, 1), (2048, 8), (64, 3), (64, 128), (32, 64)):
        with pytest.raises(_lib.PSRError):
            slab.forward(p, n, res, 2.0, g)
