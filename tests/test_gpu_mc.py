"""GPU parity of the Marching Cubes layer (psr_marching_cubes and its
backward, main Sec. 3.2, Eq. 6) against the FP64 oracle (oracle/mc.py).

Both sides read the same float32 grid (an analytic field, or the oracle's
own chi rounded once to float32), so every sign decision is taken on the same
values: vertex edge ids and triangles must agree exactly; positions and
normals within 1e-5 (positions in domain units, normals as unit vectors);
dL/dchi of the backward within 1e-4 relative L2 (the gradient bar)."""
import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, host, l2_rel, require_gpu, to_dev, torch
from oracle import mc as omc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _field(kind, r, seed=0):
    x = np.indices((r, r, r)).transpose(1, 2, 3, 0) / r - 0.5
    if kind == "sphere":
        f = np.linalg.norm(x, axis=-1) - 0.31
    elif kind == "torus":
        rho = np.hypot(x[..., 0], x[..., 1])
        f = np.hypot(rho - 0.24, x[..., 2]) - 0.09
    elif kind == "noise":
        f = np.random.default_rng(seed).standard_normal((r, r, r))
        for a in range(3):
            idx = [slice(None)] * 3
            idx[a] = [0, r - 1]
            f[tuple(idx)] = 1.0
    else:
        raise ValueError(kind)
    return f.astype(np.float32)


def _compare(chi32, dev, iso=0.0, capacity=None):
    from paper_2106_03452_amd import mesh as M
    m = M.marching_cubes(to_dev(chi32, dev), iso, capacity=capacity)
    ref = omc.marching_cubes(chi32.astype(np.float64), iso)
    assert np.array_equal(m.edges.cpu().numpy().astype(np.int64), ref["edge"])
    assert np.array_equal(m.faces.cpu().numpy().astype(np.int64), ref["faces"])
    e_p = float(np.abs(host(m.verts) - ref["verts"]).max())
    e_n = float(np.abs(host(m.normals) - ref["normals"]).max())
    return m, ref, e_p, e_n


@pytest.mark.parametrize("kind,r", [("sphere", 8), ("noise", 8), ("sphere", 16), ("sphere", 64), ("torus", 128),
                                    ("noise", 32), ("sphere", 256), ("torus", 512)])
def test_mesh_matches_oracle(dev, kind, r):
    announce(f"marching cubes {kind} {r}^3")
    m, ref, e_p, e_n = _compare(_field(kind, r), dev)
    print(f"MC {kind} {r}^3: V={len(ref['verts'])} F={len(ref['faces'])} e_pos={e_p:.2e} e_normal={e_n:.2e}")
    assert len(ref["faces"]) > 0
    assert e_p <= 1e-5 and e_n <= 1e-5


def test_mesh_of_the_solver_output(dev):
    """The oracle's chi of the 128^3 torus + sphere workload, rounded to
    float32, meshed on both sides; iso = 0 and a shifted level."""
    announce("marching cubes of the oracle's 128^3 chi")
    sh = S.config_c2()
    chi, _ = oracle.forward(sh.points, sh.normals, sh.res, sh.sigma)
    chi32 = chi.astype(np.float32)
    for iso in (0.0, 0.1):
        m, ref, e_p, e_n = _compare(chi32, dev, iso)
        print(f"MC of chi at iso {iso}: V={len(ref['verts'])} e_pos={e_p:.2e} e_normal={e_n:.2e}")
        assert e_p <= 1e-5 and e_n <= 1e-5


def test_capacity_overflow_reruns(dev):
    announce("marching cubes with too small buffers")
    chi32 = _field("sphere", 64)
    m, ref, _, _ = _compare(chi32, dev, capacity=(100, 100))
    assert m.verts.shape[0] == len(ref["verts"]) > 100


@pytest.mark.parametrize("kind,r", [("sphere", 8), ("noise", 16), ("sphere", 32), ("noise", 32), ("torus", 128),
                                    ("sphere", 256), ("torus", 512)])
def test_backward_matches_oracle(dev, kind, r):
    from paper_2106_03452_amd import mesh as M
    announce(f"marching cubes backward {kind} {r}^3")
    chi32 = _field(kind, r)
    m = M.marching_cubes(to_dev(chi32, dev))
    ref = omc.marching_cubes(chi32.astype(np.float64))
    dv = np.random.default_rng(r).standard_normal(ref["verts"].shape).astype(np.float32)
    g = M.marching_cubes_backward(to_dev(chi32, dev), m, to_dev(dv, dev))
    g_ref = omc.mc_backward(ref, dv.astype(np.float64), r)
    e = l2_rel(host(g), g_ref)
    print(f"MC backward {kind} {r}^3: e_dchi={e:.2e}")
    assert e <= 1e-4
    # deterministic: the same bits again
    assert torch.equal(g, M.marching_cubes_backward(to_dev(chi32, dev), m, to_dev(dv, dev)))


def test_points_to_mesh_chain(dev):
    """main Eq. 5: a loss on the mesh vertices back to the oriented points,
    through Marching Cubes (Eq. 6) and the solver's adjoint. GPU chain
    (solve -> mesh -> loss -> autograd) against the oracle chain
    (forward -> mc -> mc_backward -> backward) on a 64^3 sphere."""
    from paper_2106_03452_amd import function as F
    from paper_2106_03452_amd import mesh as M
    announce("points -> chi -> mesh -> loss chain 64^3")
    sh = S.tiny_case(4, 64, 4000, kind="sphere")
    chi_r, aux = oracle.forward(sh.points, sh.normals, 64, 2.0)
    # no grid value near the level, so both sides' float32 grids give the same mesh
    assert np.abs(chi_r).min() > 1e-4
    pts = to_dev(sh.points, dev).requires_grad_(True)
    nrm = to_dev(sh.normals, dev).requires_grad_(True)
    chi = F.solve(pts, nrm, 64, 2.0)
    verts, faces, normals = M.mesh(chi)
    ref = omc.marching_cubes(chi_r)
    assert np.array_equal(faces.cpu().numpy().astype(np.int64), ref["faces"])
    w = np.random.default_rng(9).standard_normal(ref["verts"].shape)
    (verts * to_dev(w, dev)).sum().backward()
    G = omc.mc_backward(ref, w, 64)
    dc, dn = oracle.backward(aux, G)
    e_c, e_n = l2_rel(host(pts.grad), dc), l2_rel(host(nrm.grad), dn)
    print(f"chain 64^3: V={len(ref['verts'])} e_dpoints={e_c:.2e} e_dnormals={e_n:.2e}")
    assert e_c <= 1e-4 and e_n <= 1e-4


def test_backward_refuses_state_of_another_grid(dev):
    import ctypes
    from paper_2106_03452_amd import _lib
    from paper_2106_03452_amd import mesh as M
    announce("marching cubes backward with a mismatched state")
    chi32 = _field("sphere", 32)
    m = M.marching_cubes(to_dev(chi32, dev))
    dchi = torch.zeros((32, 32, 32), dtype=torch.float32, device=dev)
    dv = torch.ones_like(m.verts)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = _lib.lib().psr_marching_cubes_backward(_lib.context(0).handle, p(to_dev(chi32, dev)), 32, 0.5,
                                                p(m.state), p(m.normals), p(dv), m.verts.shape[0], p(dchi), st)
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.isnan(dchi).all()
