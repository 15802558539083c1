"""GPU parity of the optimisation loop's pieces (psr_mesh_sample and its
backward, psr_chamfer and its backward, psr_mesh_components) against the
FP64 oracle (oracle/opt.py), and the loop itself (main Sec. 3.2).

Both sides read the same float32 inputs (the oracle's Marching Cubes mesh of
an analytic field rounded once to float32, the same random numbers, the same
clouds). Integer results (triangle picked, component labels, the largest
component) must agree exactly; positions, distances and gradients within
1e-5 relative. A nearest neighbour is an integer decided by FP32 distances on
the GPU: where the two sides pick different neighbours, both must be at the
same (minimal) distance within that tolerance.
"""
import numpy as np
import pytest

import oracle
import psr_synth as S
from gpu_common import announce, host, l2_rel, require_gpu, to_dev, torch
from oracle import mc as omc
from oracle import opt as oopt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return require_gpu()


def _mesh32(kind="sphere", r=48):
    x = np.indices((r, r, r)).transpose(1, 2, 3, 0) / r
    if kind == "sphere":
        f = np.linalg.norm(x - 0.5, axis=-1) - 0.3
    else:  # two spheres
        f = np.minimum(np.linalg.norm(x - [0.3, 0.5, 0.5], axis=-1) - 0.15,
                       np.linalg.norm(x - [0.72, 0.5, 0.5], axis=-1) - 0.1)
    m = omc.marching_cubes(f.astype(np.float32).astype(np.float64))
    return (m["verts"].astype(np.float32), m["faces"].astype(np.int32), m["normals"].astype(np.float32))


def test_sampling_matches_oracle(dev):
    from paper_2106_03452_amd import optimize as O
    announce("mesh sampling vs oracle")
    v, f, vn = _mesh32("two")
    u = np.random.default_rng(0).random((20000, 3)).astype(np.float32)
    w = (np.arange(len(f)) % 3 != 0).astype(np.float32)  # a subset of the faces
    for weight in (None, w):
        pts, nrm, face, bary = O.sample_raw(to_dev(v, dev), torch.from_numpy(f).to(dev), to_dev(u, dev),
                                            to_dev(vn, dev), to_dev(weight, dev) if weight is not None else None)
        ref = oopt.sample_mesh(v, f, u, vn, weight)
        same = host(face) == ref["face"]
        print(f"sampling: {same.mean() * 100:.4f}% same triangle")
        assert same.all()
        assert np.abs(host(pts) - ref["points"]).max() <= 1e-6
        assert np.abs(host(nrm) - ref["normals"]).max() <= 1e-5
        assert np.abs(host(bary) - ref["bary"]).max() <= 1e-6


def test_sampling_backward_matches_oracle(dev):
    from paper_2106_03452_amd import optimize as O
    announce("mesh sampling backward vs oracle")
    v, f, _ = _mesh32()
    u = np.random.default_rng(1).random((30000, 3)).astype(np.float32)
    dp = np.random.default_rng(2).standard_normal((30000, 3)).astype(np.float32)
    V = to_dev(v, dev).requires_grad_(True)
    x = O.SampleFunction.apply(V, torch.from_numpy(f).to(dev), to_dev(u, dev))
    (x * to_dev(dp, dev)).sum().backward()
    ref = oopt.sample_mesh(v, f, u)
    g = oopt.sample_mesh_backward(f, ref, dp, len(v))
    e = l2_rel(host(V.grad), g)
    print(f"sampling backward e={e:.2e}")
    assert e <= 1e-5


# (40000, 3000): the five-kernel sort (32^3 cells); (300000, 256): 64^3 cells,
# and the queries of the small cloud list the large one's tiles in ten passes
@pytest.mark.parametrize("nx,ny", [(20000, 20000), (5000, 30000), (257, 1), (40000, 3000), (300000, 256)])
def test_chamfer_matches_oracle(dev, nx, ny):
    from paper_2106_03452_amd import optimize as O
    announce(f"chamfer {nx} x {ny} vs oracle")
    rng = np.random.default_rng(nx + ny)
    x = rng.random((nx, 3)).astype(np.float32)
    y = rng.random((ny, 3)).astype(np.float32)
    loss, nnx, dx, nny, dy = O.chamfer_raw(to_dev(x, dev), to_dev(y, dev))
    ref = oopt.chamfer(x, y)
    for d_g, d_r, nn_g, a, b in ((host(dx), ref["d_x"], host(nnx).astype(np.int64), x, y),
                                 (host(dy), ref["d_y"], host(nny).astype(np.int64), y, x)):
        assert np.abs(d_g - d_r).max() <= 1e-5 * max(d_r.max(), 1e-12)
        # a different neighbour only on a tie at the tolerance
        dd = ((a.astype(np.float64) - b.astype(np.float64)[nn_g]) ** 2).sum(1)
        assert np.abs(dd - d_r).max() <= 1e-5 * max(d_r.max(), 1e-12)
    assert abs(float(loss) - ref["loss"]) <= 1e-6 * ref["loss"]
    X = to_dev(x, dev).requires_grad_(True)
    O.ChamferFunction.apply(X, to_dev(y, dev)).backward()
    e = l2_rel(host(X.grad), ref["grad"])
    print(f"chamfer {nx}x{ny}: loss {float(loss):.6e} (ref {ref['loss']:.6e}), grad e={e:.2e}")
    assert e <= 1e-5


def _check_nn(d_g, nn_g, a, b, d_r):
    assert np.abs(d_g - d_r).max() <= 1e-5 * max(d_r.max(), 1e-12)
    assert nn_g.min() >= 0 and nn_g.max() < len(b)
    dd = ((a.astype(np.float64) - b.astype(np.float64)[nn_g]) ** 2).sum(1)
    assert np.abs(dd - d_r).max() <= 1e-5 * max(d_r.max(), 1e-12)


@pytest.mark.parametrize("case", ["surfaces", "outside_and_clustered", "one_cell", "duplicates", "single_query"])
def test_chamfer_structured_clouds_match_oracle(dev, case):
    """The search skips tiles of the sorted reference cloud by their boxes; it
    must still return the brute-force neighbours on clouds that stress that:
    two surfaces apart (the loop's clouds), points outside [0,1)^3 and a dense
    cluster (cells spanning many tiles), every point in one cell, exact
    duplicates (equal distances: the lower index), a lone query."""
    from paper_2106_03452_amd import optimize as O
    announce(f"chamfer {case} vs oracle")
    rng = np.random.default_rng(3)
    if case == "surfaces":
        x = S.tiny_case(7, 64, 9000, kind="sphere").points
        y = S.tiny_case(11, 64, 12000, kind="torus").points
    elif case == "outside_and_clustered":
        x = rng.uniform(-0.5, 1.5, (7000, 3)).astype(np.float32)
        y = np.concatenate([rng.normal(0.5, 0.03, (9000, 3)), rng.uniform(0, 1, (1000, 3))]).astype(np.float32)
    elif case == "one_cell":
        x = rng.uniform(0.40, 0.401, (3000, 3)).astype(np.float32)
        y = rng.uniform(0.40, 0.401, (5000, 3)).astype(np.float32)
    elif case == "duplicates":
        x = rng.random((6000, 3)).astype(np.float32)
        y0 = rng.random((4000, 3)).astype(np.float32)
        y = np.concatenate([y0, y0])
    else:
        x = rng.random((1, 3)).astype(np.float32)
        y = rng.random((20000, 3)).astype(np.float32)
    loss, nnx, dx, nny, dy = O.chamfer_raw(to_dev(x, dev), to_dev(y, dev))
    ref = oopt.chamfer(x, y)
    nnx_g, nny_g = host(nnx).astype(np.int64), host(nny).astype(np.int64)
    _check_nn(host(dx), nnx_g, x, y, ref["d_x"])
    _check_nn(host(dy), nny_g, y, x, ref["d_y"])
    if case == "duplicates":
        # the copies of a target point are at exactly equal distances
        assert nnx_g.max() < len(y0)
        assert np.array_equal(nny_g[:len(y0)], nny_g[len(y0):])
    # the same neighbours as the oracle wherever its nearest distance is not
    # tied within the tolerance by another point
    for nn_g, nn_r, a, b in ((nnx_g, ref["nn_x"], x, y), (nny_g, ref["nn_y"], y, x)):
        diff = np.nonzero(nn_g != nn_r)[0]
        for i in diff[:200]:
            da = ((a[i].astype(np.float64) - b[nn_g[i]]) ** 2).sum()
            db = ((a[i].astype(np.float64) - b[nn_r[i]]) ** 2).sum()
            assert abs(da - db) <= 1e-5 * max(db, 1e-12), (i, da, db)
    assert abs(float(loss) - ref["loss"]) <= 1e-6 * ref["loss"]
    print(f"chamfer {case}: loss {float(loss):.6e} (ref {ref['loss']:.6e}), "
          f"{int((nnx_g != ref['nn_x']).sum() + (nny_g != ref['nn_y']).sum())} tied neighbours differ")


def test_chamfer_is_deterministic(dev):
    """The search sorts the points with atomics, so their order within a
    cell changes from call to call; the neighbours, the distances and the
    loss must not."""
    from paper_2106_03452_amd import optimize as O
    announce("chamfer: repeated calls")
    x = to_dev(S.tiny_case(7, 64, 20000, kind="sphere").points, dev)
    y = to_dev(S.tiny_case(11, 64, 20000, kind="torus").points, dev)
    first = [host(t) for t in O.chamfer_raw(x, y)]
    for _ in range(4):
        again = [host(t) for t in O.chamfer_raw(x, y)]
        for a, b in zip(first, again):
            assert np.array_equal(a, b)


def test_chamfer_nan_point_has_no_neighbour(dev):
    """A sample with a NaN coordinate is nobody's nearest neighbour and has
    none itself (index -1, distance +inf, NaN gradient); the other samples'
    neighbours and gradients are those of the cloud without it."""
    from paper_2106_03452_amd import optimize as O
    announce("chamfer with a NaN sample")
    rng = np.random.default_rng(9)
    x = rng.random((3000, 3)).astype(np.float32)
    y = rng.random((2000, 3)).astype(np.float32)
    xn = x.copy()
    xn[17, 1] = np.nan
    loss, nnx, dx, nny, dy = O.chamfer_raw(to_dev(xn, dev), to_dev(y, dev))
    nnx, dx, nny, dy = host(nnx), host(dx), host(nny), host(dy)
    assert nnx[17] == -1 and np.isinf(dx[17]) and np.isinf(float(loss))
    keep = np.arange(len(x)) != 17
    ref = oopt.chamfer(x[keep], y)
    remap = np.nonzero(keep)[0]
    _check_nn(dx[keep], nnx[keep].astype(np.int64), x[keep], y, ref["d_x"])
    _check_nn(dy, nny.astype(np.int64), y, xn, ref["d_y"])
    assert (nny != 17).all()
    print(f"NaN sample: {int((remap[ref['nn_y']] != nny).sum())} tied neighbours differ")
    X = to_dev(xn, dev).requires_grad_(True)
    O.ChamferFunction.apply(X, to_dev(y, dev)).backward()
    g = host(X.grad)
    assert np.isnan(g[17]).all() and np.isfinite(g[keep]).all()


def test_components_match_oracle(dev):
    from paper_2106_03452_amd import optimize as O
    announce("mesh components vs oracle")
    v, f, _ = _mesh32("two", 64)
    lab, w = O.components(to_dev(v, dev), torch.from_numpy(f).to(dev))
    ref = oopt.components(f, len(v))
    assert np.array_equal(host(lab).astype(np.int64), ref)
    assert np.array_equal(host(w), oopt.largest_component_faces(v, f))


def test_one_step_gradient_matches_oracle_chain(dev):
    """main Eq. 5 end to end: the Chamfer loss of area samples of the mesh of
    the solved grid, back to the points and normals (Eq. 6 through the mesh),
    against the oracle's chain on the same inputs and random numbers."""
    from paper_2106_03452_amd import function as F
    from paper_2106_03452_amd import mesh as M
    from paper_2106_03452_amd import optimize as O
    announce("optimisation step gradient vs oracle chain, 32^3")
    res, sigma = 32, 2.0
    rng = np.random.default_rng(5)
    sh = S.tiny_case(7, res, 2000, kind="sphere")
    target = S.tiny_case(11, res, 3000, kind="torus").points
    u = rng.random((3000, 3)).astype(np.float32)
    chi_r, aux = oracle.forward(sh.points, sh.normals, res, sigma)
    assert np.abs(chi_r).min() > 1e-4  # both sides' grids give the same mesh
    pts = to_dev(sh.points, dev).requires_grad_(True)
    nrm = to_dev(sh.normals, dev).requires_grad_(True)
    loss, _ = O.step_loss(pts, nrm, to_dev(target, dev), res, sigma, to_dev(u, dev))
    loss.backward()
    m = omc.marching_cubes(chi_r)
    s = oopt.sample_mesh(m["verts"], m["faces"], u)
    c = oopt.chamfer(s["points"], target)
    dv = oopt.sample_mesh_backward(m["faces"], s, c["grad"], len(m["verts"]))
    G = omc.mc_backward(m, dv, res)
    dc, dn = oracle.backward(aux, G)
    e_l = abs(float(loss) - c["loss"]) / c["loss"]
    e_c, e_n = l2_rel(host(pts.grad), dc), l2_rel(host(nrm.grad), dn)
    print(f"step: loss {float(loss):.6e} (ref {c['loss']:.6e}) e_dpoints={e_c:.2e} e_dnormals={e_n:.2e}")
    assert e_l <= 1e-5 and e_c <= 1e-4 and e_n <= 1e-4


def _adam_reference_step(p, n, target, res, sigma, u, lr, steps):
    """The iteration through the autograd Functions and PyTorch's Adam."""
    from paper_2106_03452_amd import optimize as O
    p, n = p.clone().requires_grad_(True), n.clone().requires_grad_(True)
    opt = torch.optim.Adam([p, n], lr=lr, fused=True)
    losses = []
    for k in range(steps):
        opt.zero_grad(set_to_none=True)
        loss, _ = O.step_loss(p, n, target, res, sigma, u[k])
        loss.backward()
        opt.step()
        with torch.no_grad():
            p.remainder_(1.0)
        losses.append(float(loss))
    return p.detach(), n.detach(), losses


def test_native_step_matches_the_autograd_step(dev):
    """psr_opt_step runs the same kernels as the separate calls: the loss is
    the same, and after three Adam steps the cloud agrees with PyTorch's Adam
    on the autograd path (the float atomics of two backward stages reorder
    the last bits of a few gradients; Adam's first steps move each value by
    about lr times the sign of its gradient)."""
    from paper_2106_03452_amd import optimize as O
    announce("native optimisation step vs the autograd step, 32^3")
    res, sigma, lr = 32, 2.0, 2e-3
    sh = S.tiny_case(7, res, 3000, kind="sphere")
    target = to_dev(S.tiny_case(11, res, 4000, kind="torus").points, dev)
    p0, n0 = to_dev(sh.points, dev), to_dev(sh.normals, dev)
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    u = [torch.rand((2500, 3), generator=g, device=dev) for _ in range(3)]
    pr, nr, losses = _adam_reference_step(p0, n0, target, res, sigma, u, lr, 3)
    p, n = p0.clone(), n0.clone()
    moments = [torch.zeros_like(p) for _ in range(4)]
    step = O.NativeStep(dev, 3000, 4000, 2500, res)
    for k in range(3):
        loss = float(step(p, n, moments, k + 1, lr, target, u[k], sigma))
        assert abs(loss - losses[k]) <= 1e-5 * losses[k], (k, loss, losses[k])
    ep, en = float((p - pr).abs().max()), float((n - nr).abs().max())
    print(f"native step: losses {losses}; max |dp| {ep:.2e}, max |dn| {en:.2e}")
    assert ep <= 1e-5 and en <= 1e-5
    assert bool(((p >= 0) & (p < 1)).all())


def test_native_step_grows_its_mesh_cap(dev):
    """A mesh larger than the workspace's cap leaves the cloud untouched
    (PSR_ETOOBIG); the step then grows the cap and runs again, with the same
    result as a step that had room from the start."""
    from paper_2106_03452_amd import optimize as O
    announce("native optimisation step with a small mesh cap")
    res, sigma = 32, 2.0
    sh = S.tiny_case(7, res, 3000, kind="sphere")
    target = to_dev(S.tiny_case(11, res, 4000, kind="torus").points, dev)
    u = torch.rand((2500, 3), generator=torch.Generator(device=dev).manual_seed(5), device=dev)
    outs = []
    for cap in (None, 16):
        p, n = to_dev(sh.points, dev), to_dev(sh.normals, dev)
        moments = [torch.zeros_like(p) for _ in range(4)]
        step = O.NativeStep(dev, 3000, 4000, 2500, res)
        if cap:
            step.vcap = step.tcap = cap
            step._alloc()
        loss = float(step(p, n, moments, 1, 2e-3, target, u, sigma))
        if cap:
            assert step.vcap > cap and step.tcap > cap
        outs.append((loss, p, n))
    assert outs[0][0] == outs[1][0]
    assert float((outs[0][1] - outs[1][1]).abs().max()) <= 1e-6
    assert float((outs[0][2] - outs[1][2]).abs().max()) <= 1e-6


def test_short_optimisation_lowers_chamfer(dev):
    from paper_2106_03452_amd import optimize as O
    announce("short coarse-to-fine optimisation")
    target = to_dev(S.tiny_case(8, 64, 5000, kind="torus").points, dev)
    sched = [O.Level(32, 2.0, 150), O.Level(64, 2.0, 100)]
    for native in (True, False):
        r = O.optimise(target, sched, npoints=5000, resample_every=100, log_every=25, seed=1, native=native)
        first, last = r.history[0][3], r.history[-1][3]
        print(f"native={native}: Chamfer {first:.3e} -> {last:.3e}; ms/iter {r.ms_per_iter}")
        assert last < 0.3 * first
        assert torch.isfinite(r.points).all() and r.faces.shape[0] > 0
