"""Pins of the optimisation-loop oracle (oracle/opt.py) against what the
definitions and library routines fix:

  * sampling: evenly spaced u0 splits the samples between triangles in
    proportion to their areas (within one sample); the barycentric map is
    area-uniform (sample mean of a triangle = its centroid); samples of a
    planar mesh lie in its plane; the backward is the finite-difference
    derivative of the samples with respect to the vertices;
  * Chamfer: nearest distances equal scipy's k-d tree, identical clouds give
    zero loss and gradient, and the gradient is the finite-difference
    derivative of the loss (both terms and their 1/M, 1/T weights);
  * components: scipy's connected components of the vertex graph, and the
    largest by area is the bigger of two spheres.
"""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from oracle import mc
from oracle import opt


def two_triangles():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [3, 0, 0], [3, 2, 0], [3, 0, 1.5]], dtype=np.float64)
    f = np.array([[0, 1, 2], [3, 4, 5]])
    return v, f  # areas 0.5 and 1.5


def test_sampling_follows_area():
    v, f = two_triangles()
    M = 4000
    u = np.stack([(np.arange(M) + 0.5) / M, np.full(M, 0.3), np.full(M, 0.6)], 1)
    s = opt.sample_mesh(v, f, u)
    n0 = int((s["face"] == 0).sum())
    assert abs(n0 - M * 0.5 / 2.0) <= 1


def test_barycentric_map_is_area_uniform():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float64)
    f = np.array([[0, 1, 2]])
    k = 200
    g = (np.arange(k) + 0.5) / k
    u1, u2 = np.meshgrid(g, g, indexing="ij")
    u = np.stack([np.zeros(k * k), u1.ravel(), u2.ravel()], 1)
    p = opt.sample_mesh(v, f, u)["points"]
    assert np.allclose(p.mean(0), [1 / 3, 1 / 3, 0], atol=2e-4)
    assert np.all(p[:, :2] >= -1e-15) and np.all(p[:, 0] + p[:, 1] <= 1 + 1e-15)


def test_samples_of_a_plane_lie_in_it():
    r = 16
    chi = np.broadcast_to((np.arange(r) / r - 0.41)[:, None, None], (r, r, r)).copy()
    m = mc.marching_cubes(chi)
    u = np.random.default_rng(0).random((500, 3))
    s = opt.sample_mesh(m["verts"], m["faces"], u, m["normals"])
    assert np.allclose(s["points"][:, 0], 0.41, atol=1e-14)
    assert np.allclose(s["normals"], [1, 0, 0], atol=1e-14)


def test_sampling_backward_is_the_derivative():
    rng = np.random.default_rng(1)
    v = rng.random((12, 3))
    f = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11], [0, 4, 8]])
    u = rng.random((50, 3))
    w = rng.standard_normal((50, 3))
    s = opt.sample_mesh(v, f, u)
    g = opt.sample_mesh_backward(f, s, w, len(v))
    h = 1e-7
    for i in range(len(v)):
        for d in range(3):
            vp, vm = v.copy(), v.copy()
            vp[i, d] += h
            vm[i, d] -= h
            sp, sm = opt.sample_mesh(vp, f, u), opt.sample_mesh(vm, f, u)
            if not (np.array_equal(sp["face"], s["face"]) and np.array_equal(sm["face"], s["face"])):
                continue  # a sample changed triangle: not differentiable there
            fd = ((sp["points"] - sm["points"]) * w).sum() / (2 * h)
            assert abs(fd - g[i, d]) <= 1e-6 * max(1.0, abs(fd))


def test_chamfer_distances_match_kdtree():
    rng = np.random.default_rng(2)
    x, y = rng.random((700, 3)), rng.random((500, 3))
    c = opt.chamfer(x, y, block=128)
    dx, _ = cKDTree(y).query(x)
    dy, _ = cKDTree(x).query(y)
    assert np.allclose(c["d_x"], dx ** 2, rtol=1e-12, atol=1e-15)
    assert np.allclose(c["d_y"], dy ** 2, rtol=1e-12, atol=1e-15)
    assert np.isclose(c["loss"], (dx ** 2).mean() + (dy ** 2).mean(), rtol=1e-12)
    z = opt.chamfer(x, x)
    assert z["loss"] == 0.0 and not z["grad"].any()


def test_chamfer_gradient_is_the_derivative():
    rng = np.random.default_rng(3)
    x, y = rng.random((60, 3)), rng.random((45, 3))
    c = opt.chamfer(x, y)
    h = 1e-7
    for i in range(len(x)):
        for d in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            fd = (opt.chamfer(xp, y)["loss"] - opt.chamfer(xm, y)["loss"]) / (2 * h)
            assert abs(fd - c["grad"][i, d]) <= 1e-6 * max(1e-3, abs(fd))


def _two_spheres(r=48):
    x = np.indices((r, r, r)).transpose(1, 2, 3, 0) / r
    a = np.linalg.norm(x - [0.3, 0.5, 0.5], axis=-1) - 0.15
    b = np.linalg.norm(x - [0.72, 0.5, 0.5], axis=-1) - 0.1
    return np.minimum(a, b)


def test_components_match_scipy_and_largest_is_the_bigger_sphere():
    m = mc.marching_cubes(_two_spheres())
    f, V = m["faces"], len(m["verts"])
    lab = opt.components(f, V)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    n, ref = connected_components(coo_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(V, V)), directed=False)
    assert n == 2 and len(np.unique(lab)) == 2
    # same partition; each label is its component's smallest vertex
    for c in range(n):
        members = np.flatnonzero(ref == c)
        assert np.all(lab[members] == members.min())
    keep = opt.largest_component_faces(m["verts"], f)
    centre = m["verts"][f[keep > 0]].mean(axis=(0, 1))
    assert abs(centre[0] - 0.3) < 0.01
