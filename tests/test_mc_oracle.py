"""Pins of the Marching Cubes oracle (oracle/mc.py) against what geometry and
the mathematics fix, independent of the oracle's own formulas:

  * every sign pattern of a cell appears in a random field, and the mesh is
    closed and edge-manifold (each directed edge once, its reverse once);
  * Euler characteristic 2 for a sphere and 0 for a torus;
  * vertices lie on the level (linear interpolation along their edge);
  * a plane gives exactly the plane, exact unit normals and 2 (r-1)^2
    triangles;
  * a sphere's area and enclosed volume converge to 4 pi R^2 and 4/3 pi R^3
    at second order, every triangle facing outward;
  * main Eq. 6: on a tilted plane with a unit gradient the normal component
    of the finite-difference derivative of the vertex positions with respect
    to any grid value equals the backward's -n spread (exact there); a
    uniform increase of chi moves every vertex inward.
"""
from collections import Counter

import numpy as np
import pytest

from oracle import mc


def grid_points(r):
    return np.indices((r, r, r)).transpose(1, 2, 3, 0) / r


def closed_and_manifold(F):
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    c = Counter(map(tuple, e))
    return all(v == 1 for v in c.values()) and all((b, a) in c for (a, b) in c)


def euler(V, F):
    e = set(tuple(sorted(x)) for x in np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]]))
    return len(V) - len(e) + len(F)


def area_volume(V, F):
    cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    return 0.5 * np.linalg.norm(cr, axis=1).sum(), np.einsum("ij,ij->i", V[F[:, 0]], cr).sum() / 6.0


def test_every_case_closed_and_manifold_on_random_fields():
    rng = np.random.default_rng(0)
    seen = set()
    for trial in range(3):
        r = 20
        chi = rng.standard_normal((r, r, r))
        for a in range(3):  # outside on the border: the level set stays inside the grid
            idx = [slice(None)] * 3
            idx[a] = [0, r - 1]
            chi[tuple(idx)] = 1.0
        inside = chi < 0
        case = np.zeros((r - 1,) * 3, dtype=int)
        for k, o in enumerate(mc.CUBE_CORNERS):
            case |= inside[o[0]:o[0] + r - 1, o[1]:o[1] + r - 1, o[2]:o[2] + r - 1].astype(int) << k
        seen |= set(np.unique(case).tolist())
        m = mc.marching_cubes(chi)
        assert closed_and_manifold(m["faces"])
        assert len(set(map(tuple, np.sort(m["faces"], axis=1)))) == len(m["faces"])  # no repeated triangle
    assert seen == set(range(256))


def test_vertices_on_the_level_and_on_their_edges():
    rng = np.random.default_rng(1)
    r = 12
    chi = rng.standard_normal((r, r, r)) + 0.3
    iso = 0.25
    m = mc.marching_cubes(chi, iso)
    e = m["edge"]
    a = e % 3
    j = np.stack(np.unravel_index(e // 3, (r, r, r)), 1)
    jb = j.copy()
    jb[np.arange(len(e)), a] += 1
    ca, cb = chi[tuple(j.T)], chi[tuple(jb.T)]
    t = m["t"]
    assert np.all((t >= 0) & (t <= 1))
    assert np.allclose((1 - t) * ca + t * cb, iso, atol=1e-14, rtol=0)
    assert np.all((ca < iso) != (cb < iso))
    assert np.allclose(m["verts"] * r, j + t[:, None] * np.eye(3)[a], atol=1e-12)
    assert np.all(np.diff(e) > 0)


def test_plane():
    r, q = 16, 0.3717
    chi = np.broadcast_to((np.arange(r) / r - q)[:, None, None], (r, r, r)).copy()
    m = mc.marching_cubes(chi)
    assert len(m["verts"]) == r * r and len(m["faces"]) == 2 * (r - 1) ** 2
    assert np.allclose(m["verts"][:, 0], q, atol=1e-14)
    assert np.allclose(m["normals"], [1.0, 0.0, 0.0], atol=1e-14)
    V, F = m["verts"], m["faces"]
    cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    assert np.all(cr[:, 0] > 0)  # facing +x, the chi > 0 side


@pytest.mark.parametrize("shape,chi_expected", [("sphere", 2), ("torus", 0)])
def test_euler_characteristic(shape, chi_expected):
    r = 40
    x = grid_points(r) - 0.5
    if shape == "sphere":
        chi = np.linalg.norm(x, axis=-1) - 0.3
    else:
        rho = np.hypot(x[..., 0], x[..., 1])
        chi = np.hypot(rho - 0.25, x[..., 2]) - 0.1
    m = mc.marching_cubes(chi)
    assert closed_and_manifold(m["faces"])
    assert euler(m["verts"], m["faces"]) == chi_expected


def test_sphere_area_volume_converge_and_face_outward():
    R = 0.3
    errs = []
    for r in (24, 48):
        chi = np.linalg.norm(grid_points(r) - 0.5, axis=-1) - R
        m = mc.marching_cubes(chi)
        V, F = m["verts"], m["faces"]
        A, Vol = area_volume(V, F)
        errs.append((abs(A / (4 * np.pi * R ** 2) - 1), abs(Vol / (4 / 3 * np.pi * R ** 3) - 1)))
        cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
        assert np.all(np.einsum("ij,ij->i", cr, V[F].mean(1) - 0.5) > 0)
        assert np.all(np.einsum("ij,ij->i", m["normals"], V - 0.5) > 0)
    (a1, v1), (a2, v2) = errs
    assert a2 < 3e-3 and v2 < 3e-3
    assert a1 / a2 > 2.5 and v1 / v2 > 2.5  # second order: 4x per halving of the cell


def _tilted_plane(r):
    nu = np.array([0.48, 0.6, 0.64])  # unit
    return grid_points(r) @ nu - 0.5, nu


def test_backward_is_the_normal_derivative_on_a_plane():
    """L = sum_v s_v n_v . p_v with the normals held fixed: dL/dchi by central
    differences of the oracle's vertex positions (FP64) against mc_backward.
    On a linear field with |grad chi| = 1 the paper's dp/dchi = -n spread with
    (1 - t, t) is exactly the normal part of the derivative."""
    r = 10
    chi, nu = _tilted_plane(r)
    m = mc.marching_cubes(chi)
    # the field is linear but not periodic: the central differences wrap at
    # the border, so only vertices whose stencils stay inside carry the loss
    e = m["edge"]
    lo = np.stack(np.unravel_index(e // 3, (r, r, r)), 1)
    hi = lo + np.eye(3, dtype=int)[e % 3]
    inner = np.all((lo >= 1) & (hi <= r - 2), axis=1)
    assert inner.sum() > 20
    assert np.allclose(m["normals"][inner], nu, atol=1e-12)
    rng = np.random.default_rng(2)
    s = rng.standard_normal(len(m["verts"])) * inner
    dverts = s[:, None] * m["normals"]
    G = mc.mc_backward(m, dverts, r)
    e0 = m["edge"]
    touched = np.unique(np.concatenate([e0 // 3, (e0 // 3) + np.array([r * r, r, 1])[e0 % 3]]))
    pick = np.concatenate([touched[:: max(1, len(touched) // 40)], rng.integers(0, r ** 3, 10)])
    h = 1e-6
    for k in pick:
        idx = np.unravel_index(k, (r, r, r))
        out = []
        for sgn in (1, -1):
            c2 = chi.copy()
            c2[idx] += sgn * h
            m2 = mc.marching_cubes(c2)
            assert np.array_equal(m2["edge"], e0)  # same topology under the small change
            out.append(np.einsum("v,vd,vd->", s, m["normals"], m2["verts"]))
        fd = (out[0] - out[1]) / (2 * h)
        assert abs(fd - G[idx]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, G[idx])


def test_uniform_increase_moves_vertices_inward():
    r = 24
    chi = np.linalg.norm(grid_points(r) - 0.5, axis=-1) - 0.3
    m = mc.marching_cubes(chi)
    m2 = mc.marching_cubes(chi + 1e-7)
    assert np.array_equal(m["edge"], m2["edge"])
    d = np.einsum("vd,vd->v", m2["verts"] - m["verts"], m["normals"])
    assert np.all(d < 0)
    # and the backward of a uniform perturbation: sum of dchi = sum_v -(dL/dp . n)
    dverts = np.random.default_rng(3).standard_normal(m["verts"].shape)
    G = mc.mc_backward(m, dverts, r)
    assert np.isclose(G.sum(), -np.einsum("vd,vd->", dverts, m["normals"]), rtol=1e-12)
