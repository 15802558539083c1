"""FP64 CPU oracle of the optimisation-based reconstruction loop's pieces -- TEST INFRASTRUCTURE.

Only the tests may import this module. It shares no code with the HIP
library. What it computes (Peng et al., "Shape As Points", main Sec. 3.2):

  * mesh sampling -- points drawn uniformly by area on the Marching Cubes
                     mesh, the mesh points p_mesh of Eq. 5. The random numbers
                     are inputs: u0 picks the triangle through the cumulative
                     area (the first triangle whose running area sum exceeds
                     u0 times the total), u1, u2 place the point with the
                     barycentric weights (1 - sqrt(u1), sqrt(u1) (1 - u2),
                     sqrt(u1) u2) (Turk, Graphics Gems 1990). The normal of a
                     sample is the mesh normal interpolated with the same
                     weights, normalised. The backward spreads dL/dp to the
                     triangle's three vertices with those weights.
  * Chamfer loss  -- the bidirectional L2 Chamfer distance of Eq. 5 between
                     the mesh samples x and the target cloud y,
                     L = mean_i min_j |x_i - y_j|^2 + mean_j min_i |y_j - x_i|^2,
                     and its gradient with respect to x (each term through its
                     nearest neighbour; equal distances go to the lower index).
  * components    -- the connected components of the mesh (triangles sharing
                     a vertex), for the resampling from the largest component
                     (main Sec. 3.2, "Resampling"); the largest is the one with
                     the greatest area (ties: the lowest label), and a
                     component's label is its smallest vertex index.
"""
from __future__ import annotations

import numpy as np

__all__ = ["face_areas", "sample_mesh", "sample_mesh_backward", "chamfer", "components", "largest_component_faces"]


def face_areas(verts, faces):
    v = np.asarray(verts, dtype=np.float64)
    f = np.asarray(faces, dtype=np.int64)
    return 0.5 * np.linalg.norm(np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]]), axis=1)


def _pick(areas, u0):
    csum = np.cumsum(areas)
    tot = csum[-1]
    # first face whose running sum exceeds u0 * total (u0 in [0, 1))
    idx = np.searchsorted(csum, np.asarray(u0, dtype=np.float64) * tot, side="right")
    return np.minimum(idx, len(areas) - 1)


def sample_mesh(verts, faces, u, normals=None, face_weight=None):
    """Samples [M, 3] (and their normals) for the random numbers u [M, 3].
    face_weight (0/1 per face) restricts the draw to a subset of the faces."""
    v = np.asarray(verts, dtype=np.float64)
    f = np.asarray(faces, dtype=np.int64)
    u = np.asarray(u, dtype=np.float64)
    a = face_areas(v, f)
    if face_weight is not None:
        a = a * np.asarray(face_weight, dtype=np.float64)
    fi = _pick(a, u[:, 0])
    s = np.sqrt(u[:, 1])
    bary = np.stack([1.0 - s, s * (1.0 - u[:, 2]), s * u[:, 2]], 1)
    tri = f[fi]
    pts = np.einsum("mk,mkd->md", bary, v[tri])
    out = {"points": pts, "face": fi, "bary": bary}
    if normals is not None:
        nv = np.asarray(normals, dtype=np.float64)
        n = np.einsum("mk,mkd->md", bary, nv[tri])
        out["normals"] = n / np.linalg.norm(n, axis=1, keepdims=True)
    return out


def sample_mesh_backward(faces, sample, dpoints, nverts):
    """dL/dverts [V, 3] from dL/dpoints of the samples."""
    f = np.asarray(faces, dtype=np.int64)
    g = np.zeros((nverts, 3))
    tri = f[sample["face"]]
    for k in range(3):
        np.add.at(g, tri[:, k], sample["bary"][:, k:k + 1] * np.asarray(dpoints, dtype=np.float64))
    return g


def _nearest(a, b):
    """For every row of a, the index of the nearest row of b (lowest index on ties) and the squared distance."""
    d = ((a[:, None, :] - b[None, :, :]) ** 2).sum(-1)
    j = np.argmin(d, axis=1)
    return j, d[np.arange(len(a)), j]


def chamfer(x, y, block=2048):
    """Loss and dL/dx of the bidirectional L2 Chamfer distance."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    jx, dx = np.empty(len(x), dtype=np.int64), np.empty(len(x))
    for s in range(0, len(x), block):
        jx[s:s + block], dx[s:s + block] = _nearest(x[s:s + block], y)
    iy, dy = np.empty(len(y), dtype=np.int64), np.empty(len(y))
    for s in range(0, len(y), block):
        iy[s:s + block], dy[s:s + block] = _nearest(y[s:s + block], x)
    loss = dx.mean() + dy.mean()
    g = 2.0 * (x - y[jx]) / len(x)
    np.add.at(g, iy, 2.0 * (x[iy] - y) / len(y))
    return {"loss": loss, "grad": g, "nn_x": jx, "d_x": dx, "nn_y": iy, "d_y": dy}


def components(faces, nverts):
    """Component label of every vertex (its component's smallest vertex index),
    by repeated relaxation over the triangles until nothing changes."""
    f = np.asarray(faces, dtype=np.int64)
    lab = np.arange(nverts)
    while True:
        m = lab[f].min(axis=1)
        new = lab.copy()
        for k in range(3):
            np.minimum.at(new, f[:, k], m)
        new = new[new]  # follow labels to their own labels
        if np.array_equal(new, lab):
            return lab
        lab = new


def largest_component_faces(verts, faces):
    """0/1 per face: the faces of the component with the greatest area."""
    f = np.asarray(faces, dtype=np.int64)
    lab = components(f, len(verts))
    fl = lab[f[:, 0]]
    a = face_areas(verts, f)
    tot = {}
    for l, ar in zip(fl.tolist(), a.tolist()):
        tot[l] = tot.get(l, 0.0) + ar
    best = min(tot, key=lambda l: (-tot[l], l))
    return (fl == best).astype(np.float64)
