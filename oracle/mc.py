"""FP64 CPU oracle of the Marching Cubes layer and its inverse-normal gradient -- TEST INFRASTRUCTURE.

Only the tests may import this module; the product path never does. It
shares no code with the HIP library (which builds its own case table in C++
from the same rule).

What it computes (Peng et al., "Shape As Points", main Sec. 3.2):

  * forward  -- the indicator grid chi is turned into a triangle mesh by
                Marching Cubes (Lorensen and Cline, SIGGRAPH 1987): every grid
                edge whose two end values lie on different sides of the level
                carries one mesh vertex at the linear zero of chi along it,
                and every cell joins the vertices on its edges into polygons
                according to the signs of its 8 corners.
  * backward -- main Eq. (6): the derivative of a mesh point with respect to
                chi is taken as the inverse surface normal, dp/dchi = -n. A
                mesh vertex lies on the edge (a, b) at p = a + t (b - a), where
                chi interpolated linearly along the edge equals the level, so
                chi at p depends on the two edge values with weights (1 - t)
                and t. The loss gradient on the grid is therefore
                    dL/dchi[a] += (1 - t) (-(dL/dp . n)),
                    dL/dchi[b] +=     t   (-(dL/dp . n)).
                On a linear field with a unit gradient this equals the exact
                derivative of the vertex positions along the normal (the pins
                check it by finite differences); the tangential part of the
                exact derivative (the vertex sliding along its edge) does not
                move the surface and the paper drops it.

Readings where the paper is silent (listed in the design notes too):
  level     the surface is chi = iso with iso = 0 by default: main Eq. (2)
            makes the mean of chi at the input points zero, so the zero level
            passes through them.
  cells     the grid is sampled as an image volume: cells (j, j + 1) along
            each axis for j in [0, r - 2] (no wrap), vertex j at position j/r,
            as the paper's scikit-image Marching Cubes does on the array.
  inside    a corner is "inside" when chi < iso (outward normals make chi
            negative inside); an edge crosses when exactly one end is inside;
            t = (chi_a - iso) / (chi_a - chi_b).
  faces     a cell face with four crossing edges (inside corners on one
            diagonal) is cut so that each inside corner is separated from the
            other; neighbouring cells see the same face signs and so cut it
            the same way, which keeps the mesh closed.
  polygons  the face segments of a cell chain into closed loops, each
            listed from its smallest local edge id and split into a fan from
            the first vertex whose diagonals all cross the cell's interior (a
            diagonal lying in a face could be drawn by the neighbouring cell
            as well); triangles are ordered by cell (row-major), then loop,
            then fan position; a triangle's vertices run counter-clockwise
            seen from the outside (chi > iso side).
  normals   n at a vertex is the central-difference gradient of chi (periodic,
            the grid of the solver is periodic), linearly interpolated along
            the edge with the same t, normalised.
  numbering vertices are numbered by the global edge id 3 * (row-major index
            of the edge's lower end) + axis, in increasing order.
"""
from __future__ import annotations

import numpy as np

__all__ = ["CUBE_CORNERS", "CUBE_EDGES", "case_table", "marching_cubes", "mc_backward", "grid_normals"]

# corner k of a cell sits at offset o = (k & 1, (k >> 1) & 1, (k >> 2) & 1) along axes (0, 1, 2)
CUBE_CORNERS = np.array([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], dtype=np.int64)


def _edges():
    """The 12 cell edges: edge 4a + u + 2v runs along axis a from the corner
    whose other two coordinates (in increasing axis order) are (u, v)."""
    out = []
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        for v in (0, 1):
            for u in (0, 1):
                lo = [0, 0, 0]
                lo[b], lo[c] = u, v
                hi = list(lo)
                hi[a] = 1
                out.append((a, tuple(lo), tuple(hi)))
    return out


CUBE_EDGES = _edges()  # (axis, low corner offset, high corner offset)


def _corner_index(o):
    return int(o[0]) + 2 * int(o[1]) + 4 * int(o[2])


def _case_polygons(case: int):
    """Closed loops of local edge ids for one sign pattern (bit k = corner k inside)."""
    inside = [(case >> k) & 1 for k in range(8)]
    crossing = [inside[_corner_index(lo)] != inside[_corner_index(hi)] for (_, lo, hi) in CUBE_EDGES]
    mid = [np.array(lo, dtype=float) + 0.5 * (np.array(hi) - np.array(lo)) for (_, lo, hi) in CUBE_EDGES]
    nxt = {}
    for a in range(3):
        for side in (0, 1):
            normal = np.zeros(3)
            normal[a] = 1.0 if side else -1.0
            fe = [e for e, (ax, lo, hi) in enumerate(CUBE_EDGES) if ax != a and lo[a] == side]
            corners = [k for k in range(8) if CUBE_CORNERS[k][a] == side]
            ce = [e for e in fe if crossing[e]]
            if not ce:
                continue
            if len(ce) == 2:
                segs = [(ce[0], ce[1], next(k for k in corners if inside[k]))]
            else:  # four crossings: cut off each inside corner on its own
                segs = []
                for k in corners:
                    if not inside[k]:
                        continue
                    adj = [e for e in fe if _corner_index(CUBE_EDGES[e][1]) == k or _corner_index(CUBE_EDGES[e][2]) == k]
                    segs.append((adj[0], adj[1], k))
            for e1, e2, q in segs:
                A, B = mid[e1], mid[e2]
                # walking A -> B seen from outside the face, the inside corner is on the right
                if np.dot(np.cross(B - A, CUBE_CORNERS[q] - A), normal) > 0:
                    e1, e2 = e2, e1
                assert e1 not in nxt
                nxt[e1] = e2
    loops = []
    seen = set()
    for e0 in sorted(nxt):
        if e0 in seen:
            continue
        loop = [e0]
        seen.add(e0)
        e = nxt[e0]
        while e != e0:
            loop.append(e)
            seen.add(e)
            e = nxt[e]
        loops.append(loop)
    return loops


def _edge_faces(e):
    """The two cell faces (axis, side) that local edge e lies on."""
    a, lo, _ = CUBE_EDGES[e]
    return {(b, lo[b]) for b in range(3) if b != a}


def _fan_apex(loop):
    """First loop position whose fan diagonals all cross the cell's interior:
    a diagonal between two vertices on one face would lie in that face, where
    the neighbouring cell may draw it too (an edge of four triangles)."""
    n = len(loop)
    for s in range(n):
        if all(not (_edge_faces(loop[s]) & _edge_faces(loop[i]))
               for i in range(n) if i not in (s, (s + 1) % n, (s - 1) % n)):
            return s
    raise AssertionError("no interior fan apex")


def case_table():
    """For each of the 256 sign patterns, the triangles as triples of local edge ids."""
    table = []
    for case in range(256):
        tris = []
        for loop in _case_polygons(case):
            s = _fan_apex(loop)
            lp = loop[s:] + loop[:s]
            for i in range(1, len(lp) - 1):
                tris.append((lp[0], lp[i], lp[i + 1]))
        table.append(tris)
    return table


def grid_normals(chi):
    """Central-difference gradient of the periodic grid, in domain units ([3, r, r, r])."""
    r = chi.shape[0]
    return np.stack([(np.roll(chi, -1, axis=a) - np.roll(chi, 1, axis=a)) * (r / 2.0) for a in range(3)])


def marching_cubes(chi, iso: float = 0.0):
    """Mesh of the level set chi = iso.

    Returns a dict with ``verts`` [V, 3] (positions in [0, 1]^3), ``normals``
    [V, 3] (unit, pointing to chi > iso), ``faces`` [F, 3] (vertex indices),
    ``edge`` [V] (global edge id 3 * lin(j) + axis of each vertex) and ``t``
    [V] (position along the edge)."""
    chi = np.asarray(chi, dtype=np.float64)
    r = chi.shape[0]
    assert chi.shape == (r, r, r)
    inside = chi < iso
    grad = grid_normals(chi)
    lin = np.arange(r ** 3).reshape(r, r, r)
    ids, ts, pos, nrm = [], [], [], []
    for a in range(3):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[a] = slice(0, r - 1)
        hi[a] = slice(1, r)
        lo, hi = tuple(lo), tuple(hi)
        cross = inside[lo] != inside[hi]
        ca, cb = chi[lo][cross], chi[hi][cross]
        t = (ca - iso) / (ca - cb)
        j = np.argwhere(cross)  # lower-end vertex coordinates (lo slice starts at 0)
        p = j.astype(np.float64)
        p[:, a] += t
        g = (1.0 - t)[:, None] * np.stack([grad[d][lo][cross] for d in range(3)], 1) + \
            t[:, None] * np.stack([grad[d][hi][cross] for d in range(3)], 1)
        ids.append(3 * lin[lo][cross] + a)
        ts.append(t)
        pos.append(p / r)
        nrm.append(g / np.linalg.norm(g, axis=1, keepdims=True))
    ids = np.concatenate(ids)
    order = np.argsort(ids, kind="stable")
    ids = ids[order]
    verts = np.concatenate(pos)[order]
    normals = np.concatenate(nrm)[order]
    t = np.concatenate(ts)[order]
    vindex = {int(e): i for i, e in enumerate(ids)}
    # cells and their sign patterns
    case = np.zeros((r - 1,) * 3, dtype=np.int64)
    for k, o in enumerate(CUBE_CORNERS):
        case |= inside[o[0]:o[0] + r - 1, o[1]:o[1] + r - 1, o[2]:o[2] + r - 1].astype(np.int64) << k
    table = case_table()
    faces = []
    for c in np.argwhere((case != 0) & (case != 255)):
        for tri in table[case[tuple(c)]]:
            f = []
            for e in tri:
                a, lo, _ = CUBE_EDGES[e]
                jv = c + np.array(lo)
                f.append(vindex[3 * int(lin[tuple(jv)]) + a])
            faces.append(f)
    faces = np.array(faces, dtype=np.int64).reshape(-1, 3)
    return {"verts": verts, "normals": normals, "faces": faces, "edge": ids, "t": t}


def mc_backward(mesh, dverts, r: int):
    """dL/dchi [r, r, r] from dL/dverts [V, 3] with dp/dchi = -n (main Eq. (6)),
    spread onto the two ends of each vertex's edge with weights (1 - t, t)."""
    dverts = np.asarray(dverts, dtype=np.float64)
    g = -np.einsum("vd,vd->v", dverts, mesh["normals"])
    e = mesh["edge"]
    a = e % 3
    j = np.stack(np.unravel_index(e // 3, (r, r, r)), 1)
    jb = j.copy()
    jb[np.arange(len(e)), a] += 1
    G = np.zeros((r, r, r))
    np.add.at(G, (j[:, 0], j[:, 1], j[:, 2]), (1.0 - mesh["t"]) * g)
    np.add.at(G, (jb[:, 0], jb[:, 1], jb[:, 2]), mesh["t"] * g)
    return G
