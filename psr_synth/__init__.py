"""Seeded synthetic oriented point clouds (positions + normals).

This module only *generates inputs*; it holds none of the solver's arithmetic.
Both the FP64 oracle tests and the HIP path consume the float32 arrays it
returns, so the two sides see bit-identical inputs.

Rules shared by every generator:
  * RNG is ``numpy.random.Generator(PCG64(seed))``.
  * Everything is computed in float64 and rounded once to float32.
  * Shapes are centred near (0.5, 0.5, 0.5) and stay inside [0.05, 0.95]^3
    of the unit periodic domain.

The shapes stand in for the paper's datasets (ShapeNet, Thingi10K, SRB,
D-FAUST), which are not available: spheres, tori and superellipsoids with exact
analytic normals, sampled uniformly by surface area.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng_for", "sphere", "torus", "superellipsoid", "random_rotation",
    "Shape", "config_c1", "config_c2", "config_c2_outliers", "config_c3", "config_c3_outliers", "config_c4",
    "config_c5",
    "random_shape", "tiny_case", "loss_gradient", "thin_plate",
]


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _unit(v: np.ndarray) -> np.ndarray:
    nrm = np.linalg.norm(v, axis=-1, keepdims=True)
    nrm = np.where(nrm > 0, nrm, 1.0)
    return v / nrm


# --------------------------------------------------------------------------
# primitive surfaces (float64)
# --------------------------------------------------------------------------
def sphere(rng, P, center, radius):
    """P points uniform on a sphere (normalised Gaussian directions), outward normals."""
    d = _unit(rng.standard_normal((P, 3)))
    return np.asarray(center, np.float64) + radius * d, d


def torus(rng, P, center, R, r, rot=None):
    """P points uniform by area on a torus with axis z (then rotated by ``rot``).

    Tube angle v is drawn by rejection with acceptance (R + r cos v)/(R + r),
    which is the area element normalised to its maximum.
    """
    out_u = np.empty(0)
    out_v = np.empty(0)
    while out_u.size < P:
        m = 2 * (P - out_u.size) + 64
        u = rng.uniform(0.0, 2 * np.pi, m)
        v = rng.uniform(0.0, 2 * np.pi, m)
        acc = rng.uniform(0.0, 1.0, m) < (R + r * np.cos(v)) / (R + r)
        out_u = np.concatenate([out_u, u[acc]])
        out_v = np.concatenate([out_v, v[acc]])
    u, v = out_u[:P], out_v[:P]
    p = np.stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)], axis=1)
    n = np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)], axis=1)
    if rot is not None:
        p = p @ rot.T
        n = n @ rot.T
    return np.asarray(center, np.float64) + p, n


def _spow(x, e):
    return np.sign(x) * np.abs(x) ** e


def superellipsoid(rng, P, center, axes, eps1, eps2, table=(2048, 4096)):
    """P points uniform by area on an axis-aligned superellipsoid (Barr).

    x(eta, omega) = (a C(eta)^e1 C(omega)^e2, b C(eta)^e1 S(omega)^e2, c S(eta)^e1)
    with signed powers. The area density is tabulated on a ``table`` grid of
    (eta, omega) cells (parallelogram area of each cell), cells are drawn in
    proportion to area and a uniform jitter places the sample inside the cell.
    Normals are the normalised gradient of the implicit function
    F = (|x/a|^(2/e2) + |y/b|^(2/e2))^(e2/e1) + |z/c|^(2/e1) - 1.
    """
    a, b, c = axes
    ne, nw = table
    eta = np.linspace(-np.pi / 2, np.pi / 2, ne + 1)
    om = np.linspace(-np.pi, np.pi, nw + 1)

    def pos(et, omg):
        ce, se = np.cos(et), np.sin(et)
        co, so = np.cos(omg), np.sin(omg)
        return np.stack([a * _spow(ce, eps1) * _spow(co, eps2),
                         b * _spow(ce, eps1) * _spow(so, eps2),
                         c * _spow(se, eps1) * np.ones_like(omg)], axis=-1)

    E, O = np.meshgrid(eta, om, indexing="ij")
    X = pos(E, O)
    d1 = X[1:, :-1] - X[:-1, :-1]
    d2 = X[:-1, 1:] - X[:-1, :-1]
    d3 = X[1:, 1:] - X[1:, :-1]
    d4 = X[1:, 1:] - X[:-1, 1:]
    area = 0.5 * (np.linalg.norm(np.cross(d1, d2), axis=-1) + np.linalg.norm(np.cross(d3, d4), axis=-1))
    del X, d1, d2, d3, d4, E, O
    prob = area.ravel() / area.sum()
    cells = rng.choice(prob.size, size=P, p=prob)
    ie, iw = np.divmod(cells, nw)
    et = eta[ie] + rng.uniform(0, 1, P) * (eta[1] - eta[0])
    omg = om[iw] + rng.uniform(0, 1, P) * (om[1] - om[0])
    p = pos(et, omg)
    # gradient of the implicit function
    with np.errstate(all="ignore"):
        ax, ay, az = np.abs(p[:, 0] / a), np.abs(p[:, 1] / b), np.abs(p[:, 2] / c)
        A = ax ** (2 / eps2) + ay ** (2 / eps2)
        pre = A ** (eps2 / eps1 - 1.0)
        gx = pre * ax ** (2 / eps2 - 1.0) * np.sign(p[:, 0]) / a
        gy = pre * ay ** (2 / eps2 - 1.0) * np.sign(p[:, 1]) / b
        gz = az ** (2 / eps1 - 1.0) * np.sign(p[:, 2]) / c
        g = np.stack([gx, gy, gz], axis=1)
    g[~np.isfinite(g)] = 0.0
    bad = np.linalg.norm(g, axis=1) == 0
    g[bad] = np.stack([np.zeros(bad.sum()), np.zeros(bad.sum()), np.where(p[bad, 2] >= 0, 1.0, -1.0)], axis=1)
    return np.asarray(center, np.float64) + p, _unit(g)


def random_rotation(rng):
    """Uniform random rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# --------------------------------------------------------------------------
# benchmark / test configurations
# --------------------------------------------------------------------------
@dataclass
class Shape:
    res: int
    sigma: float
    points: np.ndarray            # (P, 3) float32
    normals: np.ndarray           # (P, 3) float32
    points_clean: np.ndarray | None = None
    normals_clean: np.ndarray | None = None
    kind: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def P(self) -> int:
        return int(self.points.shape[0])


def config_c1(seed: int = 0) -> Shape:
    """32^3, sigma 2; 3,000 points uniform on a sphere r=0.3 at the centre."""
    rng = rng_for(seed)
    p, n = sphere(rng, 3000, (0.5, 0.5, 0.5), 0.3)
    return Shape(32, 2.0, _f32(p), _f32(n), kind="sphere")


def config_c2(seed: int = 1, P: int = 20000) -> Shape:
    """128^3, sigma 2; torus (R .25, r .1, centre z .45) U sphere (r .15, centre z .72).

    Points are split between the two surfaces in proportion to area; the
    inputs are jittered by N(0, 0.002^2) while ``points_clean`` are not.
    """
    rng = rng_for(seed)
    a_t = 4 * np.pi ** 2 * 0.25 * 0.1
    a_s = 4 * np.pi * 0.15 ** 2
    on_torus = rng.uniform(0, 1, P) < a_t / (a_t + a_s)
    nt = int(on_torus.sum())
    pt, nt_ = torus(rng, nt, (0.5, 0.5, 0.45), 0.25, 0.1)
    ps, ns = sphere(rng, P - nt, (0.5, 0.5, 0.72), 0.15)
    p = np.concatenate([pt, ps])
    n = np.concatenate([nt_, ns])
    perm = rng.permutation(P)
    p, n = p[perm], n[perm]
    pj = p + rng.normal(0.0, 0.002, p.shape)
    return Shape(128, 2.0, _f32(pj), _f32(n), _f32(p), _f32(n), kind="torus+sphere")


def config_c2_outliers(seed: int = 1, P: int = 20000, frac: float = 0.5) -> Shape:
    """C2 with a fraction of its points replaced by outliers: uniform in [0,1)^3,
    random directions, |n| ~ U[0, 0.05] (the paper's outlier setting; the
    low-locality worst case for binning). ``points_clean``/``normals_clean``
    are C2's clean surface points at the same indices."""
    base = config_c2(seed, P)
    rng = rng_for(seed + 1000)
    k = int(round(frac * P))
    idx = rng.choice(P, k, replace=False)
    p = base.points.astype(np.float64)
    n = base.normals.astype(np.float64)
    p[idx] = rng.uniform(0.0, 1.0, (k, 3))
    n[idx] = _unit(rng.standard_normal((k, 3))) * rng.uniform(0.0, 0.05, (k, 1))
    return Shape(128, 2.0, _f32(p), _f32(n), base.points_clean, base.normals_clean, kind="torus+sphere+outliers",
                 meta=dict(outliers=k))


def config_c3(seed: int = 2, P: int = 100000, table=(2048, 4096)) -> Shape:
    """256^3, sigma 2; one random superellipsoid, noisy (renormalised) normals."""
    rng = rng_for(seed)
    axes = rng.uniform(0.15, 0.35, 3)
    e1, e2 = rng.uniform(0.3, 2.0, 2)
    p, n = superellipsoid(rng, P, (0.5, 0.5, 0.5), axes, e1, e2, table)
    nn = _unit(n + rng.normal(0.0, 0.05, n.shape))
    return Shape(256, 2.0, _f32(p), _f32(nn), _f32(p), _f32(n), kind="superellipsoid",
                 meta=dict(axes=axes.tolist(), eps1=float(e1), eps2=float(e2)))


def config_c3_outliers(seed: int = 2, P: int = 100000, frac: float = 0.5) -> Shape:
    """The C3 cloud (256^3) with a fraction of its points replaced by outliers:
    uniform in [0,1)^3, random directions, |n| ~ U[0, 0.05]. With half of 100k
    points uniform, every j0 plane and every row tile holds points, so no pass
    can skip anything (the dense worst case of the byte model)."""
    base = config_c3(seed, P)
    rng = rng_for(seed + 1000)
    k = int(round(frac * P))
    idx = rng.choice(P, k, replace=False)
    p = base.points.astype(np.float64)
    n = base.normals.astype(np.float64)
    p[idx] = rng.uniform(0.0, 1.0, (k, 3))
    n[idx] = _unit(rng.standard_normal((k, 3))) * rng.uniform(0.0, 0.05, (k, 1))
    return Shape(256, 2.0, _f32(p), _f32(n), base.points_clean, base.normals_clean,
                 kind="superellipsoid+outliers", meta=dict(outliers=k))


def random_shape(rng, res: int, P: int, sigma: float = 2.0, table=(256, 512)) -> Shape:
    """One shape of the mixed batch/serving workloads: sphere, rotated torus or superellipsoid."""
    kind = ["sphere", "torus", "superellipsoid"][int(rng.integers(0, 3))]
    centre = 0.5 + rng.uniform(-0.05, 0.05, 3)
    if kind == "sphere":
        p, n = sphere(rng, P, centre, rng.uniform(0.15, 0.35))
    elif kind == "torus":
        R = rng.uniform(0.18, 0.28)
        r = rng.uniform(0.05, 0.10)
        p, n = torus(rng, P, centre, R, r, random_rotation(rng))
    else:
        axes = rng.uniform(0.15, 0.35, 3)
        e1, e2 = rng.uniform(0.3, 2.0, 2)
        p, n = superellipsoid(rng, P, centre, axes, e1, e2, table)
    return Shape(res, sigma, _f32(p), _f32(n), kind=kind)


def config_c4(seed: int = 3, n_shapes: int = 64) -> list[Shape]:
    """64 shapes, res uniform in {64, 128}, P log-uniform in [1e3, 5e4]."""
    rng = rng_for(seed)
    out = []
    for _ in range(n_shapes):
        res = int(rng.choice([64, 128]))
        P = int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e4)))))
        out.append(random_shape(rng, res, P))
    return out


def _c5_shape(args):
    res, P, seed = args
    return random_shape(rng_for(seed), res, P)


def config_c5(seed: int = 4, n_requests: int = 2000, workers: int = 1):
    """Serving request stream: res in {64,128,256}, P log-uniform [3e3, 2e5], 50/50 fwd vs fwd+bwd.

    Returns a list of (Shape, needs_backward) in arrival order; inter-arrival
    times are drawn separately by the load generator for each QPS level as
    unit-rate exponentials (``arrivals_unit``), scaled by 1/QPS. Each request's
    shape comes from its own seed (drawn from the stream's generator), so a
    process pool of ``workers`` can build them in parallel with the same result.
    """
    rng = rng_for(seed)
    specs, bwds = [], []
    for _ in range(n_requests):
        res = int(rng.choice([64, 128, 256]))
        P = int(round(math.exp(rng.uniform(math.log(3e3), math.log(2e5)))))
        bwds.append(bool(rng.uniform() < 0.5))
        specs.append((res, P, int(rng.integers(0, 2 ** 62))))
    arrivals_unit = rng.exponential(1.0, n_requests)
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            shapes = pool.map(_c5_shape, specs, chunksize=8)
    else:
        shapes = [_c5_shape(a) for a in specs]
    return list(zip(shapes, bwds)), arrivals_unit


def config_scene(seed: int = 5, P: int = 1_000_000, res: int = 1024, n_objects: int = 16,
                 table=(512, 1024)) -> Shape:
    """Large-scene stand-in for the slab solve (1024^3, sigma 2): n_objects
    spheres, rotated tori and superellipsoids of size 0.04 to 0.12 at uniform
    places in [0.12, 0.88]^3, points shared in proportion to size squared (a
    proxy for area), positions jittered by N(0, (0.25 / res)^2)."""
    rng = rng_for(seed)
    size = rng.uniform(0.04, 0.12, n_objects)
    share = size ** 2 / (size ** 2).sum()
    counts = np.floor(share * P).astype(np.int64)
    counts[: P - counts.sum()] += 1
    ps, ns = [], []
    for k in range(n_objects):
        kind = int(rng.integers(0, 3))
        c = rng.uniform(0.12, 0.88, 3)
        if kind == 0:
            p, n = sphere(rng, int(counts[k]), c, size[k])
        elif kind == 1:
            p, n = torus(rng, int(counts[k]), c, size[k], size[k] * rng.uniform(0.25, 0.45), random_rotation(rng))
        else:
            axes = size[k] * rng.uniform(0.5, 1.0, 3)
            e1, e2 = rng.uniform(0.3, 2.0, 2)
            p, n = superellipsoid(rng, int(counts[k]), c, axes, e1, e2, table)
        ps.append(p)
        ns.append(n)
    p = np.concatenate(ps)
    n = np.concatenate(ns)
    perm = rng.permutation(P)
    p, n = p[perm], n[perm]
    pj = p + rng.normal(0.0, 0.25 / res, p.shape)
    return Shape(res, 2.0, _f32(pj), _f32(n), _f32(p), _f32(n), kind="scene", meta=dict(objects=n_objects))


def thin_plate(seed: int, P: int, res: int, half_thickness: float = 0.006, table=(256, 512)) -> Shape:
    """A thin closed plate: P points by area on a flat superellipsoid with axes
    (half_thickness, 0.3, 0.3) along grid axes (0, 1, 2) (exponents 0.5 across
    the plate, 1.0 round its rim), centred on the middle of cell res/2 along
    axis 0, so at 64^3 every point sits in one floor plane. Its two faces carry
    opposite normals a fraction of a cell apart: they cancel inside the
    splat's cells (the case that stresses the splat's summation precision)."""
    rng = rng_for(seed)
    centre = ((res // 2 + 0.5) / res, 0.5, 0.5)
    # generated thin along z (the superellipsoid's eta axis), then axes rolled so z -> axis 0
    p, n = superellipsoid(rng, P, (0.0, 0.0, 0.0), (0.3, 0.3, half_thickness), 0.5, 1.0, table)
    p = p[:, [2, 0, 1]] + np.asarray(centre)
    n = n[:, [2, 0, 1]]
    return Shape(res, 2.0, _f32(p), _f32(n), kind="thin_plate", meta=dict(half_thickness=half_thickness))


def loss_gradient(res: int, seed: int) -> np.ndarray:
    """A dense stand-in for dL/dchi: float32 standard normal on the res^3 grid
    (PCG64(seed), float32 draws), the same array wherever it is drawn."""
    return rng_for(seed).standard_normal((res, res, res), dtype=np.float32)


def tiny_case(seed: int, res: int, P: int, sigma: float = 2.0, kind: str = "sphere") -> Shape:
    """Small cases for parity tests: a sphere, a torus, a small off-centre sphere,
    or a uniform cloud with random normals."""
    rng = rng_for(seed)
    if kind == "sphere":
        p, n = sphere(rng, P, 0.5 + rng.uniform(-0.05, 0.05, 3), rng.uniform(0.2, 0.35))
    elif kind == "uniform":
        p = rng.uniform(0.0, 1.0, (P, 3))
        n = rng.standard_normal((P, 3))
    elif kind == "torus":
        p, n = torus(rng, P, 0.5 + rng.uniform(-0.05, 0.05, 3), 0.25, 0.08, random_rotation(rng))
    elif kind == "small":
        # a small off-centre sphere: most grid planes and row tiles hold no point
        p, n = sphere(rng, P, np.array([0.3, 0.62, 0.45]) + rng.uniform(-0.02, 0.02, 3), 0.06)
    else:
        raise ValueError(kind)
    return Shape(res, sigma, _f32(p), _f32(n), kind=kind)
