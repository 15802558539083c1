"""The GPU splat's integer accumulation rule, simulated on the CPU (supplement Sec. A.1).

The HIP splat adds every corner contribution w * n_d of a point (supplement
Sec. A.1, v_{j<-i} = T(c_i, j/r, 1/r) n_i) to LDS as an integer,
rint(w * n_d * 2^S), and converts each vertex's integer sum back with 2^-S.
Integer sums do not depend on the order of the atomic adds, so the splat is
bitwise reproducible; the price is a fixed step 2^-S per contribution.

These tests replay that rule in NumPy (FP32 weight products in the kernel's
order, the kernel's choice of S) on the 64^3 plane spans (one j0 plane of one
channel; the points whose floor plane is j0 - 1 or j0), feed the resulting
field into the FP64 oracle's spectral solve and normalisation, and compare chi
with the oracle's own:

* the former rule, one 32-bit accumulator per sample and 2^S T max|n_d| <= 2^30
  (T = points of the span), misses the 1e-5 bar on a thin closed plate at 64^3:
  its two faces put opposite normals into the same cells, the sums cancel,
  while the step grows with T;
* the rule the kernels use now, a 64-bit accumulator per sample and
  2^S max|n_d| <= 2^30 (each contribution fits 31 bits, any sum of at most
  2^30 of them fits 61), stays at FP32 level on the same plate.
"""
import numpy as np
import pytest

import oracle
import psr_synth as S


def _exp2_above(x):
    """e with x < 2^e <= 2x (frexp exponent), for float32 x > 0: what the kernel
    reads from the exponent bits."""
    return np.frexp(np.float32(x))[1]


def _plane_spans(b0, r):
    """T, the point count of each plane span j0 (floor planes j0 - 1 and j0)."""
    cnt = np.bincount(b0, minlength=r)
    return cnt + np.roll(cnt, 1)


def simulated_splat(points, normals, r, rule):
    """The field v [3, r, r, r] the kernel's integer rule produces for plane spans.

    rule "int32_T": 2^S T maxabs <= 2^30 (the former kernel rule);
    rule "int64":   2^S maxabs <= 2^30 (the current kernel rule).
    """
    x = points.astype(np.float64)
    u = x - np.floor(x)
    t = u * r
    b = np.floor(t).astype(np.int64) % r
    f = (t - np.floor(t)).astype(np.float32)  # exact in FP32 (r a power of two)
    one = np.float32(1.0)
    T = _plane_spans(b[:, 0], r)
    v = np.zeros((3, r, r, r))
    for d in range(3):
        val = normals[:, d].astype(np.float32)
        absn = np.abs(val)
        # per floor plane max|n_d|, then per span (floor planes j0 - 1 and j0)
        mx_floor = np.zeros(r, dtype=np.float32)
        np.maximum.at(mx_floor, b[:, 0], absn)
        mx = np.maximum(mx_floor, np.roll(mx_floor, 1))
        acc = np.zeros((r, r, r), dtype=np.int64)
        for o0 in (0, 1):
            j0 = (b[:, 0] + o0) % r
            if rule == "int32_T":
                bound = (T[j0].astype(np.float32) * mx[j0]).astype(np.float32)
            else:
                bound = mx[j0]
            S_ = np.where(bound > 0, 30 - np.array([_exp2_above(q) if q > 0 else 0 for q in bound]), 0)
            sc = np.ldexp(np.float32(1.0), S_).astype(np.float32)
            w0 = f[:, 0] if o0 else one - f[:, 0]
            for o1 in (0, 1):
                w1 = f[:, 1] if o1 else one - f[:, 1]
                j1 = (b[:, 1] + o1) % r
                for o2 in (0, 1):
                    w2 = f[:, 2] if o2 else one - f[:, 2]
                    # FP32 products in each kernel's order
                    if rule == "int32_T":
                        w = ((w0 * w1) * val) * w2
                    else:
                        w = ((w2 * w0) * w1) * val
                    q = np.rint((w * sc).astype(np.float32)).astype(np.int64)
                    if rule == "int32_T":
                        assert np.abs(q).max() < 2 ** 31
                    j2 = (b[:, 2] + o2) % r
                    np.add.at(acc, (j0, j1, j2), q)
        if rule == "int32_T":
            # the former bound keeps every partial sum inside 31 bits
            assert np.abs(acc).max() < 2 ** 31
        # back to floats: (float) sum * 2^-S of the plane's S
        for j0 in range(r):
            bound = (T[j0] * mx[j0]) if rule == "int32_T" else mx[j0]
            s = 30 - _exp2_above(np.float32(bound)) if bound > 0 else 0
            v[d, j0] = acc[j0].astype(np.float32).astype(np.float64) * 2.0 ** (-s)
    return v


def chi_from_field(v, points, r, sigma, m=0.5):
    """The oracle's steps after the splat (main Eqs. 3-4, reading B) on a given field."""
    chi_p, _ = oracle.spectral_solve(v, sigma)
    mu = oracle.gather(chi_p, points.astype(np.float64), r).mean()
    c = chi_p[0, 0, 0] - mu
    return m / abs(c) * (chi_p - mu)


def _err(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def plate64():
    sh = S.thin_plate(0, 60000, 64)
    ref, _ = oracle.forward(sh.points, sh.normals, 64, 2.0)
    return sh, ref


def test_plate_lies_in_one_floor_plane(plate64):
    sh, ref = plate64
    b0 = np.floor(sh.points[:, 0].astype(np.float64) * 64)
    assert np.unique(b0).size == 1
    # well conditioned: max|chi| / m stays near 1, so chi errors are not amplified
    assert np.abs(ref).max() / 0.5 < 1.5


def test_former_int32_rule_misses_the_bar_on_a_thin_plate(plate64):
    sh, ref = plate64
    v = simulated_splat(sh.points, sh.normals, 64, "int32_T")
    e = _err(chi_from_field(v, sh.points, 64, 2.0), ref)
    assert e > 3e-5, e  # measured 1.9e-4


def test_int64_rule_holds_the_bar_on_a_thin_plate(plate64):
    sh, ref = plate64
    v = simulated_splat(sh.points, sh.normals, 64, "int64")
    vo = oracle.splat(sh.points, sh.normals, 64)
    assert _err(v, vo) < 1e-6
    e = _err(chi_from_field(v, sh.points, 64, 2.0), ref)
    assert e < 1e-6, e
