"""Pins of the FP64 oracle against values the paper and mathematics fix.

None of these re-types the oracle's own formulas: each compares it with an
independent statement (the tent-function form of the trilinear weight, the
DFT's defining sum, single-Fourier-mode closed forms, the dense periodic
spectral-differentiation matrices of Trefethen, adjoint identities, central
finite differences, invariants of Eq. 2).
"""
import json
import os

import numpy as np
import pytest

import oracle
import psr_synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def tent_weight(c, r):
    """T(c, j/r, 1/r) for every vertex j: prod_a max(0, 1 - r*|minimum-image distance|).

    The trilinear weight written as a tent (hat) function of the distance to the
    vertex, supplement Sec. A.1, evaluated over ALL vertices (brute force).
    """
    j = np.arange(r) / r
    out = np.ones((r, r, r))
    for a, shape in enumerate([(r, 1, 1), (1, r, 1), (1, 1, r)]):
        d = (c[a] - j + 0.5) % 1.0 - 0.5
        out = out * np.maximum(0.0, 1.0 - r * np.abs(d)).reshape(shape)
    return out


# ---------------------------------------------------------------- splat / gather
def test_splat_worked_example_golden():
    g = json.load(open(os.path.join(GOLDEN, "splat_worked_example.json")))
    r = g["res"]
    c = np.array([g["point"]])
    n = np.array([g["normal"]])
    v = oracle.splat(c, n, r)
    expect = np.zeros((3, r, r, r))
    for e in g["nonzero_vertices"]:
        j = tuple(e["j"])
        for d in range(3):
            expect[(d,) + j] = e["weight"] * g["normal"][d]
    assert np.array_equal(v, expect)  # exact in binary
    jj = np.indices((r, r, r))
    ramp = jj[0] + 10.0 * jj[1] + 100.0 * jj[2]
    assert oracle.gather(ramp, c, r)[0] == g["gather_of_ramp"]["value"]


@pytest.mark.parametrize("r", [4, 8, 16])
def test_splat_matches_brute_force_tent(r):
    rng = _rng(r)
    P = 40
    c = rng.uniform(-0.5, 1.5, (P, 3))  # includes wrap-around positions
    c[0] = [0.0, 0.5, 1.0 - 1e-12]
    c[1] = [3.0 / r, 0.0, 1.0 / r]      # exactly on vertices
    n = rng.standard_normal((P, 3))
    v = oracle.splat(c, n, r)
    ref = np.zeros((3, r, r, r))
    for i in range(P):
        T = tent_weight(c[i], r)
        for d in range(3):
            ref[d] += T * n[i, d]
    np.testing.assert_allclose(v, ref, rtol=0, atol=1e-12)


def test_splat_partition_of_unity():
    rng = _rng(7)
    c = rng.uniform(0, 1, (500, 3))
    n = rng.standard_normal((500, 3))
    v = oracle.splat(c, n, 16)
    np.testing.assert_allclose(v.reshape(3, -1).sum(1), n.sum(0), rtol=1e-12)
    W = oracle.splat_scalar(c, 16)
    assert abs(W.sum() - 500) < 1e-9


@pytest.mark.parametrize("r", [4, 8])
def test_gather_matches_brute_force_and_is_splat_transpose(r):
    rng = _rng(11 + r)
    P = 30
    c = rng.uniform(0, 1, (P, 3))
    n = rng.standard_normal((P, 3))
    u = rng.standard_normal((3, r, r, r))
    for i in range(P):
        T = tent_weight(c[i], r)
        np.testing.assert_allclose(oracle.gather(u[0], c[i:i + 1], r)[0], (T * u[0]).sum(), atol=1e-12)
    lhs = (oracle.splat(c, n, r) * u).sum()
    rhs = sum((n[:, d] * oracle.gather(u[d], c, r)).sum() for d in range(3))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_gather_grad_fd():
    rng = _rng(3)
    r = 8
    c = rng.uniform(0.1, 0.9, (20, 3))
    u = rng.standard_normal((r, r, r))
    g = oracle.gather_grad(u, c, r)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (oracle.gather(u, c + e, r) - oracle.gather(u, c - e, r)) / (2 * h)
        frac = (r * c[:, a]) % 1.0
        ok = (frac > 1e-3) & (frac < 1 - 1e-3)
        np.testing.assert_allclose(g[ok, a], fd[ok], rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------- transforms
@pytest.mark.parametrize("r", [4, 8])
def test_fft_matches_naive_dft(r):
    rng = _rng(r)
    x = rng.standard_normal((r, r, r)) + 1j * rng.standard_normal((r, r, r))
    j = np.indices((r, r, r)).reshape(3, -1)
    k = j
    # defining sum: X(k) = sum_j x[j] exp(-2 pi i k.j / r)
    phase = np.exp(-2j * np.pi * (k.T @ j) / r)
    X = (phase @ x.ravel()).reshape(r, r, r)
    np.testing.assert_allclose(oracle.fft3(x), X, atol=1e-9)
    xi = (np.conj(phase).T @ X.ravel()).reshape(r, r, r) / r ** 3
    np.testing.assert_allclose(oracle.ifft3(X), xi, atol=1e-12)
    np.testing.assert_allclose(oracle.ifft3(oracle.fft3(x)), x, atol=1e-12)


def _mode_grid(r, k):
    jj = np.indices((r, r, r)).astype(np.float64) / r
    return 2 * np.pi * (k[0] * jj[0] + k[1] * jj[1] + k[2] * jj[2])


@pytest.mark.parametrize("r,k,d,sigma", [
    (8, (1, 0, 0), 0, 2.0), (8, (1, 2, -3), 1, 2.0), (16, (-3, 5, 2), 2, 1.5),
    (16, (7, -7, 1), 0, 3.0), (32, (2, -9, 15), 1, 2.0), (8, (0, 0, 3), 2, 0.0),
])
def test_spectral_single_mode_closed_form(r, k, d, sigma):
    """v_d = cos(2 pi k.x) -> chi' = g k_d sin(2 pi k.x)/(2 pi |k|^2); v_d = sin -> -g k_d cos/(...)."""
    th = _mode_grid(r, k)
    k2 = float(np.dot(k, k))
    g = np.exp(-2 * sigma ** 2 * k2 / r ** 2)
    v = np.zeros((3, r, r, r))
    v[d] = np.cos(th)
    chi, _ = oracle.spectral_solve(v, sigma)
    np.testing.assert_allclose(chi, g * k[d] * np.sin(th) / (2 * np.pi * k2), atol=1e-12)
    v[d] = np.sin(th)
    chi, _ = oracle.spectral_solve(v, sigma)
    np.testing.assert_allclose(chi, -g * k[d] * np.cos(th) / (2 * np.pi * k2), atol=1e-12)


@pytest.mark.parametrize("r", [8, 16])
def test_spectral_nyquist_conventions(r):
    """Odd factor 0 at Nyquist; |kappa|^2 keeps (r/2)^2 (seen through the Gaussian and the Laplacian)."""
    sigma = 2.0
    jj = np.indices((r, r, r)).astype(np.float64)
    alt = (-1.0) ** jj[0]
    v = np.zeros((3, r, r, r))
    v[0] = alt
    chi, _ = oracle.spectral_solve(v, sigma)
    assert np.abs(chi).max() < 1e-13
    v[:] = 1.0
    chi, _ = oracle.spectral_solve(v, sigma)
    assert np.abs(chi).max() < 1e-13
    ky = 3
    v = np.zeros((3, r, r, r))
    v[1] = alt * np.cos(2 * np.pi * ky * jj[1] / r)
    chi, _ = oracle.spectral_solve(v, sigma)
    K2 = (r / 2) ** 2 + ky ** 2
    expect = np.exp(-2 * sigma ** 2 * K2 / r ** 2) * ky * alt * np.sin(2 * np.pi * ky * jj[1] / r) / (2 * np.pi * K2)
    np.testing.assert_allclose(chi, expect, atol=1e-13)


def trefethen_D(N):
    """Periodic spectral first-derivative matrix on [0, 2pi), N even (Trefethen 2000, ch. 3)."""
    h = 2 * np.pi / N
    i = np.arange(N)
    diff = i[:, None] - i[None, :]
    with np.errstate(divide="ignore"):
        D = 0.5 * (-1.0) ** diff / np.tan(diff * h / 2)
    D[diff == 0] = 0.0
    return D


def trefethen_D2(N):
    """Periodic spectral second-derivative matrix on [0, 2pi), N even (Trefethen 2000, ch. 3)."""
    h = 2 * np.pi / N
    i = np.arange(N)
    diff = i[:, None] - i[None, :]
    with np.errstate(divide="ignore"):
        D2 = -0.5 * (-1.0) ** diff / np.sin(diff * h / 2) ** 2
    D2[diff == 0] = -np.pi ** 2 / (3 * h ** 2) - 1.0 / 6.0
    return D2


@pytest.mark.parametrize("r,sigma", [(4, 2.0), (8, 2.0), (8, 0.0), (8, 5.0)])
def test_spectral_solve_matches_dense_trefethen(r, sigma):
    """chi' = (G1 x G1 x G1) L^+ (Dx vx + Dy vy + Dz vz), FFT-free, on the unit domain."""
    rng = _rng(100 + r)
    v = rng.standard_normal((3, r, r, r))
    D = 2 * np.pi * trefethen_D(r)
    D2 = (2 * np.pi) ** 2 * trefethen_D2(r)
    I = np.eye(r)
    kron3 = lambda a, b, c: np.kron(np.kron(a, b), c)
    L = kron3(D2, I, I) + kron3(I, D2, I) + kron3(I, I, D2)
    div = kron3(D, I, I) @ v[0].ravel() + kron3(I, D, I) @ v[1].ravel() + kron3(I, I, D) @ v[2].ravel()
    j = np.arange(r)
    kappa = np.where(j < r // 2, j, j - r)
    g1 = np.exp(-2 * sigma ** 2 * kappa ** 2 / r ** 2)
    col = np.array([(g1 * np.cos(2 * np.pi * j * m / r)).sum() / r for m in range(r)])
    G1 = np.array([[col[(a - b) % r] for b in range(r)] for a in range(r)])
    chi_dense = kron3(G1, G1, G1) @ (np.linalg.pinv(L) @ div)
    chi, _ = oracle.spectral_solve(v, sigma)
    np.testing.assert_allclose(chi.ravel(), chi_dense, atol=1e-10 * np.abs(chi_dense).max())


def test_spectral_adjoint_dot_product():
    rng = _rng(5)
    r, sigma = 8, 2.0
    v = rng.standard_normal((3, r, r, r))
    h = rng.standard_normal((r, r, r))
    chi, _ = oracle.spectral_solve(v, sigma)
    A = oracle.spectral_factor(r, sigma)
    adj = oracle.ifft3(np.conj(A) * oracle.fft3(h)[None]).real
    assert abs((chi * h).sum() - (v * adj).sum()) < 1e-12


# ---------------------------------------------------------------- normalisation / invariants
def test_normalisation_constraints_eq2():
    sh = S.tiny_case(1, 16, 300)
    chi, aux = oracle.forward(sh.points, sh.normals, 16, 2.0)
    assert abs(abs(chi[0, 0, 0]) - 0.5) < 1e-15          # |chi(0)| = m
    assert abs(oracle.gather(chi, sh.points, 16).mean()) < 1e-15  # chi = 0 at the points (mean)
    chiA, auxA = oracle.forward(sh.points, sh.normals, 16, 2.0, reading="A")
    assert abs(auxA["s"] * abs(auxA["c0"]) - 0.5) < 1e-15


def test_scale_and_sign_invariance():
    sh = S.tiny_case(2, 16, 200, kind="torus")
    chi, _ = oracle.forward(sh.points, sh.normals, 16, 2.0)
    chi2, _ = oracle.forward(sh.points, 3.5 * sh.normals.astype(np.float64), 16, 2.0)
    chi3, _ = oracle.forward(sh.points, -sh.normals.astype(np.float64), 16, 2.0)
    np.testing.assert_allclose(chi2, chi, atol=1e-13)
    np.testing.assert_allclose(chi3, -chi, atol=1e-13)


def test_shift_rolls_chi_prime():
    r = 16
    rng = _rng(9)
    c = rng.integers(0, 2 ** 10, (100, 3)) / 2 ** 10   # dyadic, so shifts are exact
    n = rng.standard_normal((100, 3))
    _, aux = oracle.forward(c, n, r, 2.0)
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0 / r
        _, aux2 = oracle.forward(c + e, n, r, 2.0)
        np.testing.assert_allclose(aux2["chi_prime"], np.roll(aux["chi_prime"], 1, axis=a), atol=1e-13)
        assert abs(aux2["mu"] - aux["mu"]) < 1e-13


def test_axis_permutation_and_point_order():
    sh = S.tiny_case(4, 16, 250, kind="uniform")
    c, n = sh.points.astype(np.float64), sh.normals.astype(np.float64)
    chi, _ = oracle.forward(c, n, 16, 2.0)
    perm = [2, 0, 1]
    chip, _ = oracle.forward(c[:, perm], n[:, perm], 16, 2.0)
    np.testing.assert_allclose(chip, np.transpose(chi, perm), atol=1e-12)
    order = _rng(1).permutation(250)
    chio, _ = oracle.forward(c[order], n[order], 16, 2.0)
    np.testing.assert_allclose(chio, chi, atol=1e-13)


def test_sphere_sanity_c1():
    sh = S.config_c1()
    chi, _ = oracle.forward(sh.points, sh.normals, 32, 2.0)
    r = 32
    x = np.indices((r, r, r)).reshape(3, -1).T / r
    d = np.linalg.norm(x - 0.5, axis=1)
    inside = chi.ravel()[d < 0.3 - 3 / r]
    outside = chi.ravel()[d > 0.3 + 3 / r]
    assert -0.65 <= inside.mean() <= -0.50 and inside.std() < 0.03
    assert abs(outside.mean() - 0.5) < 0.01 and outside.std() < 0.03


def test_degenerate_zero_normals():
    c = _rng(0).uniform(0, 1, (10, 3))
    chi, aux = oracle.forward(c, np.zeros((10, 3)), 8, 2.0)
    assert aux["status"] == "degenerate" and np.isnan(chi).all()


# ---------------------------------------------------------------- gradients
@pytest.mark.parametrize("reading", ["B", "A"])
def test_backward_matches_central_fd(reading):
    r, P, h = 16, 120, 1e-5
    sh = S.tiny_case(6, r, P, kind="torus")
    c, n = sh.points.astype(np.float64), sh.normals.astype(np.float64) * 0.7
    G = _rng(12).standard_normal((r, r, r))
    _, aux = oracle.forward(c, n, r, 2.0, reading=reading)
    dc, dn = oracle.backward(aux, G)
    L = lambda cc, nn: (G * oracle.forward(cc, nn, r, 2.0, reading=reading)[0]).sum()
    rng = _rng(13)
    scale = max(np.abs(dc).max(), np.abs(dn).max())
    checked = 0
    for _ in range(60):
        i, a = rng.integers(0, P), rng.integers(0, 3)
        frac = (r * c[i, a]) % 1.0
        if not (2 * r * h < frac < 1 - 2 * r * h):
            continue
        e = np.zeros_like(c)
        e[i, a] = h
        fd_c = (L(c + e, n) - L(c - e, n)) / (2 * h)
        fd_n = (L(c, n + e) - L(c, n - e)) / (2 * h)
        assert abs(fd_c - dc[i, a]) <= 1e-6 * max(abs(fd_c), 1e-3 * scale)
        assert abs(fd_n - dn[i, a]) <= 1e-6 * max(abs(fd_n), 1e-3 * scale)
        checked += 1
    assert checked >= 20
