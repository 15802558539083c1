"""FP64 CPU oracle of the differentiable Poisson solver (DPSR) -- TEST INFRASTRUCTURE.

This module is the plain, slow, obviously-correct statement of what the GPU
library computes. Only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import it; the product path never does.

Each function follows a passage of Peng et al., "Shape As Points: A
Differentiable Poisson Solver" (NeurIPS 2021):

  * splat / gather    -- supplement Sec. A.1 "Point Rasterization" (the
                         trilinear weight T(c_i, s*j + c0, s) and the sum over
                         the neighbourhood N_j), main Sec. 3.1.
  * spectral solve    -- main Eq. (3) and supplement Sec. A.2 (divergence
                         2*pi*i(u . v~), Laplacian -4*pi^2 |u|^2, Gaussian
                         g = exp(-2 sigma^2 |u|^2 / r^2), FT sign e^{-2 pi i x.u}).
  * normalisation     -- main Eq. (4) / supplement "chi" equation, with the
                         constraint of main Eq. (2) (|chi(0)| = m, m = 0.5).
  * adjoint           -- the paper differentiates with autograd (Sec. 3.1,
                         Sec. 3.2 "Backward pass"); the adjoint here is the
                         exact derivative of the forward above, derived by hand.

Readings taken where the paper is silent or ambiguous (each one is listed in
the design notes of the repository):
  grid       domain [0,1)^3, c0 = 0, voxel size 1/r, vertex j at j/r; periodic
             (the FFT implies it): points are taken mod 1 and corner indices
             wrap mod r.
  corners    always the floor vertex b and b+1 per axis, weights (1-f, f).
  units      u is the integer wavenumber kappa (k for k < r/2, else k - r), so
             sigma is measured in grid cells.
  dot        "i u (.) v~" in the supplement is read as the dot product of main
             Eq. (3).
  Nyquist    the odd (derivative) factor kappa_d is 0 at k_d = r/2, while
             |kappa|^2 keeps (r/2)^2. This is what the real part of the complex
             formula gives and what the periodic spectral differentiation
             matrices give.
  DC         chi~(0) = 0.
  scale      reading "B" (default): c = chi'(0) - mean, so |chi(0)| = m holds
             exactly (main Eq. (2)); reading "A" takes abs(chi'(0)) literally
             from Eq. (4). "x = 0" is grid vertex (0,0,0).
  normals    used as given, never renormalised (supplement, outlier handling).
  FFT norm   forward unnormalised, inverse 1/N.
  degenerate c == 0 or non-finite -> chi is NaN (status "degenerate").
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "cell_coords", "corner_weights", "corner_weight_grads", "splat", "splat_scalar", "gather",
    "gather_grad", "wavenumbers", "spectral_factor", "spectral_solve", "forward", "backward",
    "fft3", "ifft3",
]

# the 8 corner offsets o in {0,1}^3, in a fixed order
OFFSETS = np.array([[o0, o1, o2] for o0 in (0, 1) for o1 in (0, 1) for o2 in (0, 1)], dtype=np.int64)


def cell_coords(c, r):
    """Floor vertex b (int) and fractional offset f (float64) of each point.

    Positions are wrapped into [0,1) (periodic grid), scaled by r (the voxel
    size is 1/r) and split into integer and fractional parts.
    """
    c = np.asarray(c, dtype=np.float64)
    u = c - np.floor(c)
    u = np.where(u >= 1.0, 0.0, u)
    t = r * u
    b = np.floor(t)
    f = t - b
    return b.astype(np.int64) % r, f


def corner_weights(f):
    """Trilinear weights w[i, o] = prod_a (o_a ? f_a : 1 - f_a), shape (P, 8)."""
    w = np.ones((f.shape[0], 8))
    for k, o in enumerate(OFFSETS):
        for a in range(3):
            w[:, k] *= f[:, a] if o[a] else (1.0 - f[:, a])
    return w


def corner_weight_grads(f, r):
    """d w[i, o] / d c[i, a] = r * (o_a ? +1 : -1) * prod_{b != a}(...), shape (P, 8, 3)."""
    g = np.ones((f.shape[0], 8, 3))
    for k, o in enumerate(OFFSETS):
        for a in range(3):
            g[:, k, a] = r * (1.0 if o[a] else -1.0)
            for b in range(3):
                if b != a:
                    g[:, k, a] *= f[:, b] if o[b] else (1.0 - f[:, b])
    return g


def _corner_index(b, r):
    """Flat grid index of each of the 8 corners, shape (P, 8)."""
    idx = np.empty((b.shape[0], 8), dtype=np.int64)
    for k, o in enumerate(OFFSETS):
        j = (b + o) % r
        idx[:, k] = (j[:, 0] * r + j[:, 1]) * r + j[:, 2]
    return idx


def splat(c, n, r):
    """Rasterise normals onto the grid: v_d[j] = sum_i T(c_i, j/r, 1/r) n_{i,d}.

    Supplement Sec. A.1 (v_{j<-i} and v_j equations). Returns (3, r, r, r).
    """
    b, f = cell_coords(c, r)
    w = corner_weights(f)
    idx = _corner_index(b, r)
    n = np.asarray(n, dtype=np.float64)
    v = np.zeros((3, r * r * r))
    for d in range(3):
        np.add.at(v[d], idx.ravel(), (w * n[:, d:d + 1]).ravel())
    return v.reshape(3, r, r, r)


def splat_scalar(c, r, values=None):
    """Scalar splat W[j] = sum_i T(c_i, j/r, 1/r) * values_i (values default to 1)."""
    b, f = cell_coords(c, r)
    w = corner_weights(f)
    if values is not None:
        w = w * np.asarray(values, dtype=np.float64)[:, None]
    idx = _corner_index(b, r)
    out = np.zeros(r * r * r)
    np.add.at(out, idx.ravel(), w.ravel())
    return out.reshape(r, r, r)


def gather(grid, c, r):
    """Trilinear interpolation of a periodic grid at the points (the transpose of the splat)."""
    b, f = cell_coords(c, r)
    w = corner_weights(f)
    idx = _corner_index(b, r)
    return (w * np.asarray(grid, dtype=np.float64).ravel()[idx]).sum(axis=1)


def gather_grad(grid, c, r):
    """Gradient of the trilinear interpolant w.r.t. the point position, shape (P, 3)."""
    b, f = cell_coords(c, r)
    dw = corner_weight_grads(f, r)
    idx = _corner_index(b, r)
    vals = np.asarray(grid, dtype=np.float64).ravel()[idx]
    return (dw * vals[:, :, None]).sum(axis=1)


def wavenumbers(r):
    """kappa(k) = k for k < r/2 else k - r; the odd factor is 0 at k = r/2 (Nyquist)."""
    k = np.arange(r)
    kappa = np.where(k < r // 2, k, k - r).astype(np.float64)
    kappa_odd = kappa.copy()
    if r % 2 == 0:
        kappa_odd[r // 2] = 0.0
    return kappa, kappa_odd


def fft3(x):
    """Unnormalised 3D DFT with the e^{-2 pi i k.j / r} sign (supplement FT definition)."""
    return np.fft.fftn(x, axes=(-3, -2, -1))


def ifft3(X):
    """Inverse 3D DFT with the e^{+2 pi i k.j / r} sign and 1/N normalisation."""
    return np.fft.ifftn(X, axes=(-3, -2, -1))


def spectral_factor(r, sigma):
    """A_d(k) = g(k) * i * kappa_d^odd / (-2 pi |kappa|^2), with A_d(0) = 0.

    Main Eq. (3): chi~ = g (.) i u.v~ / (-2 pi |u|^2), g = exp(-2 sigma^2 |u|^2 / r^2).
    Returns the three operator grids, shape (3, r, r, r), complex128.
    """
    kappa, kappa_odd = wavenumbers(r)
    K2 = kappa[:, None, None] ** 2 + kappa[None, :, None] ** 2 + kappa[None, None, :] ** 2
    g = np.exp(-2.0 * sigma ** 2 * K2 / r ** 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        base = g / (-2.0 * np.pi * K2)
    base[0, 0, 0] = 0.0
    A = np.empty((3, r, r, r), dtype=np.complex128)
    A[0] = 1j * base * kappa_odd[:, None, None]
    A[1] = 1j * base * kappa_odd[None, :, None]
    A[2] = 1j * base * kappa_odd[None, None, :]
    return A


def spectral_solve(v, sigma):
    """Unnormalised indicator chi' = Re IFFT( sum_d A_d * FFT(v_d) ), main Eq. (3)."""
    r = v.shape[-1]
    A = spectral_factor(r, sigma)
    chi_hat = (A * fft3(v)).sum(axis=0)
    out = ifft3(chi_hat)
    return out.real, chi_hat


def forward(c, n, r, sigma, m=0.5, reading="B"):
    """DPSR forward: splat -> spectral solve -> normalise (main Eqs. 2-4).

    Returns (chi, aux) where aux holds every intermediate the adjoint needs and
    the tests inspect: v, chi_prime, mu, c0 (chi'(0)), cscale, s, status.
    """
    c = np.asarray(c, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    v = splat(c, n, r)
    chi_p, chi_hat = spectral_solve(v, sigma)
    f = gather(chi_p, c, r)
    mu = f.mean()
    c0 = chi_p[0, 0, 0]
    cscale = (c0 - mu) if reading == "B" else c0
    status = "ok"
    if cscale == 0.0 or not np.isfinite(cscale):
        status = "degenerate"
        s = np.nan
    else:
        s = m / abs(cscale)
    chi = s * (chi_p - mu)
    aux = dict(c=c, n=n, r=r, sigma=sigma, m=m, reading=reading, v=v, chi_prime=chi_p,
               chi_hat=chi_hat, f=f, mu=mu, c0=c0, cscale=cscale, s=s, chi=chi, status=status)
    return chi, aux


def backward(aux, G):
    """Adjoint of :func:`forward`: given G = dL/dchi, return (dL/dc, dL/dn), each (P, 3).

    With chi = s (chi' - mu), s = m/|c|, mu = (1/P) sum_i gather(chi', c_i):
      S_G = sum G,  Q = sum(G chi) / c,  g_mu = -s S_G + Q   (reading B; A drops +Q)
      H   = s G + (g_mu / P) W - Q delta_0        (W = splat of ones)
      g_v_d = IFFT( conj(A_d) * FFT(H) )          (same operator and 1/N as forward)
      dL/dn_{i,d} = gather(g_v_d, c_i)
      dL/dc_{i,a} = sum_o dw/dc_a (sum_d n_{i,d} g_v_d + (g_mu/P) chi')[corner o]
    """
    c, n, r = aux["c"], aux["n"], aux["r"]
    P = c.shape[0]
    G = np.asarray(G, dtype=np.float64)
    s, chi, cs = aux["s"], aux["chi"], aux["cscale"]
    S_G = G.sum()
    Q = (G * chi).sum() / cs
    g_mu = -s * S_G + (Q if aux["reading"] == "B" else 0.0)
    W = splat_scalar(c, r)
    H = s * G + (g_mu / P) * W
    H[0, 0, 0] -= Q
    A = spectral_factor(r, aux["sigma"])
    Hh = fft3(H)
    gv = ifft3(np.conj(A) * Hh[None]).real
    dn = np.stack([gather(gv[d], c, r) for d in range(3)], axis=1)
    b, f = cell_coords(c, r)
    dw = corner_weight_grads(f, r)
    idx = _corner_index(b, r)
    field = (n[:, None, 0] * gv[0].ravel()[idx] + n[:, None, 1] * gv[1].ravel()[idx]
             + n[:, None, 2] * gv[2].ravel()[idx] + (g_mu / P) * aux["chi_prime"].ravel()[idx])
    dc = (dw * field[:, :, None]).sum(axis=1)
    return dc, dn
