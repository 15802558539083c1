"""Plant plausible mistakes in the oracle (on the CPU) and check the pins catch each one.

Each mutation patches one oracle function with a version that carries a
typical bug (dropped term, wrong sign or index, transposed operand, wrong
convention). The test passes only if at least one pin of
``test_oracle_pins`` fails under that mutation.

(Keeping the odd factor -r/2 at the Nyquist index is *not* in this list: on a
real field that term is anti-Hermitian, so the real part of the inverse
removes it exactly and the oracle's result is unchanged.)
"""
import numpy as np
import pytest

import oracle
from oracle import dpsr
import test_oracle_pins as pins

_orig_factor = dpsr.spectral_factor
_orig_fft3 = dpsr.fft3
_orig_ifft3 = dpsr.ifft3
_orig_weights = dpsr.corner_weights
_orig_wgrads = dpsr.corner_weight_grads
_orig_backward = dpsr.backward
_orig_forward = dpsr.forward


def factor_sign(r, sigma):
    return -_orig_factor(r, sigma)


def factor_no_gauss(r, sigma):
    return _orig_factor(r, 0.0)


def factor_half_exponent(r, sigma):
    return _orig_factor(r, sigma / np.sqrt(2.0))


def factor_nyquist_dropped(r, sigma):
    # a common shortcut: discard the Nyquist planes altogether
    A = _orig_factor(r, sigma).copy()
    h = r // 2
    A[:, h, :, :] = 0
    A[:, :, h, :] = 0
    A[:, :, :, h] = 0
    return A


def factor_axes_swapped(r, sigma):
    A = _orig_factor(r, sigma)
    return A[[2, 1, 0]]


def fft_sign_flipped(x):
    n = np.prod(x.shape[-3:])
    return np.fft.ifftn(x, axes=(-3, -2, -1)) * n


def ifft_unnormalised(X):
    n = np.prod(X.shape[-3:])
    return _orig_ifft3(X) * n


def weights_swapped(f):
    return _orig_weights(1.0 - f)


def wgrads_sign(f, r):
    return -_orig_wgrads(f, r)


def forward_reading_b_uses_c0(c, n, r, sigma, m=0.5, reading="B"):
    chi, aux = _orig_forward(c, n, r, sigma, m=m, reading="A")
    aux["reading"] = reading
    return chi, aux


def backward_drops_delta(aux, G):
    # adjoint without the -Q delta_0 term (forgets that chi'(0) sets the scale)
    return _backward_variant(aux, G, drop_delta=True)


def backward_no_conj(aux, G):
    return _backward_variant(aux, G, no_conj=True)


def _backward_variant(aux, G, drop_delta=False, no_conj=False):
    c, n, r = aux["c"], aux["n"], aux["r"]
    P = c.shape[0]
    s, chi, cs = aux["s"], aux["chi"], aux["cscale"]
    Q = (G * chi).sum() / cs
    g_mu = -s * G.sum() + (Q if aux["reading"] == "B" else 0.0)
    H = s * G + (g_mu / P) * dpsr.splat_scalar(c, r)
    if not drop_delta:
        H[0, 0, 0] -= Q
    A = _orig_factor(r, aux["sigma"])
    op = A if no_conj else np.conj(A)
    gv = _orig_ifft3(op * _orig_fft3(H)[None]).real
    dn = np.stack([dpsr.gather(gv[d], c, r) for d in range(3)], axis=1)
    b, f = dpsr.cell_coords(c, r)
    dw = _orig_wgrads(f, r)
    idx = dpsr._corner_index(b, r)
    field = sum(n[:, None, d] * gv[d].ravel()[idx] for d in range(3)) + (g_mu / P) * aux["chi_prime"].ravel()[idx]
    dc = (dw * field[:, :, None]).sum(axis=1)
    return dc, dn


PINS = [
    lambda: pins.test_splat_worked_example_golden(),
    lambda: pins.test_splat_matches_brute_force_tent(8),
    lambda: pins.test_gather_grad_fd(),
    lambda: pins.test_fft_matches_naive_dft(4),
    lambda: pins.test_spectral_single_mode_closed_form(16, (-3, 5, 2), 2, 1.5),
    lambda: pins.test_spectral_single_mode_closed_form(16, (7, -7, 1), 0, 3.0),
    lambda: pins.test_spectral_nyquist_conventions(8),
    lambda: pins.test_spectral_solve_matches_dense_trefethen(8, 2.0),
    lambda: pins.test_normalisation_constraints_eq2(),
    lambda: pins.test_backward_matches_central_fd("B"),
]

MUTATIONS = {
    "operator sign flipped": ("spectral_factor", factor_sign),
    "Gaussian dropped": ("spectral_factor", factor_no_gauss),
    "Gaussian exponent halved": ("spectral_factor", factor_half_exponent),
    "Nyquist planes dropped": ("spectral_factor", factor_nyquist_dropped),
    "operator axes transposed": ("spectral_factor", factor_axes_swapped),
    "FFT sign flipped": ("fft3", fft_sign_flipped),
    "inverse FFT missing 1/N": ("ifft3", ifft_unnormalised),
    "trilinear weights swapped": ("corner_weights", weights_swapped),
    "weight gradient sign": ("corner_weight_grads", wgrads_sign),
    "scale reading B computed as A": ("forward", forward_reading_b_uses_c0),
    "adjoint drops delta_0 term": ("backward", backward_drops_delta),
    "adjoint without conjugate": ("backward", backward_no_conj),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(dpsr, attr, fn)
    monkeypatch.setattr(oracle, attr, fn)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failures += 1
    assert failures >= 1, f"no pin caught: {name}"
