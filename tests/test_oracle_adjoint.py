"""Pins of the oracle's adjoint T (synthesis): the dot-product identity, the
closed-form inverse Fourier transform of a basis function (Eq.(IFT_FB), with
the sign of i^k derived from the Jacobi-Anger expansion), and the near-unitary
spectrum of T*T claimed in Sec. II-B (Fig. TTT)."""

import math

import numpy as np
import pytest
from scipy import special

import oracle


def _random_coeffs(pl, n, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((n, pl.p_half)) + 1j * rng.standard_normal((n, pl.p_half))
    b[:, :pl.p[0]] = b[:, :pl.p[0]].real
    return b


@pytest.mark.parametrize("L,c,R", [(16, 0.5, 8), (15, 0.5, 7.5), (32, 0.5, 16)])
def test_dot_product_identity(L, c, R):
    pl = oracle.plan(L, c, R)
    I = np.random.default_rng(4).standard_normal((3, L, L))
    b = _random_coeffs(pl, 3, 5)
    lhs = oracle.coeff_inner(oracle.expand(I, pl), b, pl)
    rhs = np.sum(I * oracle.adjoint(b, pl), axis=(1, 2))
    assert np.max(np.abs(lhs - rhs) / np.abs(lhs)) <= 1e-12


def _ift_fb(pl, k, q, x1, x2):
    """F^{-1}(psi_c^{k,q})(r, phi) = 2 c sqrt(pi) (-1)^q i^k R J_k(2 pi c r) e^{ik phi} / ((2 pi c r)^2 - R^2)
    (Eq.(IFT_FB) with i^k in the numerator)."""
    c = pl.c
    Rkq = pl.roots[k][q - 1]
    r = np.hypot(x1, x2)
    phi = np.arctan2(x2, x1)
    z = 2 * math.pi * c * r
    return (2 * c * math.sqrt(math.pi) * (-1) ** q * (1j) ** k * Rkq * special.jv(k, z)
            * np.exp(1j * k * phi) / (z ** 2 - Rkq ** 2))


@pytest.mark.parametrize("k,q", [(0, 1), (0, 4), (1, 1), (1, 6), (2, 3), (3, 2), (7, 4), (12, 1)])
def test_adjoint_matches_closed_form_basis_image(k, q):
    L, c, R = 32, 0.5, 16
    pl = oracle.plan(L, c, R)
    e = np.zeros((1, pl.p_half), dtype=complex)
    e[0, pl.coef_off[k] + q - 1] = 1.0
    img = oracle.adjoint(e, pl)[0]
    x = oracle.pixel_coords(L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    inside = np.hypot(X1, X2) < R
    f = _ift_fb(pl, k, q, X1, X2)
    # coefficient vector e_{kq} with a_{-k,q} = conj(a_{k,q}) represents psi^{kq} + psi^{-k,q}
    ref = f.real if k == 0 else 2.0 * f.real
    err = np.max(np.abs(img - ref)[inside])
    assert err <= 1e-7 * np.max(np.abs(ref)), err


def test_printed_sign_would_fail_for_odd_k():
    # The printed 1/i^k differs from i^k by (-1)^k: a real check that the test above
    # discriminates between the two readings.
    L, c, R = 32, 0.5, 16
    pl = oracle.plan(L, c, R)
    k, q = 1, 2
    e = np.zeros((1, pl.p_half), dtype=complex)
    e[0, pl.coef_off[k] + q - 1] = 1.0
    img = oracle.adjoint(e, pl)[0]
    x = oracle.pixel_coords(L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    inside = np.hypot(X1, X2) < R
    printed = 2.0 * ((-1) ** k * _ift_fb(pl, k, q, X1, X2)).real
    assert np.max(np.abs(img - printed)[inside]) > 0.5 * np.max(np.abs(printed))


def _real_matrix_of_expand(pl):
    """T* as a real P x L^2 matrix in coordinates where the coefficient inner
    product is Euclidean: a_{0q} -> a_{0q}; a_{kq} (k>0) -> sqrt2 Re, sqrt2 Im."""
    L = pl.L
    eye = np.eye(L * L).reshape(L * L, L, L)
    A = oracle.expand(eye, pl, chunk=256)                     # [L^2, p_half]
    p0 = pl.p[0]
    cols = [A[:, :p0].real, math.sqrt(2) * A[:, p0:].real, math.sqrt(2) * A[:, p0:].imag]
    return np.concatenate(cols, axis=1).T                   # [P, L^2]


def test_near_unitarity_of_TstarT():
    """Sec. II-B, Fig. TTT: most eigenvalues of T*T are 1 and the smallest are close to 1."""
    pl = oracle.plan(32, 0.5, 16)
    M = _real_matrix_of_expand(pl)
    assert M.shape[0] == pl.p_total
    ev = np.linalg.eigvalsh(M @ M.T)
    assert abs(np.median(ev) - 1.0) < 1e-3
    assert np.mean(np.abs(ev - 1.0) < 1e-2) > 0.8
    assert ev.max() < 1.01 and ev.min() > 0.8


def test_adjoint_is_synthesis_left_inverse_on_basis():
    """T* T e_{kq} is close to e_{kq} (near-unitarity, Sec. II-B): a sanity level
    of agreement, not a parity gate."""
    pl = oracle.plan(32, 0.5, 16)
    for k, q in [(0, 2), (3, 3), (10, 1)]:
        e = np.zeros((1, pl.p_half), dtype=complex)
        e[0, pl.coef_off[k] + q - 1] = 1.0
        back = oracle.expand(oracle.adjoint(e, pl), pl)[0]
        assert np.max(np.abs(back - e[0])) < 1e-2


@pytest.mark.parametrize("k,q", [(0, 4), (3, 2), (12, 1)])
def test_adjoint_pixels_matches_closed_form(k, q):
    """The pixel-sampled adjoint at scattered pixels inside the disk against the closed form
    of Eq.(IFT_FB), and against the whole-image adjoint for random coefficients."""
    L, c, R = 32, 0.5, 16
    pl = oracle.plan(L, c, R)
    x = oracle.pixel_coords(L)
    rng = np.random.default_rng(7)
    rows, cols = [], []
    while len(rows) < 24:
        r, cc = rng.integers(0, L, 2)
        if math.hypot(x[r], x[cc]) < R:
            rows.append(int(r))
            cols.append(int(cc))
    e = np.zeros((1, pl.p_half), dtype=complex)
    e[0, pl.coef_off[k] + q - 1] = 1.0
    got = oracle.adjoint_pixels(e, pl, rows, cols)[0]
    f = _ift_fb(pl, k, q, x[rows], x[cols])
    ref = f.real if k == 0 else 2.0 * f.real
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))
    b = _random_coeffs(pl, 2, 9)
    full = oracle.adjoint(b, pl)
    assert np.max(np.abs(oracle.adjoint_pixels(b, pl, rows, cols) - full[:, rows, cols])) <= 1e-12 * np.max(np.abs(full))
