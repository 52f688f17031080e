"""Pins of the oracle's real-space eigenimages (Sec. VI-B: the steerable principal
components evaluated on the pixel grid as linear combinations of Eq.(IFT_FB)).

The closed form is checked against routes that do not use it: the inverse polar
Fourier transform Eq.(IPFT) of the Fourier-space component g^{k,l} of Eq.(sPCArt),
reduced by the Jacobi-Anger expansion to a radial Hankel-type integral and evaluated by
Gauss-Legendre quadrature; the oracle's adjoint (a discrete transform of the same
coefficients); and the value at the centre pixel."""

import math

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import spca


def _random_orthogonal(p, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((p, p)))
    return q * np.sign(np.diag(r))[None, :]


@pytest.fixture(scope="module")
def pl32():
    return oracle.plan(32, 0.5, 16)


def _U(pl, seed=0):
    return [_random_orthogonal(pl.p[k], seed + k) for k in range(pl.k_max + 1)]


@pytest.mark.parametrize("k", [0, 1, 4, 9])
def test_matches_inverse_polar_transform_by_quadrature(pl32, k):
    """E^{k,l}(r, phi) = 2 pi i^k e^{ik phi} int_0^c f^{k,l}(xi) J_k(2 pi r xi) xi dxi, with
    f^{k,l}(xi) = sum_q N_{k,q} J_k(R_{k,q} xi / c) u_l(q) (Eqs.(IPFT),(sPCArt))."""
    pl = pl32
    U = _U(pl, 11)
    ls = [0, pl.p[k] - 1]
    E = spca.eigenimages(U, pl, k, ls)
    x = oracle.pixel_coords(pl.L)
    t, w = np.polynomial.legendre.leggauss(600)
    xi = pl.c * (t + 1) / 2
    wx = pl.c / 2 * w * xi
    rng = np.random.default_rng(3)
    pix = [(16, 16), (16, 17), (0, 0), (31, 5)] + [tuple(v) for v in rng.integers(0, pl.L, (12, 2))]
    for li, l in enumerate(ls):
        f = sum(pl.norms[k][q] * special.jv(k, pl.roots[k][q] * xi / pl.c) * U[k][q, l] for q in range(pl.p[k]))
        scale = np.max(np.abs(E[li]))
        for a, b in pix:
            r, phi = math.hypot(x[a], x[b]), math.atan2(x[b], x[a])
            ref = 2 * math.pi * (1j) ** k * np.exp(1j * k * phi) * np.sum(f * special.jv(k, 2 * math.pi * r * xi) * wx)
            assert abs(E[li][a, b] - ref) <= 1e-11 * scale, (k, l, a, b, E[li][a, b], ref)


@pytest.mark.parametrize("k", [0, 2, 5])
def test_matches_adjoint_of_component_coefficients(pl32, k):
    """The synthesis T of the coefficient vector u_l placed at angular frequency k (±k
    folded) samples 2 Re E^{k,l} (E^{0,l} for k = 0) inside the disk, to the accuracy of
    the discrete transform: a few 1e-6 of the peak for a combination of all p_k basis
    functions (a wrong sign or a dropped term would show at O(1))."""
    pl = pl32
    U = _U(pl, 5)
    l = 1
    a = np.zeros((1, pl.p_half), dtype=complex)
    a[0, pl.coef_off[k]:pl.coef_off[k] + pl.p[k]] = U[k][:, l]
    img = oracle.adjoint(a, pl)[0]
    E = spca.eigenimages(U, pl, k, [l])[0]
    ref = E.real if k == 0 else 2.0 * E.real
    x = oracle.pixel_coords(pl.L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    inside = np.hypot(X1, X2) < pl.R
    assert np.max(np.abs(img - ref)[inside]) <= 1e-5 * np.max(np.abs(ref))


def test_centre_pixel(pl32):
    """At r = 0, J_k(0) = 0 for k > 0, and for k = 0 each term of Eq.(IFT_FB) is
    2 c sqrt(pi) (-1)^q R / (0 - R^2)."""
    pl = pl32
    U = _U(pl, 8)
    i0 = int(np.argmin(np.abs(oracle.pixel_coords(pl.L))))
    for k in (0, 1, 3):
        E = spca.eigenimages(U, pl, k, range(pl.p[k]))
        if k == 0:
            q = np.arange(1, pl.p[0] + 1)
            ref = -2 * pl.c * math.sqrt(math.pi) * (((-1.0) ** q / pl.roots[0])[:, None] * U[0]).sum(axis=0)
            assert np.max(np.abs(E[:, i0, i0] - ref)) <= 1e-13 * np.max(np.abs(ref))
        else:
            assert np.all(E[:, i0, i0] == 0)


def test_continuous_across_a_root(pl32):
    """The guarded limit at z = R_{k,q} joins the plain quotient on either side."""
    pl = pl32
    U = _U(pl, 2)
    for k, q in [(0, 3), (2, 1), (6, 2)]:
        R = pl.roots[k][q - 1]
        u = U[k][:, 0]
        d = np.array([-1e-5, -1e-7, -1e-9, -1e-12, 0.0, 1e-12, 1e-9, 1e-7, 1e-5])
        v = spca.eigenimage_radial(pl, k, u, R + d)
        assert np.all(np.isfinite(v))
        slope = (v[-1] - v[0]) / 2e-5
        assert np.max(np.abs(v - (v[4] + slope * d))) <= 1e-8 * np.max(np.abs(v))
