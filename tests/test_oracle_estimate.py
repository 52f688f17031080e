"""Pins of the oracle's CTF-filtered synthesis and of its estimation of R and c (Sec. VI-C).

* The filtered synthesis of one basis function is checked against a 600-node
  Gauss-Legendre quadrature of its filtered inverse transform, reduced by the
  Jacobi-Anger expansion to a radial integral (a route that shares no step with the
  discrete transform), and a unit filter gives the plain synthesis.
* The ring power of a single-pixel image is exactly one per polar sample (|F| = 1).
* The support rule returns the edge of a step profile, for both R and c.
* The CTF filter takes its closed-form values."""

import math

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import estimate


@pytest.fixture(scope="module")
def pl32():
    return oracle.plan(32, 0.5, 16)


@pytest.mark.parametrize("k,q", [(0, 2), (1, 3), (4, 1)])
def test_filtered_synthesis_matches_quadrature(pl32, k, q):
    pl = pl32
    Bf = 20.0
    H = np.exp(-Bf * pl.xi ** 2)
    e = np.zeros((1, pl.p_half), dtype=complex)
    e[0, pl.coef_off[k] + q - 1] = 1.0
    img = oracle.adjoint(e, pl, ring_filter=H)[0]
    t, w = np.polynomial.legendre.leggauss(600)
    xi = pl.c * (t + 1) / 2
    wx = pl.c / 2 * w * xi * np.exp(-Bf * xi ** 2) * pl.norms[k][q - 1] * special.jv(k, pl.roots[k][q - 1] * xi / pl.c)
    x = oracle.pixel_coords(pl.L)
    rng = np.random.default_rng(0)
    pix = [(16, 16), (16, 20), (5, 27)] + [tuple(v) for v in rng.integers(2, 30, (8, 2))]
    scale = np.max(np.abs(img))
    for a, b in pix:
        r, phi = math.hypot(x[a], x[b]), math.atan2(x[b], x[a])
        f = 2 * math.pi * (1j) ** k * np.exp(1j * k * phi) * np.sum(wx * special.jv(k, 2 * math.pi * r * xi))
        ref = f.real if k == 0 else 2 * f.real
        assert abs(img[a, b] - ref) <= 1e-6 * scale, (a, b, img[a, b], ref)


def test_unit_filter_is_the_plain_synthesis(pl32):
    rng = np.random.default_rng(1)
    b = rng.standard_normal((2, pl32.p_half)) + 1j * rng.standard_normal((2, pl32.p_half))
    b[:, :pl32.p[0]] = b[:, :pl32.p[0]].real
    assert np.array_equal(oracle.adjoint(b, pl32, ring_filter=np.ones(pl32.n_xi)), oracle.adjoint(b, pl32))


def test_ring_power_of_single_pixels(pl32):
    pl = pl32
    L = pl.L
    imgs = np.zeros((3, L, L))
    imgs[0, 16, 16] = 1.0
    imgs[1, 3, 25] = 1.0
    imgs[2, 30, 1] = -1.0
    H = pl.n_theta // 2
    assert np.max(np.abs(estimate.polar_power(imgs, pl) - 3 * H)) <= 1e-10 * H
    same = np.repeat(imgs[:1], 2, axis=0)
    assert np.max(np.abs(estimate.polar_power(same, pl, mean_image=imgs[0]))) <= 1e-20
    pm = np.stack([imgs[0], -imgs[0]])
    assert np.max(np.abs(estimate.polar_power(pm, pl, mean_image=np.zeros((L, L))) - 2 * H)) <= 1e-10 * H


@pytest.mark.parametrize("r0,xi_cut", [(9, 0.21), (13, 0.33)])
def test_support_rule_on_step_profiles(pl32, r0, xi_cut):
    pl = pl32
    L, n, s2 = pl.L, 50, 4.0
    x = oracle.pixel_coords(L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    v = s2 + (np.rint(np.hypot(X1, X2)) <= r0)
    sum_img = np.zeros((L, L))
    sumsq_img = n * v
    ring = s2 + (pl.xi <= xi_cut)
    power = ring * n * (pl.n_theta // 2) * L * L
    R, c = estimate.estimate_support(sum_img, sumsq_img, n, power, pl, s2)
    assert R == r0
    assert c == pl.xi[pl.xi <= xi_cut].max()


def test_ctf_envelope_closed_form():
    lam, z, a, B = estimate.CTF_LAMBDA, estimate.CTF_DEFOCUS, estimate.CTF_PHASE, estimate.CTF_B
    assert estimate.ctf_envelope(0.0) == pytest.approx(a, rel=1e-15)
    f_sat = math.sqrt((1 - a) / (math.pi * lam * z))         # where pi lambda z f^2 + a reaches 1
    assert estimate.ctf_envelope(2 * f_sat) == pytest.approx(math.exp(-B * 4 * f_sat ** 2), rel=1e-14)
    assert estimate.ctf_envelope(0.5 * f_sat) == pytest.approx(
        (math.pi * lam * z * 0.25 * f_sat ** 2 + a) * math.exp(-B * 0.25 * f_sat ** 2), rel=1e-14)
    assert estimate.ctf_envelope(0.2, pixel_size=2.0) == pytest.approx(estimate.ctf_envelope(0.1), rel=1e-15)


def test_support_rule_uses_the_jacobians(pl32):
    """A flat excess over the noise with frac = 1/2: with the r dr weight the cumulative
    variance grows like r (r + 1), so half of it is reached at r = 12 of 16 (8 without the
    weight); with the xi dxi weight the cumulative power grows like xi^2, so half of it is
    reached at xi = c / sqrt(2) (c / 2 without)."""
    pl = pl32
    L, n, s2 = pl.L, 10, 1.0
    v = np.full((L, L), s2 + 1.0)
    power = (s2 + 1.0) * np.ones(pl.n_xi) * n * (pl.n_theta // 2) * L * L
    R, c = estimate.estimate_support(np.zeros((L, L)), n * v, n, power, pl, s2, frac=0.5)
    assert R == 12
    xi = pl.xi
    cum = np.cumsum(xi * pl.w)
    assert c == xi[np.argmax(cum >= 0.5 * cum[-1])]
    assert abs(c - pl.c / math.sqrt(2)) <= 0.03
