"""Pins of the oracle's precomputation (Algorithm 1, steps 1-2) against facts
that do not come from the oracle: textbook Bessel zeros, an independent
high-precision root finder, brute-force sign counting, the paper's counting
bounds (Sec. II-A) and the orthonormality that defines N_{k,q} (Eq.(FB))."""

import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
from conftest import read_golden


def test_pixel_coords_definition():
    # Sec. II: i = -ceil((L-1)/2) .. floor((L-1)/2)
    assert oracle.pixel_coords(8).tolist() == [-4, -3, -2, -1, 0, 1, 2, 3]
    assert oracle.pixel_coords(7).tolist() == [-3, -2, -1, 0, 1, 2, 3]
    assert oracle.pixel_coords(2).tolist() == [-1, 0]


def test_roots_match_textbook_zeros():
    pl = oracle.plan(64, 0.5, 32)
    for row in read_golden("bessel_zeros_textbook.txt"):
        k, q, z = row.split()
        k, q, z = int(k), int(q), float(z)
        assert q <= pl.p[k]
        assert abs(pl.roots[k][q - 1] - z) <= 1e-13 * z, (k, q)


def test_roots_match_mpmath():
    # an independent arbitrary-precision root finder (mpmath.besseljzero)
    mpmath.mp.dps = 25
    pl = oracle.plan(32, 0.5, 16)
    for k in range(0, pl.k_max + 1, 3):
        for q in range(1, pl.p[k] + 1, 2):
            ref = float(mpmath.besseljzero(k, q))
            assert abs(pl.roots[k][q - 1] - ref) <= 4e-15 * ref, (k, q)


def _count_zeros_by_sign(k, bound, step=0.005):
    # zeros of J_k are simple and more than 2 apart: a fine grid sees each once
    x = np.append(np.arange(step, bound, step), bound)
    v = special.jv(k, x)
    return int(np.count_nonzero(np.signbit(v[1:]) != np.signbit(v[:-1]))) + int(v[-1] == 0.0)


@pytest.mark.parametrize("L,c,R", [(8, 0.5, 4), (16, 0.5, 8), (32, 0.5, 16), (40, 1 / 3, 20), (30, 0.25, 15)])
def test_pk_by_brute_force_sign_count(L, c, R):
    # Eq.(criterion1): q = 1..p_k admissible iff R_{k,q+1} <= 2 pi c R
    pl = oracle.plan(L, c, R)
    bound = 2 * math.pi * c * R
    for k in range(pl.k_max + 3):
        cnt = _count_zeros_by_sign(k, bound)
        expect = max(cnt - 1, 0)
        got = pl.p[k] if k <= pl.k_max else 0
        assert got == expect, (k, got, expect)


def test_small_case_counts():
    # hand count at L=8, R=4, c=1/2: 2 pi c R = 4 pi = 12.566; zeros of J_0 below it
    # are 2.405, 5.520, 8.654, 11.79 (4 of them) so p_0 = 3; J_5's first zero 8.77
    # and second 12.34 give p_5 = 1; J_6's second zero 13.59 > 4 pi gives p_6 = 0.
    pl = oracle.plan(8, 0.5, 4)
    assert pl.p[0] == 3 and pl.p[5] == 1 and pl.k_max == 5
    assert pl.n_xi == 8 and pl.n_theta == 32


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16), (64, 0.5, 32), (128, 0.5, 64), (121, 1 / 3, 60), (240, 0.196, 98)])
def test_paper_counting_bounds(L, c, R):
    """Sec. II-A: 8(cR)^2 <= p <= 4 pi (cR)^2, Eq.(kmaxbs) for k_max, Eq.(Rkq_lb)
    for every root with q >= 2, and p_k non-increasing in k."""
    pl = oracle.plan(L, c, R)
    cR = c * R
    assert 8 * cR ** 2 <= pl.p_total <= 4 * math.pi * cR ** 2
    assert 4 * cR - 3.517 < pl.k_max < 2 * math.pi * cR - 2.042
    assert all(pl.p[k + 1] <= pl.p[k] for k in range(pl.k_max))
    for k in range(pl.k_max + 1):
        for q in range(2, pl.p[k] + 1):
            # |a_{q-1}| > [3 pi/8 (4(q-1) - 1.4)]^{2/3}, so (2/3)|a|^{3/2} > (pi/4)(4(q-1) - 1.4)
            assert pl.roots[k][q - 1] > k + (math.pi / 4) * (4 * (q - 1) - 1.4)


def test_gauss_legendre_exactness():
    # Eq.(a) uses n_xi-point Gauss-Legendre on [0, c]: exact for degree < 2 n_xi
    pl = oracle.plan(16, 0.5, 8)
    for m in range(0, 2 * pl.n_xi):
        exact = pl.c ** (m + 1) / (m + 1)
        assert abs(np.sum(pl.w * pl.xi ** m) - exact) <= 1e-14 * pl.c ** (m + 1) * (m + 1) ** 0.5 + 1e-300
    assert np.all(np.diff(pl.xi) > 0) and pl.xi[0] > 0 and pl.xi[-1] < pl.c


def test_fb_basis_orthonormal_on_disk():
    """Eq.(FB): N_{k,q} makes psi_c^{k,q} unit-norm on the disk of radius c, and
    distinct q are orthogonal (Dirichlet eigenfunctions).  Integrated with mpmath."""
    mpmath.mp.dps = 20
    c, R = 0.5, 8
    pl = oracle.plan(16, c, R)
    for k, q1, q2 in [(0, 1, 1), (0, 3, 3), (2, 2, 2), (5, 1, 1), (1, 1, 3), (3, 2, 4)]:
        r1 = pl.roots[k][q1 - 1]
        r2 = pl.roots[k][q2 - 1]
        val = 2 * mpmath.pi * mpmath.quad(
            lambda t: mpmath.besselj(k, r1 * t / c) * mpmath.besselj(k, r2 * t / c) * t, [0, c])
        val = float(val) * pl.norms[k][q1 - 1] * pl.norms[k][q2 - 1]
        assert abs(val - (1.0 if q1 == q2 else 0.0)) < 1e-12, (k, q1, q2, val)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.plan(32, 0.6, 16)
    with pytest.raises(ValueError):
        oracle.plan(32, 0.0, 16)
    with pytest.raises(ValueError):
        oracle.plan(32, 0.5, 17)
    with pytest.raises(ValueError):
        oracle.plan(1, 0.5, 0.5)
    with pytest.raises(ValueError):
        oracle.plan(4, 0.5, 0.5)     # 2 pi c R = 1.57 < j_{0,2}: nothing admissible
