"""Pins of the oracle's expansion T* (Algorithm 1): the paper's printed accuracy
example, an independent Bessel-series evaluation of the angular spectrum, and
the exact O(2) symmetries of Sec. III on the discrete grid."""

import math

import mpmath
import numpy as np
import pytest
from scipy import special

import oracle
from conftest import read_golden


def _golden_kv(name):
    out = {}
    for row in read_golden(name):
        k, v = row.split("=")
        out[k.strip()] = float(v)
    return out


def test_psi15_paper_accuracy_example():
    """Sec. II-B: F = psi_c^{1,5} at the polar nodes must give a_{1,5} = 1 and all
    other a_{k,q} = 0 with RMSE 1.2e-16 and max error 2.7e-15 (printed).  The basis
    function is evaluated here from mpmath's root and scipy's J_k, not the oracle's tables."""
    g = _golden_kv("paper_psi15_accuracy.txt")
    c, R, k0, q0 = g["c"], g["R"], int(g["k"]), int(g["q"])
    pl = oracle.plan(int(2 * R), c, R)
    root = float(mpmath.besseljzero(k0, q0))
    N = 1.0 / (c * math.sqrt(math.pi) * abs(special.jv(k0 + 1, root)))
    F = (N * special.jv(k0, root * pl.xi / c))[:, None] * np.exp(1j * k0 * pl.theta)[None, :]
    a = oracle.radial_quadrature(oracle.angular_dft(F[None], pl), pl)[0]
    target = np.zeros(pl.p_half, dtype=complex)
    target[pl.coef_off[k0] + q0 - 1] = 1.0
    err = np.abs(a - target)
    rmse = math.sqrt(np.mean(err ** 2))
    # the same order as printed; the bound leaves a decade for platform rounding
    assert rmse <= 10 * g["rmse"], rmse
    assert err.max() <= 10 * g["max_abs"], err.max()


def _angular_spectrum_bessel(image, pl, n_alias=4):
    """Fhat(xi_j, k) from the Jacobi-Anger expansion of each pixel's plane wave:
    (2pi/n) sum_l exp(-i z cos(theta_l - phi)) exp(-i k theta_l)
        = 2pi sum_p (-i)^m J_m(z) exp(-i m phi),  m = k + p n_theta,
    with z = 2 pi xi r.  A different route from Eq.(nufft) + Eq.(1DFFT)."""
    x = oracle.pixel_coords(pl.L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    r = np.hypot(X1, X2).ravel()
    phi = np.arctan2(X2, X1).ravel()
    I = image.ravel()
    out = np.zeros((pl.n_xi, pl.k_max + 1), dtype=complex)
    for k in range(pl.k_max + 1):
        for p in range(-n_alias, n_alias + 1):
            m = k + p * pl.n_theta
            z = 2 * math.pi * np.outer(pl.xi, r)                      # [n_xi, L*L]
            Jm = special.jv(abs(m), z) * (-1.0 if (m < 0 and abs(m) % 2) else 1.0)
            out[:, k] += 2 * math.pi * ((-1j) ** (m % 4)) * (Jm * np.exp(-1j * m * phi)[None, :]) @ I
    return out


@pytest.mark.parametrize("L,c,R", [(16, 0.5, 8), (15, 0.5, 7.5), (20, 1 / 3, 10)])
def test_angular_spectrum_against_bessel_series(L, c, R):
    pl = oracle.plan(L, c, R)
    rng = np.random.default_rng(1)
    img = rng.standard_normal((L, L))
    Fh = oracle.angular_dft(oracle.nudft_polar(img[None], pl), pl)[0]
    ref = _angular_spectrum_bessel(img, pl)
    assert np.max(np.abs(Fh - ref)) <= 1e-11 * np.max(np.abs(ref))


# --- exact symmetries (Sec. III, Eqs.(rot),(refl)) ---------------------------
def _index_of_neg(L):
    """array index of -i for each array index of i (None where -i is off the grid)."""
    x = oracle.pixel_coords(L).astype(int)
    pos = {int(v): a for a, v in enumerate(x)}
    return np.array([pos.get(-int(v), -1) for v in x])


def _symmetric_support(img):
    """Zero the row/column whose negative index falls off the grid (even L)."""
    L = img.shape[-1]
    neg = _index_of_neg(L)
    img = img.copy()
    img[..., neg < 0, :] = 0.0
    img[..., :, neg < 0] = 0.0
    return img


@pytest.mark.parametrize("L,c,R", [(16, 0.5, 8), (15, 0.5, 7.5), (24, 0.375, 12)])
def test_exact_o2_symmetries(L, c, R):
    pl = oracle.plan(L, c, R)
    assert pl.n_theta % 4 == 0
    rng = np.random.default_rng(2)
    I = _symmetric_support(rng.standard_normal((3, L, L)))
    neg = _index_of_neg(L)
    ok = neg >= 0
    a = oracle.expand(I, pl)
    k = pl.kq[:, 0]
    scale = np.max(np.abs(a))

    # counter-clockwise rotation by pi/2: I'(i1, i2) = I(i2, -i1)  ->  a e^{-ik pi/2}  (Eq.(rot))
    rot = np.zeros_like(I)
    for a1 in np.nonzero(ok)[0]:
        rot[:, a1, :] = I[:, :, neg[a1]]
    assert np.max(np.abs(oracle.expand(rot, pl) - a * (-1j) ** k)) <= 1e-13 * scale

    # reflection phi -> pi - phi: I'(i1, i2) = I(-i1, i2)  ->  a_{-k} = conj(a_k)  (Eq.(refl), alpha=0)
    ref = np.zeros_like(I)
    ref[:, ok, :] = I[:, neg[ok], :]
    assert np.max(np.abs(oracle.expand(ref, pl) - np.conj(a))) <= 1e-13 * scale

    # transpose = reflection with alpha = -pi/2  ->  i^k conj(a)
    tr = np.swapaxes(I, 1, 2)
    assert np.max(np.abs(oracle.expand(tr, pl) - (1j) ** k * np.conj(a))) <= 1e-13 * scale

    # rotation by pi: I'(i1, i2) = I(-i1, -i2)  ->  (-1)^k a
    r180 = np.zeros_like(I)
    r180[:, np.ix_(ok, ok)[0], np.ix_(ok, ok)[1]] = I[:, np.ix_(neg[ok], neg[ok])[0], np.ix_(neg[ok], neg[ok])[1]]
    assert np.max(np.abs(oracle.expand(r180, pl) - (-1.0) ** k * a)) <= 1e-13 * scale


def test_stages_agree_with_expand():
    pl = oracle.plan(16, 0.5, 8)
    I = np.random.default_rng(3).standard_normal((2, 16, 16))
    F, Fh, a = oracle.expand_stages(I, pl)
    assert F.shape == (2, pl.n_xi, pl.n_theta) and Fh.shape == (2, pl.n_xi, pl.k_max + 1)
    assert np.array_equal(a, oracle.expand(I, pl))
    # real images: F on the opposite ray is the conjugate (Sec. II-B)
    h = pl.n_theta // 2
    assert np.max(np.abs(F[:, :, h:] - np.conj(F[:, :, :h]))) <= 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("L", [15, 24])
def test_sparse_evaluation_matches_dense(L):
    # the sparse form drops only zero terms of the Eq.(nufft) double sum
    po = oracle.plan(L, 0.5, L / 2)
    rng = np.random.default_rng(7)
    dense = np.zeros((3, L, L))
    pix = []
    for i in range(3):
        flat = rng.choice(L * L, size=6, replace=False)
        r, c = flat // L, flat % L
        v = rng.standard_normal(6)
        dense[i, r, c] = v
        pix.append((r, c, v))
    F_dense = oracle.nudft_polar(dense, po)
    F_sparse = oracle.nudft_polar_sparse(pix, po)
    assert np.abs(F_sparse - F_dense).max() <= 1e-12 * np.abs(F_dense).max()
    a_dense = oracle.expand(dense, po)
    a_sparse = oracle.expand_sparse(pix, po)
    assert np.linalg.norm(a_sparse - a_dense) <= 1e-12 * np.linalg.norm(a_dense)


def test_pixel_combinations_match_dense_expansion():
    # images built from a pixel dictionary: the combination of the delta expansions equals the
    # dense evaluation of the same images (Algorithm 1 is linear in the image)
    L = 24
    po = oracle.plan(L, 0.5, L / 2)
    rng = np.random.default_rng(8)
    D, n = 10, 4
    flat = rng.choice(L * L, size=D, replace=False)
    rows, cols = flat // L, flat % L
    V = rng.standard_normal((n, D)) + 2.0
    dense = np.zeros((n, L, L))
    dense[:, rows, cols] = V
    a = oracle.expand_pixel_combinations(V, rows, cols, po)
    ref = oracle.expand(dense, po)
    assert np.linalg.norm(a - ref) <= 1e-12 * np.linalg.norm(ref)


def test_single_pixel_closed_form():
    # one unit pixel at (x0, y0): F(xi, theta) = exp(-2 pi i xi (x0 cos theta + y0 sin theta))
    L = 20
    po = oracle.plan(L, 0.5, 10)
    x = oracle.pixel_coords(L)
    r, c = 3, 14
    F = oracle.nudft_polar_sparse([(np.array([r]), np.array([c]), np.array([1.0]))], po)[0]
    xi1, xi2 = oracle.polar_nodes(po)
    for j, l in [(0, 0), (5, 17), (po.n_xi - 1, po.n_theta - 1)]:
        ph = -2 * mpmath.pi * (mpmath.mpf(xi1[j, l]) * x[r] + mpmath.mpf(xi2[j, l]) * x[c])
        want = complex(mpmath.cos(ph), mpmath.sin(ph))
        assert abs(F[j, l] - want) <= 1e-13


def test_brute_force_8x8_in_mpmath():
    # Algorithm 1 for an 8 x 8 image evaluated from scratch at 30 digits: Bessel roots,
    # normalisations, Gauss-Legendre nodes and weights, the polar Fourier sum, the angular
    # sum and the radial quadrature all in mpmath; only the (k, q) list comes from the oracle
    with mpmath.workdps(30):
        _brute_force_8x8()


def _brute_force_8x8():
    L, c, R = 8, 0.5, 4.0
    po = oracle.plan(L, c, R)
    rng = np.random.default_rng(8)
    img = rng.standard_normal((L, L))
    got = oracle.expand(img[None], po)[0]
    mc = mpmath.mpf(c)
    nxi, nth = po.n_xi, po.n_theta
    # Gauss-Legendre on [-1, 1] by Newton on P_n, then mapped to [0, c]
    nodes, weights = [], []
    for i in range(1, nxi + 1):
        x = mpmath.cos(mpmath.pi * (i - mpmath.mpf(1) / 4) / (nxi + mpmath.mpf(1) / 2))
        for _ in range(50):
            p0, p1 = mpmath.mpf(1), x
            for m in range(2, nxi + 1):
                p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
            dp = nxi * (x * p1 - p0) / (x * x - 1)
            dx = p1 / dp
            x -= dx
            if abs(dx) < mpmath.mpf(10) ** -28:
                break
        nodes.append(mc * (x + 1) / 2)
        weights.append(mc / ((1 - x * x) * dp * dp))
    pix = [mpmath.mpf(v) for v in oracle.pixel_coords(L)]
    F = {}
    for j in range(nxi):
        for l in range(nth):
            th = 2 * mpmath.pi * l / nth
            u1, u2 = nodes[j] * mpmath.cos(th), nodes[j] * mpmath.sin(th)
            F[j, l] = mpmath.fsum(img[a, b] * mpmath.expjpi(-2 * (u1 * pix[a] + u2 * pix[b]))
                                  for a in range(L) for b in range(L))
    want = np.zeros(po.p_half, complex)
    for idx, (k, q) in enumerate(po.kq):
        k, q = int(k), int(q)
        root = mpmath.besseljzero(k, q)
        norm = 1 / (mc * mpmath.sqrt(mpmath.pi) * abs(mpmath.besselj(k + 1, root)))
        s = mpmath.mpc(0)
        for j in range(nxi):
            fh = 2 * mpmath.pi / nth * mpmath.fsum(F[j, l] * mpmath.expjpi(-2 * mpmath.mpf(k * l) / nth)
                                                   for l in range(nth))
            s += norm * mpmath.besselj(k, root * nodes[j] / mc) * fh * nodes[j] * weights[j]
        want[idx] = complex(s)
    want[:po.p[0]] = want[:po.p[0]].real
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
