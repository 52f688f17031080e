"""Pins of the oracle's SVD route to the principal components (Sec. III-C: the left
singular vectors of A^(k) instead of the eigenvectors of C^(k)).

* A coefficient matrix built from prescribed singular values and vectors (values spread
  over ten decades) gives those values back, to the relative accuracy the SVD promises,
  where the covariance route has already lost the small ones.
* On ordinary data both routes agree (the covariance route is pinned on its own).
* The eigenvalues sum to the data's energy per image, with the mean removed from k = 0."""

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def pl():
    return oracle.plan(32, 0.5, 16)


def _orth(m, p, rng):
    q, r = np.linalg.qr(rng.standard_normal((m, p)))
    return q * np.sign(np.diag(r))[None, :]


def test_prescribed_singular_values(pl):
    rng = np.random.default_rng(0)
    n, k = 400, 1
    p = pl.p[k]
    sig = np.logspace(0, -10, p)
    V = _orth(p, p, rng)
    X = _orth(2 * n, p, rng) @ np.diag(sig) @ V.T              # rows: Re parts, then Im parts
    a = rng.standard_normal((n, pl.p_half)) + 1j * rng.standard_normal((n, pl.p_half))
    a[:, :pl.p[0]] = a[:, :pl.p[0]].real
    o = pl.coef_off[k]
    a[:, o:o + p] = X[:n] + 1j * X[n:]
    _, lam, U = oracle.svd_blocks(a, pl)
    assert np.max(np.abs(lam[k] * n / sig ** 2 - 1)) <= 1e-4
    Vs = V * np.sign(V[np.argmax(np.abs(V), axis=0), np.arange(p)])[None, :]
    assert np.max(np.abs(U[k] - Vs)) <= 1e-5
    # the covariance route squares the condition number: its smallest eigenvalues are noise
    _, C = oracle.mean_and_covariance(a, pl)
    lam_c, _ = oracle.eig_blocks(C)
    assert np.max(np.abs(lam_c[k][-3:] * n / sig[-3:] ** 2 - 1)) > 1e-2


def test_agrees_with_covariance_route(pl):
    rng = np.random.default_rng(1)
    n = 500
    a = rng.standard_normal((n, pl.p_half)) * np.linspace(2, 0.5, pl.p_half)[None, :] \
        + 1j * rng.standard_normal((n, pl.p_half))
    a[:, :pl.p[0]] = a[:, :pl.p[0]].real + 3.0                  # a mean to remove
    m_s, lam_s, U_s = oracle.svd_blocks(a, pl)
    m_c, C = oracle.mean_and_covariance(a, pl)
    lam_c, U_c = oracle.eig_blocks(C)
    assert np.max(np.abs(m_s - m_c)) <= 1e-14
    for k in range(pl.k_max + 1):
        assert np.max(np.abs(lam_s[k] - lam_c[k])) <= 1e-12 * lam_c[k][0]
        gaps = np.abs(np.diff(lam_c[k])) / lam_c[k][0]
        for l in range(pl.p[k]):
            lo = gaps[l - 1] if l > 0 else 1.0
            hi = gaps[l] if l < pl.p[k] - 1 else 1.0
            if min(lo, hi) > 1e-3:
                assert np.max(np.abs(U_s[k][:, l] - U_c[k][:, l])) <= 1e-8


def test_energy(pl):
    rng = np.random.default_rng(2)
    n = 300
    a = rng.standard_normal((n, pl.p_half)) + 1j * rng.standard_normal((n, pl.p_half))
    a[:, :pl.p[0]] = a[:, :pl.p[0]].real + 1.5
    _, lam, _ = oracle.svd_blocks(a, pl)
    for k in range(pl.k_max + 1):
        blk = a[:, pl.coef_off[k]:pl.coef_off[k] + pl.p[k]]
        if k == 0:
            e = np.sum((blk.real - blk.real.mean(axis=0)) ** 2) / n
        else:
            e = np.sum(np.abs(blk) ** 2) / n
        assert abs(np.sum(lam[k]) - e) <= 1e-12 * e
