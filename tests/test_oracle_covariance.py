"""Pins of the oracle's steerable covariance and eigendecomposition (Sec. III,
Algorithm 2): brute-force averaging over all rotations and reflections
(Eqs.(mean1),(covfcovFB) from which Eq.(cov) is derived), the Marcenko-Pastur
noise band (Sec. V, Eq.(compselect)), and eigenpair properties."""

import numpy as np
import pytest

import oracle


def _full_vector(a, pl):
    """Coefficients over k = -kmax..kmax, q = 1..p_|k| with a_{-k,q} = conj(a_{k,q})."""
    blocks, ks = [], []
    for k in range(-pl.k_max, pl.k_max + 1):
        o = pl.coef_off[abs(k)]
        blk = a[:, o:o + pl.p[abs(k)]]
        blocks.append(blk if k >= 0 else np.conj(blk))
        ks += [k] * pl.p[abs(k)]
    return np.concatenate(blocks, axis=1), np.array(ks)


def test_covariance_equals_rotation_reflection_average():
    """Average over the O(2)-augmented data set, using alpha on a uniform grid of M > 2 k_max
    angles (exact for the trigonometric polynomials involved):
      rotation:    a_{k,q} -> a_{k,q} e^{-ik alpha}        (Eq.(rot))
      reflection:  a_{k,q} -> a_{-k,q} e^{-ik alpha}       (Eq.(refl)).
    The augmented mean must be the k = 0 mean only (Eq.(mean2)) and the augmented
    covariance must be block diagonal in k with blocks equal to C^(k) (Eq.(cov))."""
    pl = oracle.plan(12, 0.5, 6)
    n = 7
    rng = np.random.default_rng(7)
    I = rng.standard_normal((n, 12, 12)) + 0.3       # a non-zero mean
    a = oracle.expand(I, pl)
    full, ks = _full_vector(a, pl)                     # [n, Pfull]
    # entry (k, q) of the reflected vector holds a_{-k,q}
    refl = np.concatenate([full[:, ks == -k] for k in range(-pl.k_max, pl.k_max + 1)], axis=1)
    M = 2 * pl.k_max + 3
    copies = []
    for m in range(M):
        alpha = 2 * np.pi * m / M
        ph = np.exp(-1j * ks * alpha)[None, :]
        copies.append(full * ph)
        copies.append(refl * ph)
    aug = np.concatenate(copies, axis=0)               # [2 M n, Pfull]
    mean = aug.mean(axis=0)
    cen = aug - mean[None, :]
    Caug = cen.T @ cen.conj() / aug.shape[0]           # (1/N) sum a a^*

    mean0, C = oracle.mean_and_covariance(a, pl)
    # Eq.(mean2): only k = 0 survives, and equals the plain mean of a_{0,q}
    assert np.max(np.abs(mean[ks != 0])) < 1e-12 * np.abs(mean).max()
    assert np.max(np.abs(mean[ks == 0] - mean0)) < 1e-12 * np.abs(mean0).max()
    scale = np.abs(Caug).max()
    for k1 in range(-pl.k_max, pl.k_max + 1):
        for k2 in range(-pl.k_max, pl.k_max + 1):
            blk = Caug[np.ix_(ks == k1, ks == k2)]
            if k1 != k2:
                assert np.max(np.abs(blk)) < 1e-12 * scale, (k1, k2)
            else:
                assert np.max(np.abs(blk - C[abs(k1)])) < 1e-12 * scale, k1


def test_pure_noise_eigenvalues_in_marcenko_pastur_band():
    """Sec. V: for white noise of variance sigma^2 the eigenvalues of C^(k) spread over
    [sigma^2 (1 - sqrt(g))^2, sigma^2 (1 + sqrt(g))^2], g_0 = p_0/n, g_k = p_k/(2n)."""
    pl = oracle.plan(32, 0.5, 16)
    n = 2000
    sigma2 = 1.0
    I = np.random.default_rng(11).standard_normal((n, 32, 32))
    _, C = oracle.mean_and_covariance(oracle.expand(I, pl, chunk=250), pl)
    lam, _ = oracle.eig_blocks(C)
    inside = 0
    total = 0
    for k in range(pl.k_max + 1):
        g = pl.p[0] / n if k == 0 else pl.p[k] / (2 * n)
        lo = sigma2 * (1 - np.sqrt(g)) ** 2
        hi = sigma2 * (1 + np.sqrt(g)) ** 2
        # T*T is close to, not exactly, the identity (Sec. II-B): allow 10 %
        assert lam[k].max() < 1.10 * hi and lam[k].min() > 0.85 * lo, k
        inside += np.count_nonzero((lam[k] <= hi * 1.01) & (lam[k] >= lo * 0.99))
        total += lam[k].size
    assert inside / total > 0.9


def test_eig_blocks_properties():
    pl = oracle.plan(16, 0.5, 8)
    I = np.random.default_rng(12).standard_normal((200, 16, 16))
    _, C = oracle.mean_and_covariance(oracle.expand(I, pl), pl)
    lam, U = oracle.eig_blocks(C)
    for k, Ck in enumerate(C):
        assert np.allclose(Ck, Ck.T, atol=1e-15)
        assert np.all(np.diff(lam[k]) <= 0)
        assert np.allclose(Ck @ U[k], U[k] * lam[k][None, :], atol=1e-12 * np.abs(lam[k]).max())
        assert np.allclose(U[k].T @ U[k], np.eye(len(lam[k])), atol=1e-12)
        for col in range(U[k].shape[1]):
            i = int(np.argmax(np.abs(U[k][:, col])))
            assert U[k][i, col] > 0
        assert lam[k].min() > -1e-12               # positive semidefinite (Sec. III)


def test_hermitian_covariance_equals_rotation_average():
    """Average over the data augmented by rotations only (no reflections), alpha on a uniform
    grid of M > 2 k_max angles: the augmented covariance (1/N) sum v v^* is block diagonal
    in k and its (k, k) block is the oracle's Hermitian C_H^(k) (Sec. III, Eq.(cov) before
    the reflection average takes the real part); for k < 0 it is the conjugate."""
    pl = oracle.plan(12, 0.5, 6)
    n = 6
    rng = np.random.default_rng(21)
    I = rng.standard_normal((n, 12, 12)) + 0.2
    a = oracle.expand(I, pl)
    full, ks = _full_vector(a, pl)
    M = 2 * pl.k_max + 3
    aug = np.concatenate([full * np.exp(-1j * ks * (2 * np.pi * m / M))[None, :] for m in range(M)], axis=0)
    cen = aug - aug.mean(axis=0)[None, :]
    Caug = cen.T @ cen.conj() / aug.shape[0]
    mean0, CH = oracle.hermitian_covariance(a, pl)
    _, C = oracle.mean_and_covariance(a, pl)
    scale = np.abs(Caug).max()
    for k1 in range(-pl.k_max, pl.k_max + 1):
        for k2 in (k1 - 1, k1 + 1):
            if abs(k2) <= pl.k_max:
                assert np.max(np.abs(Caug[np.ix_(ks == k1, ks == k2)])) < 1e-12 * scale
        blk = Caug[np.ix_(ks == k1, ks == k1)]
        want = CH[abs(k1)] if k1 >= 0 else np.conj(CH[abs(k1)])
        assert np.max(np.abs(blk - want)) < 1e-12 * scale, k1
    # real part = the O(2) covariance; the imaginary part is antisymmetric and not zero
    for k in range(1, pl.k_max + 1):
        assert np.max(np.abs(CH[k].real - C[k])) < 1e-14 * scale
        assert np.max(np.abs(CH[k].imag + CH[k].imag.T)) < 1e-15 * scale
    assert max(np.abs(CH[k].imag).max() for k in range(1, pl.k_max + 1)) > 1e-3 * scale
