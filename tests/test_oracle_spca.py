"""Pins of the steerable-PCA back end of the oracle (Algorithm 2 steps 5-6, Sec. V)."""

import math

import numpy as np
import pytest

import oracle
from oracle import spca


@pytest.fixture(scope="module")
def setup():
    L = 24
    po = oracle.plan(L, 0.5, 12)
    rng = np.random.default_rng(3)
    n = 400
    # coefficients with a few strong directions per k on top of white noise
    a = (rng.standard_normal((n, po.p_half)) + 1j * rng.standard_normal((n, po.p_half))) / math.sqrt(2)
    a[:, :po.p[0]] = rng.standard_normal((n, po.p[0]))
    mean0, C = oracle.mean_and_covariance(a, po)
    lam, U = oracle.eig_blocks(C)
    return po, a, mean0, lam, U


def test_radial_functions_orthonormal(setup):
    # psi^{k,q} are orthonormal on the disk of radius c (Eq.(FB)) and u^(k) is orthogonal,
    # so 2 pi int_0^c f^{k,l} f^{k,l'} xi dxi = delta_{l l'}: 400-point Gauss-Legendre on [0, c]
    po, a, mean0, lam, U = setup
    x, wq = np.polynomial.legendre.leggauss(400)
    xi, w = (x + 1) * po.c / 2, wq * po.c / 2
    f = spca.radial_functions(U, po, xi)
    for k in [0, 1, 3, po.k_max]:
        G = 2 * math.pi * (f[k] * (xi * w)[:, None]).T @ f[k]
        assert np.abs(G - np.eye(po.p[k])).max() <= 1e-11
    # at the plan's nodes the same definition is evaluated
    fn = spca.radial_functions(U, po)
    fi = spca.radial_functions(U, po, po.xi)
    assert np.array_equal(fn[2], fi[2])


def test_coefficients_preserve_energy_and_invert(setup):
    po, a, mean0, lam, U = setup
    c = spca.coefficients(a, mean0, U, po)
    a0 = a.copy()
    a0[:, :po.p[0]] -= mean0
    # U^(k) orthogonal: the per-image energy in each k block is unchanged
    for k in range(po.k_max + 1):
        o = po.coef_off[k]
        assert np.allclose(np.sum(np.abs(c[:, o:o + po.p[k]]) ** 2, axis=1),
                           np.sum(np.abs(a0[:, o:o + po.p[k]]) ** 2, axis=1), rtol=1e-12)
    assert np.allclose(spca.reconstruct(c, mean0, U, None, po), a, atol=1e-12)
    # the variance of c_{k,l} over images is lambda_l^(k) (C^(k) = U diag(lambda) U^T)
    for k in [0, 2]:
        o = po.coef_off[k]
        var = np.mean(np.abs(c[:, o:o + po.p[k]]) ** 2, axis=0)
        assert np.allclose(var, lam[k], rtol=1e-10)


def test_selection_on_a_spiked_model():
    # white noise of variance s2 plus r strong directions per k: exactly r components
    # per k lie above the Marcenko-Pastur edge (Eq.(compselect))
    po = oracle.plan(20, 0.5, 10)
    rng = np.random.default_rng(5)
    n, s2, r = 4000, 0.7, 2
    a = np.sqrt(s2 / 2) * (rng.standard_normal((n, po.p_half)) + 1j * rng.standard_normal((n, po.p_half)))
    a[:, :po.p[0]] = np.sqrt(s2) * rng.standard_normal((n, po.p[0]))
    spikes = [10.0, 4.0]
    truth = []
    for k in range(po.k_max + 1):
        o, pk = po.coef_off[k], po.p[k]
        V, _ = np.linalg.qr(rng.standard_normal((pk, pk)))
        for s in range(min(r, pk)):
            g = rng.standard_normal(n) if k == 0 else (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)
            a[:, o:o + pk] += np.sqrt(spikes[s]) * g[:, None] * V[:, s][None, :]
        truth.append(min(r, pk))
    mean0, C = oracle.mean_and_covariance(a, po)
    lam, U = oracle.eig_blocks(C)
    cnt = spca.select(lam, po, n, s2)
    assert np.array_equal(cnt, np.array(truth))
    # to first order the shrunk eigenvalue is the spike's signal variance
    for k in [1, 2]:
        assert abs(spca.shrink(lam[k][0], s2) - spikes[0]) <= 0.1 * spikes[0]
    # filter weights: ell / (ell + s2) on the selected components, 0 elsewhere
    w = spca.filter_weights(lam, po, n, s2)
    for k in range(po.k_max + 1):
        assert np.all(w[k][cnt[k]:] == 0) and np.all((w[k][:cnt[k]] > 0) & (w[k][:cnt[k]] < 1))


def test_mp_edges():
    po = oracle.plan(20, 0.5, 10)
    g = spca.mp_ratio(po, 1000)
    assert g[0] == po.p[0] / 1000 and g[1] == po.p[1] / 2000
    e = spca.mp_upper_edge(po, 1000, 2.0)
    assert np.allclose(e, 2.0 * (1 + np.sqrt(g)) ** 2)


def _spiked(po, n, s2, spikes, seed):
    """White noise of variance s2 plus len(spikes) directions per k with the given signal
    variances; returns the coefficients and the number of spikes per k."""
    rng = np.random.default_rng(seed)
    a = np.sqrt(s2 / 2) * (rng.standard_normal((n, po.p_half)) + 1j * rng.standard_normal((n, po.p_half)))
    a[:, :po.p[0]] = np.sqrt(s2) * rng.standard_normal((n, po.p[0]))
    truth = []
    for k in range(po.k_max + 1):
        o, pk = po.coef_off[k], po.p[k]
        V, _ = np.linalg.qr(rng.standard_normal((pk, pk)))
        for s in range(min(len(spikes), pk)):
            g = rng.standard_normal(n) if k == 0 else (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2)
            a[:, o:o + pk] += np.sqrt(spikes[s]) * g[:, None] * V[:, s][None, :]
        truth.append(min(len(spikes), pk))
    return a, truth


def test_filter_weights_match_the_spike_signal_to_noise():
    # Sec. V: for a spike of signal variance s in noise s2 the shrunk eigenvalue estimates s,
    # so the coefficient filter of a selected component is s / (s + s2) (its complement
    # s2 / (s + s2) is what a swapped numerator would give)
    po = oracle.plan(20, 0.5, 10)
    n, s2, spikes = 20000, 0.7, [10.0, 4.0]
    a, truth = _spiked(po, n, s2, spikes, seed=11)
    mean0, C = oracle.mean_and_covariance(a, po)
    lam, U = oracle.eig_blocks(C)
    w = spca.filter_weights(lam, po, n, s2)
    for k in range(po.k_max + 1):
        for s in range(truth[k]):
            expect = spikes[s] / (spikes[s] + s2)
            assert abs(w[k][s] - expect) <= 0.01, (k, s, w[k][s], expect)


def test_mp_edge_matches_pure_noise_spectra():
    # Sec. V: the top noise eigenvalue of C^(k) sits at the Marcenko-Pastur edge
    # s2 (1 + sqrt(gamma_k))^2 with gamma_0 = p_0 / n (n real samples) and gamma_k = p_k / (2n)
    # for k > 0 (Re and Im give 2n real samples); the ratios are chosen large (0.16 .. 0.3) so
    # that the edges of p_k / (2n) and p_k / n differ by about 20 %
    po = oracle.plan(64, 0.5, 32)
    n, s2 = 52, 1.3
    rng = np.random.default_rng(17)
    ratios0, ratios = [], []
    for rep in range(6):
        a = np.sqrt(s2 / 2) * (rng.standard_normal((n, po.p_half)) + 1j * rng.standard_normal((n, po.p_half)))
        a[:, :po.p[0]] = np.sqrt(s2) * rng.standard_normal((n, po.p[0]))
        mean0, C = oracle.mean_and_covariance(a, po)
        lam, U = oracle.eig_blocks(C)
        edge = spca.mp_upper_edge(po, n, s2)
        g = spca.mp_ratio(po, n)
        ratios0.append(lam[0][0] / edge[0])
        for k in range(1, 12):
            assert 0.15 <= g[k] <= 0.35
            ratios.append(lam[k][0] / edge[k])
    # at these sizes the top eigenvalue sits a few % below the asymptotic edge (the mean of
    # the Tracy-Widom fluctuation is negative); gamma_k = p_k / n for k > 0 would put the ratio
    # near 0.72, and gamma_0 = p_0 / (2n) would put the k = 0 ratio near 1.19
    assert 0.88 <= np.median(ratios) <= 1.02, np.median(ratios)
    assert 0.84 <= np.median(ratios0) <= 1.02, np.median(ratios0)
    # nothing is selected from pure noise in most blocks
    assert np.mean(spca.select(lam, po, n, s2)[1:12] == 0) >= 0.5


def test_weighted_reconstruct_one_hot_is_a_projection(setup):
    # with w = e_{k,l} the filtered reconstruction is the projection of the centred block k
    # onto u_l^(k) (plus the mean for k = 0), and every other block is zero
    po, a, mean0, lam, U = setup
    c = spca.coefficients(a, mean0, U, po)
    a0 = a.copy()
    a0[:, :po.p[0]] -= mean0
    for k, l in [(0, 1), (2, 0), (po.k_max, po.p[po.k_max] - 1)]:
        w = [np.zeros(po.p[kk]) for kk in range(po.k_max + 1)]
        w[k][l] = 1.0
        r = spca.reconstruct(c, mean0, U, w, po)
        o, pk = po.coef_off[k], po.p[k]
        u = U[k][:, l]
        proj = (a0[:, o:o + pk] @ u)[:, None] * u[None, :]
        expect = np.zeros_like(r)
        expect[:, o:o + pk] = proj
        expect[:, :po.p[0]] += mean0
        assert np.abs(r - expect).max() <= 1e-12
        # and a weight of 1/2 halves it
        w[k][l] = 0.5
        r2 = spca.reconstruct(c, mean0, U, w, po)
        assert np.abs(r2[:, o:o + pk] - (0.5 * proj + (mean0 if k == 0 else 0))).max() <= 1e-12
