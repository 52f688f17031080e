"""GPU parity of the steerable-PCA back end (Algorithm 2 steps 5-6, Sec. V) against the
FP64 oracle, through the C ABI.  Inputs (coefficients, eigenpairs, mean) come from the
oracle, rounded to the library's storage precision, so each call is checked on its own.
Tolerances: selection counts exact and filter weights 1e-12 (FP64 arithmetic on the same
eigenvalues); projection, rebuild and radial functions 1e-6 relative L2 (FP32 products of
FP32-rounded inputs over at most p_k terms)."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import rel_l2, structured_images
from oracle import spca
from paper_1412_0781_amd import Plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[(32, 0.5, 16.0), (64, 0.5, 32.0)])
def case(request):
    torch.cuda.set_device(0)
    L, c, R = request.param
    print(f"[spca] L={L}", flush=True)
    po = oracle.plan(L, c, R)
    n = 600
    img = structured_images(po, n, seed=21, snr=0.2)
    a = oracle.expand(img.astype(np.float64), po)
    a32 = np.stack([a.real, a.imag], axis=-1).astype(np.float32)
    a = a32[..., 0].astype(np.float64) + 1j * a32[..., 1].astype(np.float64)
    mean0, C = oracle.mean_and_covariance(a, po)
    lam, U = oracle.eig_blocks(C)
    plan = Plan(L, c, R)
    packed_U = np.concatenate([u.ravel() for u in U])
    packed_lam = np.concatenate(lam)
    dev = dict(a=torch.tensor(a32, device="cuda"), U=torch.tensor(packed_U, device="cuda"),
               lam=torch.tensor(packed_lam, device="cuda"), mean=torch.tensor(mean0, device="cuda"))
    return po, plan, a, mean0, lam, U, dev, n


def _cplx(t):
    x = t.cpu().numpy().astype(np.float64)
    return x[..., 0] + 1j * x[..., 1]


def test_select_matches_oracle(case):
    po, plan, a, mean0, lam, U, dev, n = case
    for sigma2 in [0.5 * float(np.median(np.concatenate(lam))), float(np.median(np.concatenate(lam)))]:
        n_sel, w = plan.spca_select(dev["lam"], n, sigma2)
        cnt = spca.select(lam, po, n, sigma2)
        wref = np.concatenate(spca.filter_weights(lam, po, n, sigma2))
        assert np.array_equal(n_sel.cpu().numpy(), cnt)
        assert np.abs(w.cpu().numpy() - wref).max() <= 1e-12


def test_coeffs_and_reconstruct_match_oracle(case):
    po, plan, a, mean0, lam, U, dev, n = case
    c = plan.spca_coeffs(dev["a"], dev["U"], dev["mean"])
    cref = spca.coefficients(a, mean0, U, po)
    assert rel_l2(_cplx(c), cref) <= 1e-6
    assert np.all(c[:, :po.p[0], 1].cpu().numpy() == 0.0)
    # rebuild without filter inverts the projection; with the selection filter it matches the oracle
    back = plan.spca_reconstruct(c, dev["U"], dev["mean"])
    assert rel_l2(_cplx(back), a) <= 2e-6
    sigma2 = float(np.median(np.concatenate(lam)))
    _, w = plan.spca_select(dev["lam"], n, sigma2)
    den = plan.spca_reconstruct(c, dev["U"], dev["mean"], w)
    c32 = _cplx(c)
    dref = spca.reconstruct(c32, mean0, U, spca.filter_weights(lam, po, n, sigma2), po)
    assert rel_l2(_cplx(den), dref) <= 1e-6


def test_radial_functions_match_oracle(case):
    po, plan, a, mean0, lam, U, dev, n = case
    f = plan.spca_radial(dev["U"]).cpu().numpy().astype(np.float64)
    fref = spca.radial_functions(U, po)
    got = plan.radial_blocks(f)
    num = sum(np.linalg.norm(got[k] - fref[k]) ** 2 for k in range(po.k_max + 1))
    den = sum(np.linalg.norm(fref[k]) ** 2 for k in range(po.k_max + 1))
    assert np.sqrt(num / den) <= 1e-6


def test_denoising_reduces_error():
    # end to end on the device: expand, covariance, eig, select with the known noise
    # variance, filter and rebuild, synthesise; the result is closer to the clean images
    torch.cuda.set_device(0)
    from paper_1412_0781_amd import synth
    L, c, R, n, seed, snr = 64, 0.5, 32.0, 3000, 4, 0.1
    plan = Plan(L, c, R)
    po = oracle.plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    idx = np.arange(n)
    a_true = synth.random_coefficients(seed, idx, k, q)
    at = torch.tensor(np.stack([a_true.real, a_true.imag], -1).astype(np.float32), device="cuda")
    clean = plan.adjoint(at)
    sigma2 = synth.noise_sigma2(k, q, L, snr)
    noisy = clean + torch.tensor(synth.noise_images(seed, idx, L, np.sqrt(sigma2)).astype(np.float32),
                                 device="cuda")
    a = plan.expand(noisy)
    st = plan.covariance(a)
    evals, evecs, Cb, mean = plan.eig(st)
    _, w = plan.spca_select(evals, n, sigma2)
    den = plan.adjoint(plan.spca_reconstruct(plan.spca_coeffs(a, evecs, mean), evecs, mean, w))
    torch.cuda.synchronize()
    e_noisy = float(((noisy - clean) ** 2).mean())
    e_den = float(((den - clean) ** 2).mean())
    print(f"  mse noisy {e_noisy:.4g}  denoised {e_den:.4g}", flush=True)
    assert e_den < 0.5 * e_noisy


def test_coeffs_and_reconstruct_large_blocks():
    """L = 456: blocks of up to 227 coefficients, more than the products keep resident in LDS,
    so their U operand is read by chunks; 300 images (a ragged last run of image blocks).
    Random coefficients, mean and orthogonal U (QR of Gaussian blocks) and weights in [0, 1],
    against the oracle's projection and rebuild."""
    torch.cuda.set_device(0)
    L, c, R, n = 456, 0.5, 228.0, 300
    print(f"[spca] L={L} large blocks", flush=True)
    po = oracle.plan(L, c, R)
    assert max(po.p) > 224
    rng = np.random.default_rng(7)
    a = rng.standard_normal((n, po.p_half)) + 1j * rng.standard_normal((n, po.p_half))
    a[:, :po.p[0]] = a[:, :po.p[0]].real
    a32 = np.stack([a.real, a.imag], axis=-1).astype(np.float32)
    a = a32[..., 0].astype(np.float64) + 1j * a32[..., 1].astype(np.float64)
    mean0 = rng.standard_normal(po.p[0])
    U = [np.linalg.qr(rng.standard_normal((pk, pk)))[0] for pk in po.p]
    w = [rng.uniform(0.0, 1.0, pk) for pk in po.p]
    plan = Plan(L, c, R)
    dU = torch.tensor(np.concatenate([u.ravel() for u in U]), device="cuda")
    dm = torch.tensor(mean0, device="cuda")
    cg = plan.spca_coeffs(torch.tensor(a32, device="cuda"), dU, dm)
    assert rel_l2(_cplx(cg), spca.coefficients(a, mean0, U, po)) <= 1e-6
    c32 = _cplx(cg)
    back = plan.spca_reconstruct(cg, dU, dm, torch.tensor(np.concatenate(w), device="cuda"))
    assert rel_l2(_cplx(back), spca.reconstruct(c32, mean0, U, w, po)) <= 1e-6
