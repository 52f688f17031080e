"""GPU parity of the CTF-filtered synthesis and of the estimation of R and c (Sec. VI-C)
against the FP64 oracle, through the C ABI.

Tolerances: filtered synthesis 1e-5 relative L2 (as the plain adjoint); per-pixel moments
1e-12 relative (FP64 sums of the same FP32 values, in another order); ring power 1e-5
relative per ring (the NUFFT's 1e-6 amplitude accuracy, doubled by the square, on
mean-subtracted images whose mean is the same float32 image on both sides); R and c from
the same moment and power arrays: equal (the device follows the stated arithmetic step by
step).  The end-to-end case checks that the estimates land on the synthesised support and
the CTF band edge."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import rel_l2
from oracle import estimate
from paper_1412_0781_amd import Plan, synth, workload

pytestmark = pytest.mark.gpu


def _sigma_for(syn, H, snr, n=256):
    """Noise standard deviation for a given SNR over the CTF-filtered clean images (their
    mean pixel power measured on n clean images of the workload)."""
    clean = workload.synthetic_images(syn, 0, n, seed=77, snr=1.0, ring_filter=H, sigma=0.0)
    return float((clean.double().pow(2).mean() / snr).sqrt())


def _coeffs(po, n, seed):
    k, q = po.kq[:, 0], po.kq[:, 1]
    return synth.random_coefficients(seed, np.arange(n), k, q)


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16.0), (64, 0.5, 32.0)])
def test_filtered_synthesis_matches_oracle(L, c, R):
    torch.cuda.set_device(0)
    print(f"[estimate] filtered synthesis L={L}", flush=True)
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    H32 = workload.ctf_ring_filter(plan)
    H = H32.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(H - estimate.ctf_envelope(po.xi))) <= 1e-7
    b = _coeffs(po, 5, 2)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    got = plan.adjoint(bt, ring_filter=H32).cpu().numpy()
    ref = oracle.adjoint(b, po, ring_filter=H)
    assert rel_l2(got, ref) <= 1e-5


def test_ctf_filter_parameters():
    """Eq.(CTFenv) through fb_ctf_filter with every parameter away from its default (so a
    swapped argument shows), against the oracle's envelope on the same rings."""
    torch.cuda.set_device(0)
    L, c, R = 128, 0.5, 64.0
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    args = dict(pixel_size=1.7, lam=0.025, z=1.8e4, a=0.07, B=60.0)
    got = plan.ctf_filter(args["pixel_size"], args["lam"], args["z"], args["a"], args["B"]).cpu().numpy()
    ref = estimate.ctf_envelope(po.xi, **args)
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))
    # the envelope reaches its cap of 1 on some rings and decays on the outer ones
    assert np.any(ref >= 0.99 * np.exp(-args["B"] * (po.xi / args["pixel_size"]) ** 2)) and ref[-1] < ref.max()


def test_pixel_moments():
    torch.cuda.set_device(0)
    plan = Plan(32, 0.5, 16.0)
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((300, 32, 32)) + 0.5).astype(np.float32)
    s, s2 = plan.pixel_moments(torch.tensor(x[:170], device="cuda"))
    s, s2 = plan.pixel_moments(torch.tensor(x[170:], device="cuda"), s, s2)
    rs, rs2 = estimate.pixel_moments(x)
    assert np.max(np.abs(s.cpu().numpy() - rs.ravel()) / np.abs(rs).max()) <= 1e-12
    assert np.max(np.abs(s2.cpu().numpy() - rs2.ravel()) / rs2.max()) <= 1e-12


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16.0), (64, 0.5, 32.0)])
def test_polar_power_matches_oracle(L, c, R):
    torch.cuda.set_device(0)
    print(f"[estimate] ring power L={L}", flush=True)
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    rng = np.random.default_rng(L)
    x = (rng.standard_normal((37, L, L)) + 0.3).astype(np.float32)
    xt = torch.tensor(x, device="cuda")
    s, _ = plan.pixel_moments(xt)
    p = plan.polar_power(xt, pixel_sum=s, count=37, batch=16).cpu().numpy()   # three passes, ragged
    mean32 = (s.cpu().numpy() / 37).astype(np.float32).reshape(L, L)
    ref = estimate.polar_power(x, po, mean_image=mean32)
    assert np.max(np.abs(p - ref) / ref) <= 1e-5
    p0 = plan.polar_power(xt).cpu().numpy()                                  # no mean removed
    ref0 = estimate.polar_power(x, po)
    assert np.max(np.abs(p0 - ref0) / ref0) <= 1e-5


def test_estimate_matches_oracle_on_the_same_arrays():
    torch.cuda.set_device(0)
    L, c, R = 64, 0.5, 32.0
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    syn = Plan(L, c, 22.0)
    n = 600
    H = workload.ctf_ring_filter(syn)
    sigma = _sigma_for(syn, H, 0.5)
    imgs = workload.synthetic_images(syn, 0, n, seed=5, snr=0.2, ring_filter=H, sigma=sigma)
    s, s2 = plan.pixel_moments(imgs)
    pw = plan.polar_power(imgs, pixel_sum=s, count=n)
    xi_dev = plan.host_tables()[2]
    for frac in (0.999, 0.9, 0.5):
        Rg, cg = plan.estimate_support(s, s2, n, pw, sigma * sigma, frac)
        Ro, co = estimate.estimate_support(s.cpu().numpy().reshape(L, L), s2.cpu().numpy().reshape(L, L), n,
                                           pw.cpu().numpy(), po, sigma * sigma, frac)
        # the same ring: the library's and the oracle's Gauss-Legendre nodes agree to rounding
        jg, jo = int(np.argmin(np.abs(xi_dev - cg))), int(np.argmin(np.abs(po.xi - co)))
        assert (Rg, jg) == (Ro, jo), (frac, Rg, cg, Ro, co)
        assert abs(cg - co) <= 1e-14


def test_estimate_end_to_end():
    """CTF-filtered images synthesised with support radius 22 (L = 64) and white noise at SNR
    1/2 (over the filtered clean power): the estimated R lies between the synthesis radius
    and L/2 (the CTF's suppression of low frequencies spreads each image over tens of
    pixels, and the 99.9 % radius follows that spread), and c at the CTF envelope's band
    edge (exp(-B f^2) is 0.02 near 0.2 cycles per pixel at 1 Angstrom per pixel)."""
    torch.cuda.set_device(0)
    print("[estimate] end to end", flush=True)
    L = 64
    plan = Plan(L, 0.5, L / 2)
    syn = Plan(L, 0.5, 22.0)
    n = 4000
    H = workload.ctf_ring_filter(syn)
    sigma = _sigma_for(syn, H, 0.5)
    imgs = workload.synthetic_images(syn, 0, n, seed=9, snr=0.2, ring_filter=H, sigma=sigma)
    s, s2 = plan.pixel_moments(imgs)
    pw = plan.polar_power(imgs, pixel_sum=s, count=n)
    R_est, c_est = plan.estimate_support(s, s2, n, pw, sigma * sigma, 0.999)
    print(f"  R = {R_est}, c = {c_est:.4f}", flush=True)
    assert 22 <= R_est <= 31
    assert 0.12 <= c_est <= 0.32


def test_estimate_arguments():
    torch.cuda.set_device(0)
    plan = Plan(32, 0.5, 16.0)
    z = torch.zeros(32 * 32, dtype=torch.float64, device="cuda")
    pw = torch.ones(plan.n_xi, dtype=torch.float64, device="cuda")
    from paper_1412_0781_amd import FBError
    with pytest.raises(FBError):
        plan.estimate_support(z, z, 0, pw, 1.0)
    with pytest.raises(FBError):
        plan.estimate_support(z, z, 10, pw, 1.0, frac=1.5)
