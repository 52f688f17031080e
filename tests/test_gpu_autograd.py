"""The differentiation workload on the GPU: forward expansion, a fixed Wiener-like
shrinkage of each coefficient, then the adjoint synthesis, as torch autograd
Functions; loss ||T(h . T* I) - I_clean||^2.  The gradient with respect to the
input images is checked against central finite differences (h = 1e-3):
along the gradient itself to 1e-4 relative, and along random directions to
1e-4 of their typical size ||grad|| ||d|| / sqrt(#pixels) (a random direction
can be nearly orthogonal to the gradient, and the FP32 rounding noise of the
loss does not shrink with it)."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import structured_images
from paper_1412_0781_amd import Plan, fb_expand, fb_synth, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _dev():
    torch.cuda.set_device(0)
    yield


def _workload(L, n, snr=1 / 20):
    po = oracle.plan(L, 0.5, L / 2)
    noisy = structured_images(po, n, seed=11, snr=snr)
    k, q = po.kq[:, 0], po.kq[:, 1]
    a = synth.random_coefficients(11, np.arange(n), k, q)
    clean = oracle.adjoint(a, po).astype(np.float32)
    v = synth.coef_variance(k, q)
    sigma2 = synth.noise_sigma2(k, q, L, snr)
    h = (v / (v + sigma2)).astype(np.float32)       # Wiener-like diagonal shrinkage, detached
    return noisy, clean, h


@pytest.mark.parametrize("L,n", [(64, 8), (128, 4)])
def test_gradient_matches_central_differences(L, n):
    print(f"[autograd] L={L} n={n}", flush=True)
    noisy, clean, h = _workload(L, n)
    plan = Plan(L, 0.5, L / 2)
    H = torch.tensor(h, device="cuda")[None, :, None]
    Ic = torch.tensor(clean, device="cuda")

    def loss(I):
        rec = fb_synth(fb_expand(I, plan) * H, plan)
        return ((rec.double() - Ic.double()) ** 2).sum()

    I = torch.tensor(noisy, device="cuda", requires_grad=True)
    f = loss(I)
    f.backward()
    grad = I.grad.double()
    rng = np.random.default_rng(5)
    step = 1e-3
    numel = noisy.size
    dirs = [(grad / grad.pow(2).mean().sqrt()).float()]
    dirs += [torch.tensor(rng.standard_normal(noisy.shape).astype(np.float32), device="cuda") for _ in range(3)]
    for t, d in enumerate(dirs):
        with torch.no_grad():
            fp = float(loss(I.detach() + step * d))
            fm = float(loss(I.detach() - step * d))
        fd = (fp - fm) / (2 * step)
        an = float((grad * d.double()).sum())
        scale = abs(an) if t == 0 else max(abs(an), float(grad.norm() * d.double().norm()) / np.sqrt(numel))
        print(f"  direction {t}: finite difference {fd:.8e} autograd {an:.8e} err/scale "
              f"{abs(fd - an) / scale:.2e}", flush=True)
        assert abs(fd - an) <= 1e-4 * scale


def test_gradient_at_full_size():
    # the differentiation configuration's shape: L = 128 and 64 images, the images and the
    # clean references generated on the device from the seed (no oracle is involved: both
    # sides of the check are the library's own gradient and loss)
    from paper_1412_0781_amd.workload import noise_sigma, synthetic_images
    L, n, seed, snr = 128, 64, 13, 1 / 20
    print(f"[autograd] L={L} n={n} (device inputs)", flush=True)
    plan = Plan(L, 0.5, L / 2)
    noisy = synthetic_images(plan, 0, n, seed, snr)
    a = synth.random_coefficients(seed, np.arange(n), plan.k.astype(np.int64), plan.q.astype(np.int64))
    at = torch.tensor(np.stack([a.real, a.imag], -1).astype(np.float32), device="cuda")
    Ic = plan.adjoint(at)
    v = synth.coef_variance(plan.k.astype(np.float64), plan.q.astype(np.float64))
    sigma2 = noise_sigma(plan, snr) ** 2
    H = torch.tensor((v / (v + sigma2)).astype(np.float32), device="cuda")[None, :, None]

    def loss(I):
        rec = fb_synth(fb_expand(I, plan) * H, plan)
        return ((rec.double() - Ic.double()) ** 2).sum()

    I = noisy.clone().requires_grad_(True)
    loss(I).backward()
    grad = I.grad.double()
    step = 1e-3
    gen = torch.Generator(device="cuda").manual_seed(7)
    dirs = [(grad / grad.pow(2).mean().sqrt()).float(),
            torch.randn(noisy.shape, generator=gen, device="cuda")]
    for t, d in enumerate(dirs):
        with torch.no_grad():
            fd = (float(loss(I.detach() + step * d)) - float(loss(I.detach() - step * d))) / (2 * step)
        an = float((grad * d.double()).sum())
        scale = abs(an) if t == 0 else max(abs(an), float(grad.norm() * d.double().norm()) / np.sqrt(noisy.numel()))
        print(f"  direction {t}: finite difference {fd:.8e} autograd {an:.8e} err/scale "
              f"{abs(fd - an) / scale:.2e}", flush=True)
        assert abs(fd - an) <= 1e-4 * scale
