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
