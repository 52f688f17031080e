"""fb_expand_noalloc (pass buffers in the library's fixed device array) against fb_expand
with a caller workspace, on two calls in a row, the second with fewer images, so that the
second reads an array that still holds the first call's data.  Both are the expansion of
Algorithm 1, steps 3-4; the kernels are shared, so the results agree to rounding."""

import numpy as np
import pytest
import torch

from paper_1412_0781_amd import Plan, synth

pytestmark = pytest.mark.gpu

# (L, first call, second call): at L = 256 the array holds 112 images per pass, so 300
# images take three passes (the last one ragged); at L = 64 it holds 1984, so 2500 take two.
CASES = [(256, 300, 50), (64, 2500, 7)]


def _rel(x, ref):
    x = x.double()
    ref = ref.double()
    per_image = ((x - ref).flatten(1).norm(dim=1) / ref.flatten(1).norm(dim=1)).max().item()
    return ((x - ref).norm() / ref.norm()).item(), per_image


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("L,n1,n2", CASES)
def test_noalloc_matches_workspace_expand(L, n1, n2, precision):
    print(f"noalloc L={L} n1={n1} n2={n2} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    plan = Plan(L, 0.5, L / 2)
    for n, seed in ((n1, 11), (n2, 12)):
        x = torch.tensor(synth.noise_images(seed, np.arange(n), L, 1.0), dtype=torch.float32, device=dev)
        ref = plan.expand(x, precision, batch=n)                   # one pass, caller workspace
        out = torch.full((n, plan.p_half, 2), float("nan"), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(dev)[0]
        plan.expand_noalloc(x, out, precision)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(dev)[0]
        if n == n2:
            # the array was loaded by the first call: the second takes no device memory
            assert free1 == free0, (free0, free1)
        assert torch.isfinite(out).all()
        err, worst = _rel(out, ref)
        print(f"  n={n}: rel-L2 {err:.2e}, worst image {worst:.2e}", flush=True)
        assert err <= 1e-6 and worst <= 1e-6, (err, worst)
    plan.close()


def test_noalloc_empty_and_arguments():
    dev = torch.device("cuda", 0)
    plan = Plan(64, 0.5, 32)
    x = torch.zeros((0, 64, 64), dtype=torch.float32, device=dev)
    out = torch.zeros((0, plan.p_half, 2), dtype=torch.float32, device=dev)
    plan.expand_noalloc(x, out)                          # n = 0: no-op
    from paper_1412_0781_amd import _lib
    lib = _lib.lib()
    assert lib.fb_expand_noalloc(plan._h, None, 4, None, 0, None) == -1
    lib.fb_profile_enable(plan._h, 1)
    x = torch.zeros((4, 64, 64), dtype=torch.float32, device=dev)
    out = torch.zeros((4, plan.p_half, 2), dtype=torch.float32, device=dev)
    assert lib.fb_expand_noalloc(plan._h, x.data_ptr(), 4, out.data_ptr(), 0, None) == -1   # timer on
    lib.fb_profile_enable(plan._h, 0)
    plan.close()
