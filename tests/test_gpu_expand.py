"""GPU parity of the expansion a = T* I (Algorithm 1) against the FP64 oracle,
through the C ABI.  Tolerance: 1e-5 relative L2 over all coefficients, for both
the FP32 and the split-BF16x3 forms; k = 0 imaginary parts must be exactly 0."""

import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_util import as_complex, max_block_rel, noise_images, rel_l2, structured_images
from paper_1412_0781_amd import Plan

pytestmark = pytest.mark.gpu
TOL = 1e-5
# every angular-frequency block on its own (max over k of the block's relative L2 error)
BLOCK_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _dev():
    torch.cuda.set_device(0)
    yield


def _run(L, c, R, n, precision, seed=0, snr=0.1, batch=None):
    print(f"[expand] L={L} c={c} R={R} n={n} {precision} seed={seed}", flush=True)
    po = oracle.plan(L, c, R)
    img = structured_images(po, n, seed=seed, snr=snr)
    ref = oracle.expand(img.astype(np.float64), po)
    plan = Plan(L, c, R)
    x = torch.tensor(img, device="cuda")
    a = plan.expand(x, precision=precision, batch=batch)
    torch.cuda.synchronize()
    got = as_complex(a)
    return got, ref, plan, po


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("L,c,R,n", [
    (32, 0.5, 16, 64),     # workload shape of the FP64 reference case
    (31, 0.5, 15.5, 37),   # odd L, ragged image count
    (40, 0.5, 20, 5),      # grid 80 = 2^4 5, angular length 80
    (48, 0.5, 24, 3),      # grid 96 = 2^5 3
    (64, 0.3, 32, 4),      # c < 1/2, angular length 77 = 7 * 11 (generic radices)
    (24, 0.375, 12, 9),
    (16, 0.5, 8, 5),       # grid 32, angular length 32: the run-time-length streaming FFTs
])
def test_expand_matches_oracle(L, c, R, n, precision):
    got, ref, plan, po = _run(L, c, R, n, precision)
    err = rel_l2(got, ref)
    worst = max(rel_l2(got[i], ref[i]) for i in range(n))
    blk = max_block_rel(got, ref, po.coef_off)
    print(f"  rel-L2 {err:.3e}  worst image {worst:.3e}  worst k block {blk:.3e}", flush=True)
    assert err <= TOL and worst <= 2 * TOL and blk <= BLOCK_TOL
    assert np.all(got[:, :po.p[0]].imag == 0.0)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_expand_L128(precision):
    got, ref, _, po = _run(128, 0.5, 64, 6, precision, snr=0.05)
    err, blk = rel_l2(got, ref), max_block_rel(got, ref, po.coef_off)
    print(f"  rel-L2 {err:.3e}  worst k block {blk:.3e}", flush=True)
    assert err <= TOL and blk <= BLOCK_TOL


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_expand_L256(precision):
    got, ref, _, po = _run(256, 0.5, 128, 2, precision, snr=0.05)
    err, blk = rel_l2(got, ref), max_block_rel(got, ref, po.coef_off)
    print(f"  rel-L2 {err:.3e}  worst k block {blk:.3e}", flush=True)
    assert err <= TOL and blk <= BLOCK_TOL


def test_multi_pass_matches_single_pass():
    # a workspace for 16 images (one image group) forces passes of 16, 16, 8
    L = 32
    po = oracle.plan(L, 0.5, 16)
    img = torch.tensor(structured_images(po, 40, seed=3), device="cuda")
    plan = Plan(L, 0.5, 16)
    a1 = plan.expand(img, batch=16).clone()
    a2 = plan.expand(img, batch=64)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)


def test_bitwise_deterministic():
    L = 64
    plan = Plan(L, 0.5, 32)
    x = torch.tensor(noise_images(L, 40, seed=5), device="cuda")
    for prec in ["fp32", "bf16x3"]:
        a1 = plan.expand(x, precision=prec).clone()
        a2 = plan.expand(x, precision=prec)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2)


def _neg_index(L):
    x = oracle.pixel_coords(L).astype(int)
    pos = {int(v): i for i, v in enumerate(x)}
    return np.array([pos.get(-int(v), -1) for v in x])


def test_exact_symmetries_on_gpu():
    """rot90 -> (-i)^k a, reflection -> conj(a), transpose -> i^k conj(a) (Eqs.(rot),(refl))."""
    L = 64
    po = oracle.plan(L, 0.5, 32)
    img = structured_images(po, 4, seed=7)
    neg = _neg_index(L)
    ok = neg >= 0
    img[:, ~ok, :] = 0
    img[:, :, ~ok] = 0
    rot = np.zeros_like(img)
    for a1 in np.nonzero(ok)[0]:
        rot[:, a1, :] = img[:, :, neg[a1]]
    ref = np.zeros_like(img)
    ref[:, ok, :] = img[:, neg[ok], :]
    tr = np.ascontiguousarray(np.swapaxes(img, 1, 2))
    plan = Plan(L, 0.5, 32)
    k = plan.k
    run = lambda z: as_complex(plan.expand(torch.tensor(z, device="cuda")))
    a = run(img)
    assert rel_l2(run(rot), a * (-1j) ** k) <= 2 * TOL
    assert rel_l2(run(ref), np.conj(a)) <= 2 * TOL
    assert rel_l2(run(tr), (1j) ** k * np.conj(a)) <= 2 * TOL


def test_empty_and_bad_arguments():
    plan = Plan(32, 0.5, 16)
    out = plan.expand(torch.zeros((0, 32, 32), device="cuda"))
    assert out.shape == (0, plan.p_half, 2)
    with pytest.raises(ValueError):
        plan.expand(torch.zeros((2, 31, 32), device="cuda"))
    with pytest.raises(TypeError):
        plan.expand(torch.zeros((2, 32, 32), device="cuda", dtype=torch.float64))
    from paper_1412_0781_amd import _lib
    ws = plan.workspace(1)
    # workspace too small for one image
    rc = _lib.lib().fb_expand(plan._h, ws.data_ptr(), 1, ws.data_ptr(), 0, ws.data_ptr(), 16, None)
    assert rc == -6
