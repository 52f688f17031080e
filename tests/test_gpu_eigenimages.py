"""GPU parity of the real-space eigenimages (Sec. VI-B, Eq.(IFT_FB)) against the FP64
oracle, through the C ABI.  The eigenvectors are seeded random orthogonal blocks packed
like fb_eig's output, the same FP64 values on both sides.  Both sides are FP64 (the device
evaluates J_k by Miller's backward recurrence, the oracle calls scipy), so the bar is
1e-9 of the image's peak: rounding of the Bessel values, divided by z^2 - R^2 at pixels
close to a root, is the largest term."""

import numpy as np
import pytest
import torch

import oracle
from oracle import spca
from paper_1412_0781_amd import FBError, Plan

pytestmark = pytest.mark.gpu


def _random_orthogonal(p, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((p, p)))
    return q * np.sign(np.diag(r))[None, :]


def _setup(L, c, R, seed):
    torch.cuda.set_device(0)
    po = oracle.plan(L, c, R)
    U = [_random_orthogonal(po.p[k], seed + k) for k in range(po.k_max + 1)]
    plan = Plan(L, c, R)
    ev = torch.tensor(np.concatenate([u.ravel() for u in U]), device="cuda")
    return po, plan, U, ev


def _check(po, plan, U, ev, k, l0, nl):
    got = plan.eigenimages(ev, k, l0, nl).cpu().numpy()
    ref = spca.eigenimages(U, po, k, range(l0, l0 + nl))
    for i in range(nl):
        scale = np.max(np.abs(ref[i]))
        err = np.max(np.abs(got[i] - ref[i]))
        assert err <= 1e-9 * scale, (k, l0 + i, err, scale)


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16.0), (33, 0.5, 16.5), (64, 0.5, 32.0)])
def test_eigenimages_match_oracle(L, c, R):
    print(f"[eigenimages] L={L}", flush=True)
    po, plan, U, ev = _setup(L, c, R, 3)
    ks = sorted({0, 1, 2, 7, po.k_max})
    for k in ks:
        pk = po.p[k]
        _check(po, plan, U, ev, k, 0, pk)                       # every component of k
        if pk > 3:
            _check(po, plan, U, ev, k, 1, pk - 2)               # an inner range


def test_eigenimages_full_size():
    """L = 256: chunk boundaries of the component loop (16 per pass), high angular
    frequencies and the largest radii."""
    print("[eigenimages] L=256", flush=True)
    po, plan, U, ev = _setup(256, 0.5, 128.0, 9)
    _check(po, plan, U, ev, 0, 0, 3)
    _check(po, plan, U, ev, 3, 5, 20)
    _check(po, plan, U, ev, 150, 0, 2)
    _check(po, plan, U, ev, po.k_max, 0, po.p[po.k_max])


def test_eigenimages_arguments():
    po, plan, U, ev = _setup(32, 0.5, 16.0, 1)
    assert plan.eigenimages(ev, 2, 1, 0).shape == (0, 32, 32)
    for k, l0, nl in [(-1, 0, 1), (po.k_max + 1, 0, 1), (0, po.p[0], 1), (0, 0, po.p[0] + 1), (1, -1, 1)]:
        with pytest.raises((FBError, IndexError)):
            plan.eigenimages(ev, k, l0, nl)
