"""GPU parity of the SVD route to the principal components (Sec. III-C) against the FP64
oracle (LAPACK's SVD of the same matrices), through the C ABI.

Inputs are float32 coefficient arrays (the library's input format), read by both sides as
the same FP64 values.  Tolerances: eigenvalues 1e-10 of each block's largest (FP64
Householder QR and Jacobi rotations are backward stable at a few ulps of the largest
singular value); eigenvectors 1e-8 where the relative gap to their neighbours exceeds
1e-3; the mean 1e-12.  The ill-conditioned case compares every eigenvalue to its own size,
which the covariance route cannot do.  Sizes span several level-1 row ranges per k
(8192 rows each) and a ragged last range, and blocks of up to 179 coefficients (L = 360)."""

import numpy as np
import pytest
import torch

import oracle
from paper_1412_0781_amd import FBError, Plan

pytestmark = pytest.mark.gpu


def _coeffs(po, n, seed, mean=2.0):
    rng = np.random.default_rng(seed)
    scale = 1.0 / (1.0 + np.arange(po.p_half)) ** 0.5
    a = np.stack([rng.standard_normal((n, po.p_half)) * scale, rng.standard_normal((n, po.p_half)) * scale], axis=-1)
    a[:, :po.p[0], 0] += mean
    a[:, :po.p[0], 1] = 0.0
    return a.astype(np.float32)


def _compare(po, plan, a32, lam_tol=1e-10, vec_tol=1e-8, relative_each=False):
    n = a32.shape[0]
    ev, U, m = plan.svd(torch.tensor(a32, device="cuda"))
    ev, U, m = ev.cpu().numpy(), U.cpu().numpy(), m.cpu().numpy()
    a = a32[..., 0].astype(np.float64) + 1j * a32[..., 1].astype(np.float64)
    m_ref, lam_ref, U_ref = oracle.svd_blocks(a, po)
    assert np.max(np.abs(m - m_ref)) <= 1e-12 * max(1.0, np.max(np.abs(m_ref)))
    for k in range(po.k_max + 1):
        o, p = po.coef_off[k], po.p[k]
        lam = ev[o:o + p]
        ref = lam_ref[k]
        if relative_each:
            assert np.max(np.abs(lam / ref - 1)) <= lam_tol, (k, lam, ref)
        else:
            assert np.max(np.abs(lam - ref)) <= lam_tol * ref[0], (k, np.max(np.abs(lam - ref)), ref[0])
        Ug = U[plan.cov_off[k]:plan.cov_off[k] + p * p].reshape(p, p)
        gaps = np.abs(np.diff(ref)) / ref[0]
        for l in range(p):
            lo = gaps[l - 1] if l > 0 else 1.0
            hi = gaps[l] if l < p - 1 else 1.0
            if min(lo, hi) > 1e-3:
                assert np.max(np.abs(Ug[:, l] - U_ref[k][:, l])) <= vec_tol, (k, l)


@pytest.mark.parametrize("L,c,R,n", [(32, 0.5, 16.0, 6000), (33, 0.5, 16.5, 900), (64, 0.5, 32.0, 9001)])
def test_svd_matches_oracle(L, c, R, n):
    torch.cuda.set_device(0)
    print(f"[svd] L={L} n={n}", flush=True)
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    _compare(po, plan, _coeffs(po, n, seed=L + n))


def test_svd_small_singular_values():
    """A k = 2 block with singular values over eight decades: every eigenvalue to 1e-6 of
    itself, far below what an eigendecomposition of C^(k) can resolve."""
    torch.cuda.set_device(0)
    print("[svd] ill-conditioned block", flush=True)
    L, c, R, n = 32, 0.5, 16.0, 5000
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    a32 = _coeffs(po, n, seed=4)
    rng = np.random.default_rng(5)
    k = 2
    p = po.p[k]
    q1, _ = np.linalg.qr(rng.standard_normal((2 * n, p)))
    q2, _ = np.linalg.qr(rng.standard_normal((p, p)))
    X = (q1 * np.logspace(1, -7, p)[None, :]) @ q2.T
    o = po.coef_off[k]
    a32[:, o:o + p, 0] = X[:n]
    a32[:, o:o + p, 1] = X[n:]
    ev, _, _ = plan.svd(torch.tensor(a32, device="cuda"))
    a = a32[..., 0].astype(np.float64) + 1j * a32[..., 1].astype(np.float64)
    _, lam_ref, _ = oracle.svd_blocks(a, po)
    lam = ev.cpu().numpy()[o:o + p]
    assert lam_ref[k][-1] < 1e-12 * lam_ref[k][0]
    assert np.max(np.abs(lam / lam_ref[k] - 1)) <= 1e-6


def test_svd_full_size():
    """L = 256 (p_k up to 127) with two level-1 ranges for k = 0 and three for k > 0."""
    torch.cuda.set_device(0)
    print("[svd] L=256", flush=True)
    L, c, R, n = 256, 0.5, 128.0, 10000
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    _compare(po, plan, _coeffs(po, n, seed=7))


@pytest.mark.parametrize("L,n", [(276, 1500), (360, 2000)])
def test_svd_blocks_above_128(L, n):
    """Blocks of more than 128 coefficients: two threads per column in 512-thread workgroups;
    at L = 276 (p_0 = 137) the p_k x p_k rotations still run in LDS, at L = 360 (p_0 = 179)
    the blocks above 141 are rotated in global memory."""
    torch.cuda.set_device(0)
    print(f"[svd] L={L} n={n}", flush=True)
    c, R = 0.5, L / 2
    po = oracle.plan(L, c, R)
    plan = Plan(L, c, R)
    assert max(po.p) > 128
    _compare(po, plan, _coeffs(po, n, seed=L))


def test_svd_arguments():
    torch.cuda.set_device(0)
    plan = Plan(32, 0.5, 16.0)
    a = torch.zeros((10, plan.p_half, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(FBError):
        plan.svd(a[:0])
    small = torch.empty(8, dtype=torch.uint8, device="cuda")
    from paper_1412_0781_amd._lib import lib
    ev = torch.empty(plan.p_half, dtype=torch.float64, device="cuda")
    U = torch.empty(plan.cov_size, dtype=torch.float64, device="cuda")
    rc = lib().fb_svd(plan._h, a.data_ptr(), 10, ev.data_ptr(), U.data_ptr(), None, small.data_ptr(), 8, None)
    assert rc != 0
