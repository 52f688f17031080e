"""Parity at the full workload sizes, through the C ABI.

* The L = 360, R = 180 shape (oversampled grid 720 = 2^4 3^2 5 and angular half length
  720: the compile-time mixed-radix streaming FFT kernels) on whole images: the expansion
  against the oracle, the adjoint against the oracle at sampled pixels, and the two against
  each other by the dot-product identity.
* n = 100 000 images at L = 256 (BF16x3) and L = 128 (FP32), expanded in the passes the
  benchmark times (up to 2048 images per pass).  The oracle cannot expand 10^5 images, so
  the outputs are sampled: sparse images (48 nonzero pixels, which the oracle evaluates
  term by term) are planted at indices on and around pass boundaries among device-generated
  N(0,1) noise images and compared with the oracle; the covariance blocks of sampled k are
  compared with an FP64 host recomputation from the library's own coefficients, and their
  eigenvalues with LAPACK on the library's finalised blocks.
* End to end at L = 256 against the FP64 oracle: 4000 images that combine a dictionary of
  192 pixels (their oracle coefficients are the same combination of the oracle expansions
  of the 192 single-pixel images), with a k = 0 mean far above the spread: coefficients,
  every C^(k), the mean and every eigenvalue, in both forms.
Tolerances: 1e-5 relative L2 (coefficients per image and per k block, covariance blocks);
the k = 0 sums within the FP32 partial-sum bound; eigenvalues 1e-9 of the block's largest
against LAPACK on the same blocks, 1e-5 against the oracle's.
"""

import functools

import numpy as np
import pytest
import torch

import oracle
from gpu_util import as_complex, dictionary_images, max_block_rel, rel_l2, sparse_images
from paper_1412_0781_amd import Plan, synth
from paper_1412_0781_amd.fb import synth_normals

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _dev():
    torch.cuda.set_device(0)
    yield


@functools.lru_cache(maxsize=None)
def _oracle_plan(L, c, R):
    """One oracle plan per shape for the module (its radial table at L = 360 takes tens of
    seconds of scipy Bessel evaluations)."""
    return oracle.plan(L, c, R)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_l360_shape_matches_oracle(precision):
    L, c, R = 360, 0.5, 180.0
    print(f"[fullsize] L={L} {precision}", flush=True)
    po = _oracle_plan(L, c, R)
    dense, pix = sparse_images(L, 3, 48, seed=11)
    ref = oracle.expand_sparse(pix, po)
    plan = Plan(L, c, R)
    got = as_complex(plan.expand(torch.tensor(dense, device="cuda"), precision=precision))
    for i in range(len(pix)):
        e = rel_l2(got[i], ref[i])
        print(f"  image {i}: rel-L2 {e:.3e}", flush=True)
        assert e <= TOL
    blk = max_block_rel(got, ref, po.coef_off)
    print(f"  worst k block {blk:.3e}", flush=True)
    assert blk <= TOL
    assert np.all(got[:, :po.p[0]].imag == 0.0)


def test_l360_adjoint_matches_oracle():
    """The adjoint at L = 360 (radial and angular transposes, spread, 720-point inverse
    column and row transforms) for 3 images of random coefficients, at 96 scattered pixels
    plus the four corners and the centre, against the oracle's type-1 sum at those pixels."""
    L, c, R = 360, 0.5, 180.0
    print(f"[fullsize] adjoint L={L}", flush=True)
    po = _oracle_plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(21, np.arange(3), k, q)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    got = plan.adjoint(bt).cpu().numpy()
    rng = np.random.default_rng(12)
    rows = list(rng.integers(0, L, 96)) + [0, 0, L - 1, L - 1, L // 2]
    cols = list(rng.integers(0, L, 96)) + [0, L - 1, 0, L - 1, L // 2]
    ref = oracle.adjoint_pixels(b, po, rows, cols)
    for i in range(len(b)):
        e = rel_l2(got[i, rows, cols], ref[i])
        print(f"  image {i}: rel-L2 at {len(rows)} pixels {e:.3e}", flush=True)
        assert e <= TOL


def test_l360_dot_product_identity():
    """<T* I, b> = <I, T b> at L = 360 with I = T b, so that both sides are close to
    ||T b||^2 and cannot cancel; 1e-6 relative in FP32."""
    L, c, R = 360, 0.5, 180.0
    print(f"[fullsize] dot test L={L}", flush=True)
    po = _oracle_plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(22, np.arange(4), k, q)
    bc = b.astype(np.complex64).astype(np.complex128)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    img = plan.adjoint(bt)
    a = as_complex(plan.expand(img))
    I = img.cpu().numpy().astype(np.float64)
    lhs = oracle.coeff_inner(a, bc, po)
    rhs = np.sum(I * I, axis=(1, 2))
    rel = np.abs(lhs - rhs) / np.abs(rhs)
    print(f"  dot test {np.max(rel):.3e}", flush=True)
    assert np.max(rel) <= 1e-6


def test_l356_grid720_with_padding():
    """L = 356, R = 176: the grid side is again 720 (712 is not 2,3,5-smooth), so the 720-point
    streaming row and column kernels run with 364 zero-padded columns per row (wider than
    the image), while the half ring of 704 points takes the run-time-length angular form.
    Expansion of sparse images against the oracle, the adjoint at sampled pixels against the
    oracle, and the dot-product identity."""
    L, c, R = 356, 0.5, 176.0
    print(f"[fullsize] L={L} R={R}", flush=True)
    po = _oracle_plan(L, c, R)
    plan = Plan(L, c, R)
    assert plan.grid_n == 720
    dense, pix = sparse_images(L, 2, 48, seed=13)
    ref = oracle.expand_sparse(pix, po)
    got = as_complex(plan.expand(torch.tensor(dense, device="cuda"), precision="fp32"))
    for i in range(len(pix)):
        e = rel_l2(got[i], ref[i])
        print(f"  expand image {i}: rel-L2 {e:.3e}", flush=True)
        assert e <= TOL
    assert max_block_rel(got, ref, po.coef_off) <= TOL
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(23, np.arange(2), k, q)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    img = plan.adjoint(bt)
    rng = np.random.default_rng(14)
    rows = list(rng.integers(0, L, 64)) + [0, L - 1, L // 2]
    cols = list(rng.integers(0, L, 64)) + [L - 1, 0, L // 2]
    aref = oracle.adjoint_pixels(b, po, rows, cols)
    I = img.cpu().numpy().astype(np.float64)
    for i in range(len(b)):
        e = rel_l2(I[i, rows, cols], aref[i])
        print(f"  adjoint image {i}: rel-L2 at {len(rows)} pixels {e:.3e}", flush=True)
        assert e <= TOL
    a = as_complex(plan.expand(img))
    bc = b.astype(np.complex64).astype(np.complex128)
    lhs = oracle.coeff_inner(a, bc, po)
    rhs = np.sum(I * I, axis=(1, 2))
    assert np.max(np.abs(lhs - rhs) / np.abs(rhs)) <= 1e-6


@pytest.mark.parametrize("L,R,precision", [(256, 128.0, "bf16x3"), (128, 64.0, "fp32")])
def test_full_n_sampled(L, R, precision):
    n, c, seed = 100000, 0.5, 5
    print(f"[fullsize] n={n} L={L} {precision}", flush=True)
    plan = Plan(L, c, R)
    idx = [0, 2031, 2032, n // 2 + 7, n - 1]
    x = synth_normals(seed, 2, 0, n, L * L, 1.0).view(n, L, L)
    dense, pix = sparse_images(L, len(idx), 48, seed=seed)
    x[idx] = torch.tensor(dense, device="cuda")
    a = plan.expand(x, precision=precision, batch=2048)
    del x
    po = oracle.plan(L, c, R)
    ref = oracle.expand_sparse(pix, po)
    got = as_complex(a[idx])
    for i, j in enumerate(idx):
        e = rel_l2(got[i], ref[i])
        print(f"  image {j}: rel-L2 {e:.3e}", flush=True)
        assert e <= TOL
    blk = max_block_rel(got, ref, po.coef_off)
    print(f"  worst k block {blk:.3e}", flush=True)
    assert blk <= TOL

    st = plan.covariance(a, precision=precision)
    evals, evecs, C, mean = plan.eig(st)
    torch.cuda.synchronize()
    assert st.count == n
    G = st.G.cpu().numpy()
    Cn = C.cpu().numpy()
    ev = evals.cpu().numpy()
    S0 = st.S0.cpu().numpy()
    a0 = a[:, :plan.p0, 0].double().cpu().numpy()
    sh = st.shift.double().cpu().numpy()
    d0 = (a[:, :plan.p0, 0] - st.shift[None, :]).double().cpu().numpy()  # the FP32 shifted values
    # S0 sums FP32 partials of at most 256 terms: |error| <= 256 * 2^-24 * sum_i |a0_i - s| per q
    assert np.all(np.abs(S0 - d0.sum(axis=0)) <= 256 * 2.0 ** -24 * np.abs(d0).sum(axis=0))
    # the mean is shift + S0 / n, within the same partial-sum bound of the plain mean
    m = mean.cpu().numpy()
    assert np.allclose(sh + S0 / n, m, rtol=1e-13, atol=0)
    assert np.all(np.abs(m - a0.mean(axis=0)) <= 256 * 2.0 ** -24 * np.abs(d0).mean(axis=0) + 1e-12 * np.abs(sh))
    for k in [0, 1, plan.k_max // 3, plan.k_max]:
        o, pk = int(plan.coef_off[k]), int(plan.p[k])
        A = a[:, o:o + pk, :].double().cpu().numpy()
        Ar, Ai = A[..., 0], (A[..., 1] if k > 0 else np.zeros_like(A[..., 1]))
        if k == 0:
            Ar = d0
        Gk_ref = Ar.T @ Ar + Ai.T @ Ai
        Gk = G[plan.cov_off[k]:plan.cov_off[k + 1]].reshape(pk, pk)
        e = rel_l2(Gk, Gk_ref)
        print(f"  G^({k}) p_k={pk}: rel-L2 {e:.3e}", flush=True)
        assert e <= TOL
        Ck = Cn[plan.cov_off[k]:plan.cov_off[k + 1]].reshape(pk, pk)
        lam_ref = np.sort(np.linalg.eigvalsh(Ck))[::-1]
        lam = ev[o:o + pk]
        assert np.abs(lam - lam_ref).max() <= 1e-9 * abs(lam_ref[0])


@pytest.fixture(scope="module")
def c3_dictionary():
    """The L = 256, R = 128 shape: 4000 images combining 192 dictionary pixels with values
    N(3, 1) (a mean image far above the spread), and their FP64 oracle coefficients, the
    covariance blocks and eigenvalues (Algorithm 2, steps 1 and 4) from those coefficients."""
    L, c, R, n, D = 256, 0.5, 128.0, 4000, 192
    po = oracle.plan(L, c, R)
    dense, V, rows, cols = dictionary_images(L, n, D, seed=21, offset=3.0)
    a_ref = oracle.expand_pixel_combinations(V, rows, cols, po)
    mean_ref, C_ref = oracle.mean_and_covariance(a_ref, po)
    lam_ref, _ = oracle.eig_blocks(C_ref)
    return po, dense, a_ref, mean_ref, C_ref, lam_ref


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_c3_covariance_and_eigenvalues_against_oracle(c3_dictionary, precision):
    """End to end at L = 256: coefficients (whole and per k block), every C^(k) (relative
    Frobenius, max over k), the k = 0 mean and every eigenvalue (per block, relative to the
    block's largest) against the FP64 oracle's, for images whose k = 0 mean dominates."""
    po, dense, a_ref, mean_ref, C_ref, lam_ref = c3_dictionary
    print(f"[fullsize] C3 dictionary n={dense.shape[0]} {precision}", flush=True)
    plan = Plan(po.L, po.c, po.R)
    x = torch.tensor(dense, device="cuda")
    a = plan.expand(x, precision=precision)
    st = plan.new_covariance()
    for s0 in range(0, x.shape[0], 1500):
        plan.covariance(a[s0:s0 + 1500], st, precision=precision)
    evals, _, C, mean = plan.eig(st)
    torch.cuda.synchronize()
    got = as_complex(a)
    e_a, e_blk = rel_l2(got, a_ref), max_block_rel(got, a_ref, po.coef_off)
    Cb = plan.blocks(C.cpu().numpy())
    e_C = max(rel_l2(Cb[k], C_ref[k]) for k in range(po.k_max + 1))
    ev = evals.cpu().numpy()
    e_lam = max(np.max(np.abs(ev[po.coef_off[k]:po.coef_off[k + 1]] - lam_ref[k])) / lam_ref[k][0]
                for k in range(po.k_max + 1))
    e_m = rel_l2(mean.cpu().numpy(), mean_ref)
    print(f"  coefficients {e_a:.3e} (worst k block {e_blk:.3e}); C^(k) max over k {e_C:.3e}; "
          f"eigenvalues {e_lam:.3e}; mean {e_m:.3e}", flush=True)
    assert np.linalg.norm(mean_ref) > 3 * np.sqrt(np.trace(C_ref[0]))  # the mean dominates
    assert e_a <= TOL and e_blk <= TOL
    assert e_C <= TOL and e_lam <= TOL and e_m <= TOL


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_l360_covariance_against_oracle(precision):
    """Covariance and mean at L = 360 from host-generated coefficients (600 images, a k = 0
    mean ten times the spread, in two accumulating calls): blocks of up to 179 coefficients
    are spread over several work items, some segments loaded by more than one item with
    the k = 0 sums taken once.  Every C^(k) (relative Frobenius) and the mean against the
    oracle on the same FP32-rounded coefficients."""
    L, c, R, n = 360, 0.5, 180.0, 600
    print(f"[fullsize] covariance L={L} n={n} {precision}", flush=True)
    po = _oracle_plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(31, np.arange(n), k, q)
    b[:, :po.p[0]] += 10.0 * np.sqrt(synth.coef_variance(k[:po.p[0]], q[:po.p[0]]))[None, :]
    b = b.astype(np.complex64)
    mean_ref, C_ref = oracle.mean_and_covariance(b.astype(np.complex128), po)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1), device="cuda")
    st = plan.new_covariance()
    plan.covariance(bt[:350], st, precision=precision)
    plan.covariance(bt[350:], st, precision=precision)
    _, _, C, mean = plan.eig(st)
    torch.cuda.synchronize()
    Cb = plan.blocks(C.cpu().numpy())
    worst = max(rel_l2(Cb[kk], C_ref[kk]) for kk in range(po.k_max + 1))
    e_m = rel_l2(mean.cpu().numpy(), mean_ref)
    print(f"  C^(k) max over k {worst:.3e}; mean {e_m:.3e}", flush=True)
    assert worst <= TOL and e_m <= TOL


def test_l360_eig_two_sided_form():
    """At L = 360 the largest blocks (p_0 = 179) exceed LDS, so the eigendecomposition takes
    the two-sided form in global memory: eigenvalues descending and equal to LAPACK's on the
    finalised blocks, eigenvectors orthonormal with residuals at FP64 rounding of ||C||."""
    L, c, R, n = 360, 0.5, 180.0, 1024
    print(f"[fullsize] eig L={L} n={n}", flush=True)
    plan = Plan(L, c, R)
    x = synth_normals(3, 2, 0, n, L * L, 1.0).view(n, L, L)
    st = plan.covariance(plan.expand(x, precision="fp32"))
    del x
    evals, evecs, C, _ = plan.eig(st)
    torch.cuda.synchronize()
    Cn, Vn, ev = C.cpu().numpy(), evecs.cpu().numpy(), evals.cpu().numpy()
    for k in [0, 1, plan.k_max // 2, plan.k_max]:
        o, pk = int(plan.coef_off[k]), int(plan.p[k])
        Ck = Cn[plan.cov_off[k]:plan.cov_off[k + 1]].reshape(pk, pk)
        V = Vn[plan.cov_off[k]:plan.cov_off[k + 1]].reshape(pk, pk)
        lam = ev[o:o + pk]
        scale = abs(lam).max()
        print(f"  k={k} p_k={pk}", flush=True)
        assert np.all(np.diff(lam) <= 0)
        assert np.allclose(V.T @ V, np.eye(pk), atol=1e-12)
        assert np.abs(Ck @ V - V * lam[None, :]).max() <= 1e-12 * scale
        assert np.abs(lam - np.sort(np.linalg.eigvalsh(Ck))[::-1]).max() <= 1e-12 * scale
