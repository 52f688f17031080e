"""GPU parity of the covariance and eigendecomposition (Algorithm 2, steps 1, 3,
4) and of the adjoint T, through the C ABI, against the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle
from gpu_util import as_complex, noise_images, rel_l2, structured_images
from paper_1412_0781_amd import FBExpand, FBSynth, Plan, synth, synth_normals, synth_words

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _dev():
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_covariance_and_eig_workload_L32(precision):
    """n = 1000, L = 32, R = 16, SNR 1/10 (the FP64 reference workload): C^(k) and lambda
    within 1e-5 relative of the oracle computed from the oracle's own coefficients."""
    L, c, R, n = 32, 0.5, 16, 1000
    print(f"[cov] L={L} n={n} {precision}", flush=True)
    po = oracle.plan(L, c, R)
    img = structured_images(po, n, seed=0, snr=0.1)
    a_ref = oracle.expand(img.astype(np.float64), po)
    mean_ref, C_ref = oracle.mean_and_covariance(a_ref, po)
    lam_ref, U_ref = oracle.eig_blocks(C_ref)

    plan = Plan(L, c, R)
    x = torch.tensor(img, device="cuda")
    st = plan.new_covariance()
    for s in range(0, n, 300):  # accumulate over several calls
        a = plan.expand(x[s:s + 300], precision=precision)
        plan.covariance(a, st, precision=precision)
    evals, evecs, C, mean = plan.eig(st)
    torch.cuda.synchronize()
    assert st.count == n
    C = C.cpu().numpy()
    Cb = plan.blocks(C)
    worst = max(np.linalg.norm(Cb[k] - C_ref[k]) / np.linalg.norm(C_ref[k]) for k in range(po.k_max + 1))
    print(f"  worst per-k C rel {worst:.3e}", flush=True)
    assert worst <= TOL
    assert rel_l2(mean.cpu().numpy(), mean_ref) <= TOL
    lam = evals.cpu().numpy()
    for k in range(po.k_max + 1):
        o = po.coef_off[k]
        assert np.max(np.abs(lam[o:o + po.p[k]] - lam_ref[k])) <= TOL * np.max(np.abs(lam_ref[k]))
    # eigenvectors where the eigenvalue gap is large enough to make them unique
    V = plan.blocks(evecs.cpu().numpy())
    for k in range(po.k_max + 1):
        lr = lam_ref[k]
        for l in range(po.p[k]):
            gap = min([abs(lr[l] - lr[m]) for m in range(po.p[k]) if m != l] or [np.inf])
            if gap > 1e-2 * abs(lr[0]):
                assert np.max(np.abs(V[k][:, l] - U_ref[k][:, l])) <= 1e-3, (k, l)


def test_eig_is_an_eigendecomposition_of_C():
    plan = Plan(64, 0.5, 32)
    x = torch.tensor(noise_images(64, 500, seed=2), device="cuda")
    st = plan.covariance(plan.expand(x))
    evals, evecs, C, _ = plan.eig(st)
    torch.cuda.synchronize()
    Cb = plan.blocks(C.cpu().numpy())
    Vb = plan.blocks(evecs.cpu().numpy())
    lam = evals.cpu().numpy()
    for k in range(plan.k_max + 1):
        o = plan.coef_off[k]
        lk = lam[o:o + plan.p[k]]
        assert np.all(np.diff(lk) <= 0)
        V = Vb[k]
        assert np.allclose(V.T @ V, np.eye(plan.p[k]), atol=1e-12)
        assert np.allclose(Cb[k] @ V, V * lk[None, :], atol=1e-12 * max(1.0, abs(lk).max()))


def test_eig_rank_deficient_blocks():
    """Fewer images than coefficients per block: the blocks have null directions and
    eigenvalues spanning many orders of magnitude.  The one-sided form accumulates its
    rotations, so the eigenvectors stay orthonormal with residuals at FP64 rounding of ||C||
    and the eigenvalues equal LAPACK's."""
    plan = Plan(64, 0.5, 32)
    po = oracle.plan(64, 0.5, 32)
    x = torch.tensor(noise_images(64, 9, seed=4), device="cuda")
    a = plan.expand(x)
    st = plan.covariance(a)
    evals, evecs, C, _ = plan.eig(st)
    torch.cuda.synchronize()
    Cb = plan.blocks(C.cpu().numpy())
    Vb = plan.blocks(evecs.cpu().numpy())
    lam = evals.cpu().numpy()
    lam_ref, _ = oracle.eig_blocks(Cb)
    for k in range(plan.k_max + 1):
        o = plan.coef_off[k]
        lk = lam[o:o + plan.p[k]]
        assert np.all(np.diff(lk) <= 0)
        V = Vb[k]
        assert np.allclose(V.T @ V, np.eye(plan.p[k]), atol=1e-12)
        scale = max(1.0, abs(lk).max())
        assert np.allclose(Cb[k] @ V, V * lk[None, :], atol=1e-12 * scale)
        assert np.max(np.abs(lk - lam_ref[k])) <= 1e-12 * scale


def test_covariance_deterministic_and_additive():
    plan = Plan(32, 0.5, 16)
    x = torch.tensor(noise_images(32, 700, seed=9), device="cuda")
    a = plan.expand(x)
    s1 = plan.covariance(a)
    s2 = plan.covariance(a)
    s3 = plan.covariance(a[:350])
    plan.covariance(a[350:], s3)
    u1 = plan.covariance(a, plan.new_covariance(shift=False))
    u3 = plan.covariance(a[:350], plan.new_covariance(shift=False))
    plan.covariance(a[350:], u3)
    torch.cuda.synchronize()
    assert torch.equal(s1.G, s2.G) and torch.equal(s1.S0, s2.S0) and torch.equal(s1.shift, s2.shift)
    # splitting the images over two calls only moves FP32 partial-sum boundaries
    assert float((u1.G - u3.G).norm() / u1.G.norm()) <= 1e-6
    assert float((u1.S0 - u3.S0).norm() / u1.S0.norm()) <= 1e-6
    # the shift of s3 comes from its first 350 images, that of s1 from the first 700: the
    # finalised blocks and means agree all the same
    e1, _, C1, m1 = plan.eig(s1)
    e3, _, C3, m3 = plan.eig(s3)
    eu, _, Cu, mu = plan.eig(u1)
    torch.cuda.synchronize()
    for C, m in [(C3, m3), (Cu, mu)]:
        assert float((C1 - C).norm() / C1.norm()) <= 1e-6
        assert float((m1 - m).norm() / m1.norm()) <= 1e-6
    # with no shift the k = 0 sums are the plain sums
    a0 = a[:, :plan.p0, 0].double()
    assert float((u1.S0 - a0.sum(0)).norm() / a0.sum(0).norm()) <= 1e-6
    assert float((s1.shift.double() + s1.S0 / 700 - a0.mean(0)).norm() / a0.mean(0).norm()) <= 1e-6


def _mean_image_workload(po, n, seed, ratio):
    """The workload's images plus one fixed image whose k = 0 coefficients are ratio times
    the standard deviation of each a_{0,q} (a large mean image, as in real data)."""
    img = structured_images(po, n, seed=seed, snr=0.1)
    m = np.zeros((1, po.p_half), np.complex128)
    q = np.arange(1, po.p[0] + 1)
    m[0, :po.p[0]] = ratio * (1.0 + q) ** -1.0
    mean_img = oracle.adjoint(m, po)[0]
    return (img + mean_img[None]).astype(np.float32)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_covariance_large_mean(precision):
    """A mean image 10x the spread of the k = 0 coefficients: the shifted accumulation keeps
    C^(0) and its eigenvalues within 1e-5 of the oracle in both forms (Algorithm 2 step 1
    subtracts the mean before the products)."""
    L, c, R, n = 32, 0.5, 16, 1000
    print(f"[cov] large mean L={L} n={n} {precision}", flush=True)
    po = oracle.plan(L, c, R)
    img = _mean_image_workload(po, n, seed=4, ratio=10.0)
    a_ref = oracle.expand(img.astype(np.float64), po)
    mean_ref, C_ref = oracle.mean_and_covariance(a_ref, po)
    lam_ref, _ = oracle.eig_blocks(C_ref)
    plan = Plan(L, c, R)
    a = plan.expand(torch.tensor(img, device="cuda"), precision=precision)
    errs = {}
    for shift in (True, False):
        st = plan.new_covariance(shift=shift)
        for s in range(0, n, 300):
            plan.covariance(a[s:s + 300], st, precision=precision)
        evals, _, C, mean = plan.eig(st)
        torch.cuda.synchronize()
        C0 = plan.blocks(C.cpu().numpy())[0]
        lam0 = evals.cpu().numpy()[:po.p[0]]
        errs[shift] = (rel_l2(C0, C_ref[0]), np.max(np.abs(lam0 - lam_ref[0])) / lam_ref[0][0],
                       rel_l2(mean.cpu().numpy(), mean_ref))
    print(f"  C^(0), lambda^(0), mean rel err: shifted {errs[True]}, unshifted {errs[False]}", flush=True)
    assert max(errs[True]) <= TOL
    assert np.linalg.norm(mean_ref) > 5 * np.sqrt(np.trace(C_ref[0]))  # the mean dominates


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_hermitian_covariance(precision):
    """The imaginary parts Im(A A^*) of the rotation-only (SO(2)) covariance: (G + i Gi)/n
    within 1e-5 of the oracle's Hermitian blocks for every k, and G bitwise the same as
    without them."""
    L, c, R, n = 32, 0.5, 16, 1000
    print(f"[cov] hermitian L={L} n={n} {precision}", flush=True)
    po = oracle.plan(L, c, R)
    img = structured_images(po, n, seed=6, snr=0.1)
    a_ref = oracle.expand(img.astype(np.float64), po)
    _, CH = oracle.hermitian_covariance(a_ref, po)
    plan = Plan(L, c, R)
    a = plan.expand(torch.tensor(img, device="cuda"), precision=precision)
    st = plan.new_covariance(hermitian=True)
    plain = plan.new_covariance()
    for s in range(0, n, 400):
        plan.covariance(a[s:s + 400], st, precision=precision)
        plan.covariance(a[s:s + 400], plain, precision=precision)
    torch.cuda.synchronize()
    assert torch.equal(st.G, plain.G) and torch.equal(st.S0, plain.S0)
    G = plan.blocks(st.G.cpu().numpy())
    Gi = plan.blocks(st.Gi.cpu().numpy())
    assert np.all(Gi[0] == 0.0)
    worst = 0.0
    for k in range(1, po.k_max + 1):
        got = (G[k] + 1j * Gi[k]) / n
        worst = max(worst, np.linalg.norm(got - CH[k]) / np.linalg.norm(CH[k]))
        assert np.array_equal(Gi[k], -Gi[k].T)
    print(f"  worst per-k Hermitian rel {worst:.3e}", flush=True)
    assert worst <= TOL


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16), (31, 0.5, 15.5), (64, 0.3, 32),
                                   (16, 0.5, 8)])   # grid and angular length 32: run-time-length FFT forms
def test_adjoint_matches_oracle(L, c, R):
    print(f"[adjoint] L={L} c={c} R={R}", flush=True)
    po = oracle.plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(4, np.arange(6), k, q)
    ref = oracle.adjoint(b, po)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    got = plan.adjoint(bt).cpu().numpy()
    assert rel_l2(got, ref) <= TOL


def test_adjoint_many_images():
    """300 images: 19 image groups, so two slices of the spread's 16-group slices (the
    second ragged) and a partly filled last group.  Sampled images against the oracle; a
    ragged sub-batch gives the same images as the full batch."""
    L, c, R = 64, 0.5, 32
    print(f"[adjoint] L={L} n=300", flush=True)
    po = oracle.plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(9, np.arange(300), k, q)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    full = plan.adjoint(bt).cpu().numpy()
    pick = [0, 17, 150, 299]
    ref = oracle.adjoint(b[pick], po)
    assert rel_l2(full[pick], ref) <= TOL
    part = plan.adjoint(bt[280:]).cpu().numpy()
    assert np.max(np.abs(part - full[280:])) <= 1e-6 * np.max(np.abs(full[280:]))


def test_adjoint_l128_split_cells_match_oracle_and_repeat():
    """L = 128: the spread shares the crowded cells near the origin over several tiles and
    gives their heaviest pairs up to 8 lane groups whose sums meet in a butterfly, and cuts
    many cells into several chunks.  Sampled images of a 300-image batch against the
    oracle; the same batch again, and in other pass sizes, bit for bit (fixed summation
    order, no atomics)."""
    L, c, R = 128, 0.5, 64
    print(f"[adjoint] L={L} n=300 split cells", flush=True)
    po = oracle.plan(L, c, R)
    k, q = po.kq[:, 0], po.kq[:, 1]
    b = synth.random_coefficients(12, np.arange(300), k, q)
    plan = Plan(L, c, R)
    bt = torch.tensor(np.stack([b.real, b.imag], axis=-1).astype(np.float32), device="cuda")
    full = plan.adjoint(bt).clone()
    again = plan.adjoint(bt)
    small = plan.adjoint(bt, batch=48)
    torch.cuda.synchronize()
    assert torch.equal(full, again)
    assert torch.equal(full, small)
    pick = [5, 211]
    ref = oracle.adjoint(b[pick], po)
    assert rel_l2(full.cpu().numpy()[pick], ref) <= TOL


@pytest.mark.parametrize("L,c,R", [(32, 0.5, 16), (128, 0.5, 64), (31, 0.5, 15.5), (256, 0.5, 128)])
def test_dot_product_identity_gpu(L, c, R):
    """<T* I, b> = <I, T b> with the folded inner product, to 1e-6 in FP32 relative to the
    inner product itself: b is the oracle's expansion of I plus 10 % noise, so <T* I, b> is
    close to ||T* I||^2 and cannot cancel."""
    plan = Plan(L, c, R)
    po = oracle.plan(L, c, R)
    rng = np.random.default_rng(1)
    I_np = rng.standard_normal((4, L, L)).astype(np.float32)
    a_or = oracle.expand(I_np.astype(np.float64), po)
    noise = rng.standard_normal(a_or.shape) + 1j * rng.standard_normal(a_or.shape)
    bc = a_or + 0.1 * np.linalg.norm(a_or, axis=1, keepdims=True) / np.sqrt(po.p_half) * noise
    bc[:, :po.p[0]] = bc[:, :po.p[0]].real
    b = np.stack([bc.real, bc.imag], axis=-1).astype(np.float32)
    bc = b[..., 0].astype(np.float64) + 1j * b[..., 1].astype(np.float64)
    I = torch.tensor(I_np, device="cuda")
    bt = torch.tensor(b, device="cuda")
    a = as_complex(plan.expand(I))
    Tb = plan.adjoint(bt).cpu().numpy().astype(np.float64)
    lhs = oracle.coeff_inner(a, bc, po)
    rhs = np.sum(I_np.astype(np.float64) * Tb, axis=(1, 2))
    rel = np.abs(lhs - rhs) / np.abs(lhs)
    # the inner products do not cancel: each is at least half of ||T* I|| ||b||
    assert np.all(np.abs(lhs) >= 0.5 * np.sqrt(oracle.coeff_inner(a, a, po) * oracle.coeff_inner(bc, bc, po)))
    print(f"  dot test {np.max(rel):.3e}", flush=True)
    assert np.max(rel) <= 1e-6


def test_dot_product_identity_large_blocks():
    """L = 456: blocks of up to 227 coefficients, more than the adjoint's radial step keeps
    resident in LDS, so its table is read by chunks; <T* I, b> = <I, T b> with b = T* I plus
    10 % noise (so that neither side cancels), to 1e-6."""
    L, c, R = 456, 0.5, 228.0
    print(f"[adjoint] dot test L={L}", flush=True)
    plan = Plan(L, c, R)
    assert max(int(x) for x in plan.p) > 224
    rng = np.random.default_rng(3)
    I_np = rng.standard_normal((3, L, L)).astype(np.float32)
    I = torch.tensor(I_np, device="cuda")
    a = plan.expand(I)
    noise = torch.tensor(rng.standard_normal(tuple(a.shape)).astype(np.float32), device="cuda")
    scale = a.norm(dim=(1, 2), keepdim=True) / np.sqrt(plan.p_half)
    bt = a + 0.1 * scale * noise
    bt[:, :int(plan.p[0]), 1] = 0.0
    Tb = plan.adjoint(bt).cpu().numpy().astype(np.float64)
    ac, bc = as_complex(a), as_complex(bt)
    p0 = int(plan.p[0])
    lhs = (np.sum(ac[:, :p0].real * bc[:, :p0].real, axis=1)
           + 2.0 * np.sum((np.conj(ac[:, p0:]) * bc[:, p0:]).real, axis=1))
    rhs = np.sum(I_np.astype(np.float64) * Tb, axis=(1, 2))
    rel = np.abs(lhs - rhs) / np.abs(lhs)
    print(f"  dot test {np.max(rel):.3e}", flush=True)
    assert np.max(rel) <= 1e-6


def test_autograd_expand_dot_identity():
    """FBExpand backward is the plain transpose of the expansion (weight 1 for every k)."""
    L = 32
    plan = Plan(L, 0.5, 16)
    rng = np.random.default_rng(2)
    I = torch.tensor(rng.standard_normal((3, L, L)).astype(np.float32), device="cuda", requires_grad=True)
    g = torch.tensor(rng.standard_normal((3, plan.p_half, 2)).astype(np.float32), device="cuda")
    g[:, :plan.p0, 1] = 0
    a = FBExpand.apply(I, plan, "fp32")
    (a * g).sum().backward()
    lhs = float((a.detach().double() * g.double()).sum())
    rhs = float((I.detach().double() * I.grad.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(a.detach().double().norm() * g.double().norm())


def test_autograd_synth_gradient():
    L = 32
    plan = Plan(L, 0.5, 16)
    rng = np.random.default_rng(3)
    b = rng.standard_normal((2, plan.p_half, 2)).astype(np.float32)
    b[:, :plan.p0, 1] = 0
    bt = torch.tensor(b, device="cuda", requires_grad=True)
    out = FBSynth.apply(bt, plan)
    G = torch.tensor(rng.standard_normal((2, L, L)).astype(np.float32), device="cuda")
    (out * G).sum().backward()
    lhs = float((out.detach().double() * G.double()).sum())
    rhs = float((bt.detach().double() * bt.grad.double()).sum())
    assert abs(lhs - rhs) <= 1e-6 * float(out.detach().double().norm() * G.double().norm())


def test_device_philox_matches_host():
    w = synth_words(123, 2, 7, 3, 10).cpu().numpy().view(np.uint32)
    ref = synth._words(123, 2, np.arange(7, 10), 10)
    assert np.array_equal(w, ref)
    z = synth_normals(5, 2, 11, 4, 1001).cpu().numpy()
    zr = synth.normals(5, 2, np.arange(11, 15), 1001)
    assert np.max(np.abs(z - zr)) <= 1e-6 * np.max(np.abs(zr))


def test_empty_batches_are_no_ops():
    """Zero images: the synthesis returns an empty batch, and the covariance state (G, the
    k = 0 sums and the count) is left exactly as it was."""
    plan = Plan(32, 0.5, 16)
    empty = torch.zeros((0, plan.p_half, 2), dtype=torch.float32, device="cuda")
    assert plan.adjoint(empty).shape == (0, 32, 32)
    x = torch.tensor(noise_images(32, 20, seed=6), device="cuda")
    st = plan.covariance(plan.expand(x))
    G0, S00, n0 = st.G.clone(), st.S0.clone(), st.count
    plan.covariance(empty, st)
    torch.cuda.synchronize()
    assert st.count == n0 == 20
    assert torch.equal(st.G, G0) and torch.equal(st.S0, S00)


def test_eig_blocks_above_128_in_lds():
    """L = 276 (p_0 = 137): the largest blocks still fit in LDS but take three entries per
    lane in the rotations; descending eigenvalues equal to LAPACK's, orthonormal
    eigenvectors, residuals at FP64 rounding of ||C||."""
    L = 276
    plan = Plan(L, 0.5, L / 2)
    assert max(plan.p) == 137
    x = torch.tensor(noise_images(L, 200, seed=8), device="cuda")
    evals, evecs, C, _ = plan.eig(plan.covariance(plan.expand(x)))
    torch.cuda.synchronize()
    Cb = plan.blocks(C.cpu().numpy())
    Vb = plan.blocks(evecs.cpu().numpy())
    lam = evals.cpu().numpy()
    for k in [0, 1, 2, plan.k_max // 2]:
        o, pk = plan.coef_off[k], plan.p[k]
        lk, V = lam[o:o + pk], Vb[k]
        scale = abs(lk).max()
        assert np.all(np.diff(lk) <= 0)
        assert np.allclose(V.T @ V, np.eye(pk), atol=1e-12)
        assert np.abs(Cb[k] @ V - V * lk[None, :]).max() <= 1e-12 * scale
        assert np.abs(lk - np.sort(np.linalg.eigvalsh(Cb[k]))[::-1]).max() <= 1e-12 * scale
