"""Shared helpers of the GPU tests: seeded inputs built on the host (never by the
HIP path) and error measures."""

import numpy as np

import oracle
from paper_1412_0781_amd import synth


def structured_images(pl_or, n, seed=0, snr=0.1, first=0):
    """Images with the workload's structure: the oracle's synthesis T a of random
    coefficients with variance (1+q)^-2 (1+|k|)^-1, plus white noise at the given SNR.
    Rounded to float32 so that both sides see identical inputs."""
    idx = np.arange(first, first + n)
    k, q = pl_or.kq[:, 0], pl_or.kq[:, 1]
    a = synth.random_coefficients(seed, idx, k, q)
    clean = oracle.adjoint(a, pl_or)
    sigma = np.sqrt(synth.noise_sigma2(k, q, pl_or.L, snr))
    img = clean + synth.noise_images(seed, idx, pl_or.L, sigma)
    return img.astype(np.float32)


def noise_images(L, n, seed=0, first=0):
    return synth.noise_images(seed, np.arange(first, first + n), L, 1.0).astype(np.float32)


def rel_l2(x, ref):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(ref)) / np.linalg.norm(np.asarray(ref)))


def as_complex(coeffs_t):
    c = coeffs_t.detach().cpu().numpy().astype(np.float64)
    return c[..., 0] + 1j * c[..., 1]


def sparse_images(L, n, npix, seed):
    """n images with npix nonzero pixels each (positions anywhere on the L x L grid,
    values N(0,1) rounded to float32), as a dense float32 array and as the pixel lists
    the oracle's sparse evaluation takes.  numpy's seeded generator; host only."""
    rng = np.random.default_rng(seed)
    dense = np.zeros((n, L, L), np.float32)
    pix = []
    for i in range(n):
        flat = rng.choice(L * L, size=npix, replace=False)
        r, c = flat // L, flat % L
        v = rng.standard_normal(npix).astype(np.float32)
        dense[i, r, c] = v
        pix.append((r, c, v.astype(np.float64)))
    return dense, pix


def max_block_rel(got, ref, coef_off):
    """Largest relative L2 error of one angular-frequency block: max over k of
    ||a_k - a_k,ref|| / ||a_k,ref||, each block taken over all images and q."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    worst = 0.0
    for k in range(len(coef_off) - 1):
        o0, o1 = int(coef_off[k]), int(coef_off[k + 1])
        d = np.linalg.norm(got[..., o0:o1] - ref[..., o0:o1])
        worst = max(worst, float(d / np.linalg.norm(ref[..., o0:o1])))
    return worst


def dictionary_images(L, n, D, seed, offset=0.0):
    """n float32 images that combine D pixels of a fixed random dictionary: image i holds
    V[i, d] at pixel (rows[d], cols[d]) and 0 elsewhere, V ~ N(offset, 1) rounded to float32
    (offset > 0 gives a large mean image).  numpy's seeded generator; host only.  Returns the
    dense images, V (float64 copy of the float32 values), rows and cols."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(L * L, size=D, replace=False)
    rows, cols = flat // L, flat % L
    V = (rng.standard_normal((n, D)) + offset).astype(np.float32)
    dense = np.zeros((n, L, L), np.float32)
    dense[:, rows, cols] = V
    return dense, V.astype(np.float64), rows, cols
