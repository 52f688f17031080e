"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the Fourier-Bessel method itself: it draws
random numbers and fixes the workload recipe (variance profile of the random
coefficients, noise level).  Turning coefficients into images is the job of
whichever synthesis operator the caller uses.

Random numbers come from Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), a counter-based generator, so that
any image of a dataset can be regenerated on its own from (seed, stream, index).
The device library carries its own implementation of the same published
generator; the two agree bit for bit on the 32-bit words.

Counter layout (one 128-bit counter per 4 words):
    ctr = (word_block, index_lo, index_hi, stream),  key = (seed_lo, seed_hi)
where ``index`` is the image index, ``stream`` selects what is drawn
(STREAM_COEF for coefficients, STREAM_NOISE for pixel noise) and
``word_block`` counts blocks of 4 words inside one image.

Normal deviates use the Box-Muller transform on consecutive word pairs:
u1 = (w0 + 1) * 2^-32 in (0, 1], u2 = w1 * 2^-32 in [0, 1),
z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = sqrt(-2 ln u1) sin(2 pi u2).
"""

from __future__ import annotations

import math

import numpy as np

PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint32(0x9E3779B9)
PHILOX_W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_COEF = 1
STREAM_NOISE = 2


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """Philox-4x32 with 10 rounds.  ctr: uint32 [..., 4], key: uint32 [..., 2]."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32).copy()
    k1 = np.asarray(key[..., 1], dtype=np.uint32).copy()
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = (k0 + PHILOX_W0).astype(np.uint32)
                k1 = (k1 + PHILOX_W1).astype(np.uint32)
            p0 = PHILOX_M0 * c[0].astype(np.uint64)
            p1 = PHILOX_M1 * c[2].astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def _words(seed: int, stream: int, index: np.ndarray, n_words: int) -> np.ndarray:
    """uint32 words [len(index), n_words] for images ``index`` of a stream."""
    index = np.asarray(index, dtype=np.uint64)
    nblk = (n_words + 3) // 4
    blk = np.arange(nblk, dtype=np.uint32)
    ctr = np.empty((index.size, nblk, 4), dtype=np.uint32)
    ctr[..., 0] = blk[None, :]
    ctr[..., 1] = (index & MASK32).astype(np.uint32)[:, None]
    ctr[..., 2] = (index >> np.uint64(32)).astype(np.uint32)[:, None]
    ctr[..., 3] = np.uint32(stream)
    key = np.empty((index.size, nblk, 2), dtype=np.uint32)
    key[..., 0] = np.uint32(seed & 0xFFFFFFFF)
    key[..., 1] = np.uint32((seed >> 32) & 0xFFFFFFFF)
    return philox4x32_10(ctr, key).reshape(index.size, nblk * 4)[:, :n_words]


def normals(seed: int, stream: int, index, n_per: int) -> np.ndarray:
    """Standard normal deviates, float64 [len(index), n_per], by Box-Muller on word pairs."""
    n_pairs = (n_per + 1) // 2
    w = _words(seed, stream, index, 2 * n_pairs).astype(np.float64)
    u1 = (w[:, 0::2] + 1.0) * 2.0 ** -32
    u2 = w[:, 1::2] * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((w.shape[0], 2 * n_pairs))
    z[:, 0::2] = rad * np.cos(2.0 * math.pi * u2)
    z[:, 1::2] = rad * np.sin(2.0 * math.pi * u2)
    return z[:, :n_per]


# ----------------------------------------------------------------------------
# Workload recipe
# ----------------------------------------------------------------------------
def coef_variance(k: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Variance profile of the random clean coefficients: (1+q)^-2 (1+|k|)^-1."""
    k = np.asarray(k, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    return 1.0 / ((1.0 + q) ** 2 * (1.0 + np.abs(k)))


def clean_signal_power(k: np.ndarray, q: np.ndarray, L: int) -> float:
    """Mean clean pixel power over the L x L grid for coefficients of variance
    ``coef_variance`` (k >= 0 listed once; +-k both counted), assuming the
    synthesis operator is close to an isometry."""
    v = coef_variance(k, q)
    k = np.asarray(k)
    return float((v[k == 0].sum() + 2.0 * v[k > 0].sum()) / (L * L))


def noise_sigma2(k, q, L: int, snr: float) -> float:
    """White-noise variance giving signal-to-noise ratio ``snr`` (power ratio)."""
    return clean_signal_power(k, q, L) / snr


def random_coefficients(seed: int, index, k: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Complex coefficients [len(index), p_half] with variance coef_variance(k, q).

    k = 0 entries are real N(0, v); k > 0 entries are circular complex
    (real and imaginary parts each N(0, v/2))."""
    k = np.asarray(k)
    v = coef_variance(k, q)
    z = normals(seed, STREAM_COEF, index, 2 * k.size)
    re = z[:, 0::2]
    im = z[:, 1::2]
    out = np.where(k[None, :] == 0, np.sqrt(v)[None, :] * re,
                   np.sqrt(v / 2.0)[None, :] * re) + 1j * np.where(
        k[None, :] == 0, 0.0, np.sqrt(v / 2.0)[None, :] * im)
    return out


def noise_images(seed: int, index, L: int, sigma: float) -> np.ndarray:
    """White Gaussian noise images, float64 [len(index), L, L], standard deviation sigma."""
    return sigma * normals(seed, STREAM_NOISE, index, L * L).reshape(-1, L, L)
