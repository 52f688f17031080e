"""Plain FP64 restatement of the CTF-filtered workload and of the estimation of the
support radius R and the band limit c from a set of noisy images (Sec. VI-C) — test
oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

Readings (the paper does not print them):
* The pixel size Delta of the CTF frequencies f = xi / Delta is a parameter, 1 Angstrom by
  default (with B = 100 A^2 the envelope is then 0.02 near xi = 0.2, where the paper's
  estimate of c lies).
* The mean radial variance is the average of the per-pixel variance over integer-radius
  bins round(|x|); the cumulative variance integrates (v(r) - sigma^2) r dr as the sum over
  bins r = 0 .. floor(L/2) of (v_r - sigma^2) r; R is the smallest bin radius at which the
  cumulative sum reaches `frac` of its total.
* The mean radial power spectrum is the average of |F(I - mean)|^2 / L^2 over the images
  and the angles of each ring xi_j of the plan (a plan with c = 1/2 covers the band up to
  Nyquist); the cumulative power integrates (p(xi) - sigma^2) xi dxi with the plan's
  Gauss-Legendre weights; c is the smallest ring xi_j at which it reaches `frac` of its
  total.  With unit normalisation of Eq.(nufft), white noise of variance sigma^2 has
  E|F|^2 / L^2 = sigma^2, the level both curves settle at.
"""

from __future__ import annotations

import math

import numpy as np

from .fb import Plan, nudft_polar, pixel_coords

# Sec. VI-C: wavelength, defocus (2.5 um), amplitude phase, B-factor
CTF_LAMBDA = 0.0197      # Angstrom
CTF_DEFOCUS = 2.5e4      # Angstrom
CTF_PHASE = 0.1          # rad
CTF_B = 100.0            # Angstrom^2


def ctf_envelope(xi, pixel_size: float = 1.0, lam: float = CTF_LAMBDA, z: float = CTF_DEFOCUS,
                 a: float = CTF_PHASE, B: float = CTF_B) -> np.ndarray:
    """Eq.(CTFenv): min(pi lambda z f^2 + a, 1) exp(-B f^2) at f = xi / pixel_size."""
    f2 = (np.asarray(xi, dtype=np.float64) / pixel_size) ** 2
    return np.minimum(math.pi * lam * z * f2 + a, 1.0) * np.exp(-B * f2)


def pixel_moments(images: np.ndarray):
    """Per-pixel sum and sum of squares over the images (FP64)."""
    x = np.asarray(images, dtype=np.float64)
    return x.sum(axis=0), (x * x).sum(axis=0)


def polar_power(images: np.ndarray, pl: Plan, mean_image: np.ndarray | None = None) -> np.ndarray:
    """sum over the images and the half-ring angles l < n_theta/2 of |F(I - mean)(xi_j, theta_l)|^2
    (Eq.(nufft) by the direct sum), per ring j.  For a real image the other half ring
    holds the same magnitudes."""
    x = np.asarray(images, dtype=np.float64)
    if mean_image is not None:
        x = x - np.asarray(mean_image, dtype=np.float64)[None]
    F = nudft_polar(x, pl)[:, :, :pl.n_theta // 2]
    return np.sum(np.abs(F) ** 2, axis=(0, 2))


def radial_variance(sum_img: np.ndarray, sumsq_img: np.ndarray, n: int, L: int) -> np.ndarray:
    """Mean radial variance v_r over integer-radius bins r = round(|x|), r = 0 .. floor(L/2)."""
    m = sum_img / n
    v = sumsq_img / n - m * m
    x = pixel_coords(L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    r = np.rint(np.hypot(X1, X2)).astype(np.int64)
    rmax = L // 2
    keep = r <= rmax
    tot = np.bincount(r[keep], weights=v[keep], minlength=rmax + 1)
    cnt = np.bincount(r[keep], minlength=rmax + 1)
    return tot / cnt


def estimate_support(sum_img, sumsq_img, n: int, power: np.ndarray, pl: Plan, noise_var: float,
                     frac: float = 0.999):
    """(R, c) by the cumulative-fraction rule of Sec. VI-C applied to the mean radial variance
    (radius R in pixels) and to the mean radial power spectrum on the plan's rings (c)."""
    v = radial_variance(np.asarray(sum_img, np.float64), np.asarray(sumsq_img, np.float64), n, pl.L)
    r = np.arange(v.size, dtype=np.float64)
    cv = np.cumsum((v - noise_var) * r)
    R = int(np.argmax(cv >= frac * cv[-1]))
    p = np.asarray(power, np.float64) / (n * (pl.n_theta // 2) * pl.L * pl.L)
    cp = np.cumsum((p - noise_var) * pl.xi * pl.w)
    c = float(pl.xi[int(np.argmax(cp >= frac * cp[-1]))])
    return R, c
