"""Seeded synthetic images on the device (the stand-in for the paper's image sets).

Image i is the synthesis T a_i of random Fourier-Bessel coefficients with variance
(1+q)^-2 (1+|k|)^-1 (k = 0 real, k > 0 circular complex) plus white Gaussian noise of
variance P_s / SNR, P_s the mean clean pixel power.  Every random number comes from
Philox-4x32-10 keyed by (seed, image index, stream), so image i is the same whichever
chunk or pass produces it.  The arithmetic runs in the library's kernels (fb_synth_normals,
fb_adjoint); this module only sizes and scales.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import synth
from .fb import synth_normals


def coefficient_scale(plan) -> torch.Tensor:
    """Per-coefficient (Re, Im) standard deviations, float32 [p_half, 2] on the plan's device."""
    k = plan.k.astype(np.float64)
    q = plan.q.astype(np.float64)
    v = synth.coef_variance(k, q)
    sc = np.zeros((plan.p_half, 2), np.float32)
    sc[:, 0] = np.where(k == 0, np.sqrt(v), np.sqrt(v / 2))
    sc[:, 1] = np.where(k == 0, 0.0, np.sqrt(v / 2))
    return torch.tensor(sc, device=plan.device)


def noise_sigma(plan, snr: float) -> float:
    return math.sqrt(synth.noise_sigma2(plan.k.astype(np.float64), plan.q.astype(np.float64), plan.L, snr))


# Sec. VI-C, CTF-filtered workload: wavelength and defocus (Angstrom), amplitude phase (rad),
# B-factor (Angstrom^2).  The pixel size is not printed; 1 Angstrom by default.
CTF_LAMBDA, CTF_DEFOCUS, CTF_PHASE, CTF_B = 0.0197, 2.5e4, 0.1, 100.0


def ctf_ring_filter(plan, pixel_size: float = 1.0, lam: float = CTF_LAMBDA, z: float = CTF_DEFOCUS,
                    a: float = CTF_PHASE, B: float = CTF_B) -> torch.Tensor:
    """Eq.(CTFenv), min(pi lambda z f^2 + a, 1) exp(-B f^2) at f = xi_j / pixel_size, on the plan's
    rings: float32 [n_xi] on the device (fb_ctf_filter), for fb_adjoint_filtered."""
    return plan.ctf_filter(pixel_size, lam, z, a, B)


def synthetic_images(plan, first: int, m: int, seed: int, snr: float, out: torch.Tensor | None = None,
                     batch: int = 2048, ring_filter: torch.Tensor | None = None,
                     sigma: float | None = None) -> torch.Tensor:
    """Images first .. first+m-1 of the seeded workload, float32 [m, L, L] on the device.
    ring_filter: a radial Fourier filter of the clean images (the CTF workload); sigma: the
    noise standard deviation (default from snr and the unfiltered clean power)."""
    L = plan.L
    if out is None:
        out = torch.empty((m, L, L), dtype=torch.float32, device=plan.device)
    if m == 0:
        return out
    a = synth_normals(seed, synth.STREAM_COEF, first, m, 2 * plan.p_half, 1.0, plan.device).view(m, plan.p_half, 2)
    a.mul_(coefficient_scale(plan))
    plan.adjoint(a, out=out, batch=min(m, batch), ring_filter=ring_filter)
    s = noise_sigma(plan, snr) if sigma is None else float(sigma)
    out.add_(synth_normals(seed, synth.STREAM_NOISE, first, m, L * L, s, plan.device).view(m, L, L))
    return out
