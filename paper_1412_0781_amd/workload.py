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


def synthetic_images(plan, first: int, m: int, seed: int, snr: float, out: torch.Tensor | None = None,
                     batch: int = 2048) -> torch.Tensor:
    """Images first .. first+m-1 of the seeded workload, float32 [m, L, L] on the device."""
    L = plan.L
    if out is None:
        out = torch.empty((m, L, L), dtype=torch.float32, device=plan.device)
    if m == 0:
        return out
    a = synth_normals(seed, synth.STREAM_COEF, first, m, 2 * plan.p_half, 1.0, plan.device).view(m, plan.p_half, 2)
    a.mul_(coefficient_scale(plan))
    plan.adjoint(a, out=out, batch=min(m, batch))
    out.add_(synth_normals(seed, synth.STREAM_NOISE, first, m, L * L, noise_sigma(plan, snr), plan.device)
             .view(m, L, L))
    return out
