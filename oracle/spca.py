"""Plain FP64 restatement of the steerable PCA back end (Algorithm 2, steps 5-6, and the
component selection and eigenvalue shrinkage of Sec. V) and of the real-space
eigenimages of Sec. VI-B — test oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.

Inputs are the oracle's blocks: eigenvalues lam[k] (descending) and eigenvectors U[k]
(columns u_l, p_k x p_k) of C^(k), the k = 0 mean, and the FB coefficients a [n][p_half].
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special

from .fb import Plan, pixel_coords


def mp_ratio(pl: Plan, n: int) -> np.ndarray:
    """gamma_k of the Marcenko-Pastur law for C^(k) (Sec. V): p_0 / n for k = 0 and
    p_k / (2 n) for k > 0 (the real and imaginary parts give 2n samples)."""
    p = np.asarray(pl.p, dtype=np.float64)
    g = p / (2.0 * n)
    g[0] = p[0] / n
    return g


def mp_upper_edge(pl: Plan, n: int, sigma2: float) -> np.ndarray:
    """lambda_+^(k) = sigma^2 (1 + sqrt(gamma_k))^2, the top of the noise eigenvalue bulk (Sec. V)."""
    return sigma2 * (1.0 + np.sqrt(mp_ratio(pl, n))) ** 2


def select(lam: list, pl: Plan, n: int, sigma2: float) -> np.ndarray:
    """Number of components per k with lambda_l^(k) above lambda_+^(k) (Eq.(compselect))."""
    edge = mp_upper_edge(pl, n, sigma2)
    return np.array([int(np.sum(lam[k] > edge[k])) for k in range(pl.k_max + 1)], dtype=np.int64)


def shrink(lam: np.ndarray, sigma2: float) -> np.ndarray:
    """First-order eigenvalue shrinkage of Sec. V: soft threshold (lambda - sigma^2)_+."""
    return np.maximum(np.asarray(lam) - sigma2, 0.0)


def filter_weights(lam: list, pl: Plan, n: int, sigma2: float) -> list:
    """Per-component coefficient filter: ell / (ell + sigma^2) with ell = (lambda - sigma^2)_+
    for the selected components, 0 for the others (the Wiener filter built from the
    shrunk eigenvalues; the reading of "filter the expansion coefficients")."""
    cnt = select(lam, pl, n, sigma2)
    out = []
    for k in range(pl.k_max + 1):
        ell = shrink(lam[k], sigma2)
        w = ell / (ell + sigma2)
        w[cnt[k]:] = 0.0
        out.append(w)
    return out


def radial_functions(U: list, pl: Plan, xi: np.ndarray | None = None) -> list:
    """f^{k,l}(xi_j) = sum_q N_{k,q} J_k(R_{k,q} xi_j / c) u_l^(k)(q)  (Eq.(sPCArad)),
    at the plan's Gauss-Legendre nodes (or at the given xi); one [n_xi, p_k] array per k."""
    xi = pl.xi if xi is None else np.asarray(xi, dtype=np.float64)
    out = []
    for k in range(pl.k_max + 1):
        R = pl.roots[k]
        N = pl.norms[k]
        Phi = N[None, :] * special.jv(k, np.outer(xi, R) / pl.c)           # [n_xi, p_k]
        out.append(Phi @ U[k])
    return out


def coefficients(a: np.ndarray, mean0: np.ndarray, U: list, pl: Plan) -> np.ndarray:
    """c^i_{k,l} = sum_q a^i_{k,q} u_l^(k)(q)  (Eq.(sPCAcoeff)), with the mean removed from
    the k = 0 coefficients first (Algorithm 2, step 1).  Complex [n][p_half], l ordered
    like q (descending eigenvalue)."""
    a = np.array(a, dtype=np.complex128, copy=True)
    a[:, :pl.p[0]] -= mean0[None, :]
    c = np.empty_like(a)
    for k in range(pl.k_max + 1):
        o = pl.coef_off[k]
        c[:, o:o + pl.p[k]] = a[:, o:o + pl.p[k]] @ U[k]
    return c


def reconstruct(c: np.ndarray, mean0: np.ndarray, U: list, w: list | None, pl: Plan) -> np.ndarray:
    """FB coefficients from steerable-PCA coefficients: a_{k,.} = U^(k) (w_k * c_{k,.}), plus the
    mean for k = 0 (the inverse of `coefficients` when w = 1)."""
    a = np.empty_like(np.asarray(c, dtype=np.complex128))
    for k in range(pl.k_max + 1):
        o = pl.coef_off[k]
        ck = c[:, o:o + pl.p[k]]
        if w is not None:
            ck = ck * w[k][None, :]
        a[:, o:o + pl.p[k]] = ck @ U[k].T
    a[:, :pl.p[0]] += mean0[None, :]
    return a


# distance |2 pi c r - R_{k,q}| below which a term of Eq.(IFT_FB) takes its limit
ROOT_GUARD = 1e-8


def eigenimage_radial(pl: Plan, k: int, u: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Radial factor of the real-space steerable principal component with coefficient
    vector u (column u_l^(k) of the eigenvectors) at z = 2 pi c r:

        2 c sqrt(pi) J_k(z) sum_q (-1)^q R_{k,q} u(q) / (z^2 - R_{k,q}^2)

    (the sum over q of Eq.(IFT_FB) with the angular factor left out).  Where z lies within
    ROOT_GUARD of R_{k,q}, J_k(z) / (z^2 - R_{k,q}^2) is replaced by its limit
    -J_{k+1}(z) / (z + R_{k,q}) (J_k(R_{k,q}) = 0 and J_k' = -J_{k+1} there)."""
    z = np.asarray(z, dtype=np.float64)
    jk = special.jv(k, z)
    jk1 = special.jv(k + 1, z)
    acc = np.zeros_like(z)
    for q in range(1, pl.p[k] + 1):
        R = pl.roots[k][q - 1]
        d = z - R
        near = np.abs(d) < ROOT_GUARD
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(near, -jk1 / (z + R), jk / (d * (z + R)))
        acc += ((-1) ** q) * R * u[q - 1] * t
    return 2.0 * pl.c * math.sqrt(math.pi) * acc


def eigenimages(U: list, pl: Plan, k: int, ls) -> np.ndarray:
    """Real-space steerable principal components g^{k,l} on the L x L pixel grid (axis 0 =
    x, axis 1 = y): E^{k,l}(x) = sum_q u_l^(k)(q) F^{-1}(psi_c^{k,q})(x), the linear
    combination of the closed-form inverse transforms of Eq.(IFT_FB) that Sec. VI-B
    evaluates instead of an inverse polar transform, with i^k in the numerator (the
    printed 1/i^k has the wrong sign for odd k).  Complex [len(ls)][L][L]."""
    x = pixel_coords(pl.L)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    z = 2.0 * math.pi * pl.c * np.hypot(X1, X2)
    ang = (1j) ** k * np.exp(1j * k * np.arctan2(X2, X1))
    return np.stack([ang * eigenimage_radial(pl, k, U[k][:, l], z) for l in ls])
