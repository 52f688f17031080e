"""Plain FP64 restatement of Algorithms 1 and 2 of the paper (test oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

Conventions (Sec. II):
  * images are real arrays [n][L][L]; axis 0 is i1 (x), axis 1 is i2 (y), and
    pixel indices run over -ceil((L-1)/2) .. floor((L-1)/2);
  * coefficients are complex arrays [n][p_half] holding a_{k,q} for k >= 0,
    ordered k ascending then q ascending (a_{-k,q} = conj(a_{k,q}), Sec. II-B);
  * the polar Fourier samples use normalisation 1 (see the package docstring).

Nothing here is blocked, fused or reordered beyond what the equations state:
the polar transform is the direct double sum of Eq.(nufft) (no FFT), the
angular step is the explicit sum of Eq.(1DFFT) (no FFT), and the radial step is
the explicit Gauss-Legendre sum of Eq.(a).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
from scipy import special

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# Sec. II: pixel grid
# ----------------------------------------------------------------------------
def pixel_coords(L: int) -> np.ndarray:
    """Pixel indices i = -ceil((L-1)/2), ..., floor((L-1)/2) (Sec. II, unit pixel)."""
    lo = -math.ceil((L - 1) / 2)
    return np.arange(lo, lo + L, dtype=np.float64)


# ----------------------------------------------------------------------------
# Algorithm 1, steps 1-2 (precomputation)
# ----------------------------------------------------------------------------
@dataclass(repr=False)
class Plan:
    L: int
    c: float
    R: float
    n_xi: int
    n_theta: int
    k_max: int
    p: list                      # p_k for k = 0..k_max
    roots: list                  # roots[k] = R_{k,1..p_k}
    norms: list                  # norms[k] = N_{k,1..p_k}   (Eq.(FB))
    xi: np.ndarray               # Gauss-Legendre nodes on [0, c]
    w: np.ndarray                # Gauss-Legendre weights on [0, c]
    theta: np.ndarray            # 2*pi*l/n_theta
    coef_off: np.ndarray = field(default=None)   # start of block k in the coefficient vector
    kq: np.ndarray = field(default=None)         # [p_half, 2] table of (k, q), q 1-based
    _B: list = field(default=None, repr=False)

    @property
    def B(self) -> list:
        """B[k][q, j] = N_{k,q} J_k(R_{k,q} xi_j / c) xi_j w_j, the radial weights of Eq.(a).

        Evaluated on first use (Algorithm 1, step 2)."""
        if self._B is None:
            self._B = [self.norms[k][:, None]
                       * special.jv(k, np.outer(self.roots[k], self.xi) / self.c)
                       * (self.xi * self.w)[None, :]
                       for k in range(self.k_max + 1)]
        return self._B

    def __repr__(self) -> str:
        return (f"Plan(L={self.L}, c={self.c}, R={self.R}, n_xi={self.n_xi}, "
                f"n_theta={self.n_theta}, k_max={self.k_max}, p_half={self.p_half})")

    @property
    def p_half(self) -> int:
        return int(sum(self.p))

    @property
    def p_total(self) -> int:
        """The paper's p = sum over k = -k_max..k_max of p_k (Sec. II-A)."""
        return int(self.p[0] + 2 * sum(self.p[1:]))


def _bessel_zeros_upto(k: int, bound: float) -> np.ndarray:
    """All positive zeros of J_k that are <= bound (scipy's tabulated root finder)."""
    m = max(2, int((bound - k) / math.pi) + 3)
    while True:
        z = special.jn_zeros(k, m)
        if z[-1] > bound:
            return z[: int(np.searchsorted(z, bound, side="right"))]
        m += 4


def plan(L: int, c: float, R: float) -> Plan:
    """Precomputation of Algorithm 1 (steps 1-2).

    * (k, q) selection by the sampling criterion Eq.(criterion1):
      R_{k,q+1} <= 2 pi c R, so p_k = (number of zeros of J_k <= 2 pi c R) - 1;
    * n_xi = ceil(4cR), n_theta = ceil(16cR) (Algorithm 1, step 1);
    * Gauss-Legendre nodes and weights on [0, c] (Eq.(a));
    * N_{k,q} = 1 / (c sqrt(pi) |J_{k+1}(R_{k,q})|) (Eq.(FB)).
    """
    if not (L >= 2):
        raise ValueError("L must be >= 2")
    if not (0.0 < c <= 0.5):
        raise ValueError("band limit c must satisfy 0 < c <= 1/2 (Sec. II)")
    if not (0.0 < R <= L / 2.0):
        raise ValueError("support radius R must satisfy 0 < R <= L/2")
    n_xi = int(math.ceil(4 * c * R))
    n_theta = int(math.ceil(16 * c * R))
    bound = 2 * math.pi * c * R

    p, roots, norms = [], [], []
    k = 0
    while True:
        z = _bessel_zeros_upto(k, bound)
        pk = len(z) - 1                      # q = 1..p_k have R_{k,q+1} <= bound (criterion1)
        if pk < 1:
            break
        p.append(pk)
        rk = z[:pk]
        roots.append(rk)
        norms.append(1.0 / (c * math.sqrt(math.pi) * np.abs(special.jv(k + 1, rk))))
        k += 1
    if not p:
        raise ValueError("no (k, q) satisfies the sampling criterion for this (c, R)")
    k_max = len(p) - 1

    x, wgl = np.polynomial.legendre.leggauss(n_xi)
    xi = c * (x + 1.0) / 2.0
    w = (c / 2.0) * wgl
    theta = TWO_PI * np.arange(n_theta) / n_theta

    off = np.zeros(k_max + 2, dtype=np.int64)
    off[1:] = np.cumsum(p)
    kq = np.array([(k, q + 1) for k in range(k_max + 1) for q in range(p[k])], dtype=np.int64)
    return Plan(L=L, c=c, R=R, n_xi=n_xi, n_theta=n_theta, k_max=k_max, p=p,
                roots=roots, norms=norms, xi=xi, w=w, theta=theta,
                coef_off=off, kq=kq)


# ----------------------------------------------------------------------------
# Algorithm 1, step 3: polar Fourier samples, Eq.(nufft), evaluated directly
# ----------------------------------------------------------------------------
def polar_nodes(pl: Plan):
    """Cartesian frequencies of the polar quadrature nodes (Sec. II-B), shape [n_xi, n_theta]."""
    xi1 = pl.xi[:, None] * np.cos(pl.theta)[None, :]
    xi2 = pl.xi[:, None] * np.sin(pl.theta)[None, :]
    return xi1, xi2


def nudft_polar(images: np.ndarray, pl: Plan, node_block: int = 4096) -> np.ndarray:
    """F(I)(xi_j, theta_l) = sum_{i1,i2} I(i1,i2) exp(-2 pi i (xi1 i1 + xi2 i2)).

    Eq.(nufft) with normalisation 1 and the sum over the full L x L grid.
    Returns complex128 [n, n_xi, n_theta] (full rings, l = 0..n_theta-1).
    The double sum is split into its two one-dimensional exponentials, which
    is the same sum written as two matrix products.
    """
    images = np.asarray(images, dtype=np.float64)
    n = images.shape[0]
    x = pixel_coords(pl.L)
    xi1, xi2 = polar_nodes(pl)
    xi1 = xi1.ravel()
    xi2 = xi2.ravel()
    out = np.empty((n, xi1.size), dtype=np.complex128)
    for s in range(0, xi1.size, node_block):
        e1 = np.exp(-1j * TWO_PI * np.outer(xi1[s:s + node_block], x))   # [nb, L] over i1
        e2 = np.exp(-1j * TWO_PI * np.outer(xi2[s:s + node_block], x))   # [nb, L] over i2
        t = images @ e2.T                                                # [n, L(i1), nb]
        out[:, s:s + node_block] = np.einsum("bi,nib->nb", e1, t)
    return out.reshape(n, pl.n_xi, pl.n_theta)


def nudft_polar_sparse(pixels, pl: Plan) -> np.ndarray:
    """Eq.(nufft) for images given by their nonzero pixels.

    pixels: a list with one entry per image, each a tuple (r, c, v) of equal-length
    arrays: array row index r (axis 0, i1), column index c (axis 1, i2) and value v.
    Every other pixel is zero, so the double sum over the L x L grid reduces to the
    sum over the listed pixels; it is evaluated term by term.  Returns complex128
    [n, n_xi, n_theta] like nudft_polar.
    """
    x = pixel_coords(pl.L)
    xi1, xi2 = polar_nodes(pl)
    out = np.zeros((len(pixels), pl.n_xi, pl.n_theta), dtype=np.complex128)
    for i, (r, c, v) in enumerate(pixels):
        for rr, cc, vv in zip(np.asarray(r), np.asarray(c), np.asarray(v, dtype=np.float64)):
            out[i] += vv * np.exp(-1j * TWO_PI * (xi1 * x[rr] + xi2 * x[cc]))
    return out


# ----------------------------------------------------------------------------
# Algorithm 1, step 4: Eq.(1DFFT) then Eq.(a)
# ----------------------------------------------------------------------------
def angular_dft(F: np.ndarray, pl: Plan) -> np.ndarray:
    """Fhat(xi_j, k) = (2 pi / n_theta) sum_l F(xi_j, theta_l) exp(-2 pi i k l / n_theta).

    Eq.(1DFFT) as an explicit sum, for k = 0..k_max.  Returns [n, n_xi, k_max+1].
    """
    l = np.arange(pl.n_theta)
    k = np.arange(pl.k_max + 1)
    phase = (np.outer(l, k) % pl.n_theta) / pl.n_theta
    W = np.exp(-1j * TWO_PI * phase)                                     # [n_theta, K+1]
    return (TWO_PI / pl.n_theta) * (F @ W)


def radial_quadrature(Fhat: np.ndarray, pl: Plan) -> np.ndarray:
    """a_{k,q} = sum_j N_{k,q} J_k(R_{k,q} xi_j / c) Fhat(xi_j, k) xi_j w_j  (Eq.(a)).

    For real images a_{0,q} is real (Sec. II-B); its imaginary part, which is
    rounding only, is checked and set to zero.
    """
    n = Fhat.shape[0]
    a = np.empty((n, pl.p_half), dtype=np.complex128)
    for k in range(pl.k_max + 1):
        o = pl.coef_off[k]
        a[:, o:o + pl.p[k]] = Fhat[:, :, k] @ pl.B[k].T
    o0 = pl.p[0]
    scale = max(1.0, float(np.abs(a).max(initial=0.0)))
    if np.abs(a[:, :o0].imag).max(initial=0.0) > 1e-9 * scale:
        raise AssertionError("a_{0,q} has a non-negligible imaginary part: input not real?")
    a[:, :o0] = a[:, :o0].real
    return a


def expand_stages(images: np.ndarray, pl: Plan):
    """Algorithm 1 for a small batch, returning every intermediate (F, Fhat, a)."""
    F = nudft_polar(images, pl)
    Fh = angular_dft(F, pl)
    a = radial_quadrature(Fh, pl)
    return F, Fh, a


def expand(images: np.ndarray, pl: Plan, chunk: int = 64) -> np.ndarray:
    """a = T* I (Eq.(transf)): Algorithm 1 applied image by image (chunked for memory)."""
    images = np.asarray(images, dtype=np.float64)
    out = np.empty((images.shape[0], pl.p_half), dtype=np.complex128)
    for s in range(0, images.shape[0], chunk):
        out[s:s + chunk] = radial_quadrature(angular_dft(nudft_polar(images[s:s + chunk], pl), pl), pl)
    return out


def expand_sparse(pixels, pl: Plan) -> np.ndarray:
    """a = T* I for images given by their nonzero pixels (see nudft_polar_sparse)."""
    out = np.empty((len(pixels), pl.p_half), dtype=np.complex128)
    for i in range(len(pixels)):
        out[i:i + 1] = radial_quadrature(angular_dft(nudft_polar_sparse(pixels[i:i + 1], pl), pl), pl)
    return out


def expand_pixel_combinations(weights: np.ndarray, rows, cols, pl: Plan) -> np.ndarray:
    """a = T* I for the images I_i = sum_d weights[i, d] delta_d, delta_d the image with a single
    1 at pixel (rows[d], cols[d]) and 0 elsewhere.

    Every step of Algorithm 1 (Eqs.(nufft),(1DFFT),(a)) is linear in the image, so the
    expansion of such an image is the same combination of the expansions of the delta
    images, which `expand_sparse` evaluates term by term.  weights: real [n, D]; returns
    complex128 [n, p_half]."""
    weights = np.asarray(weights, dtype=np.float64)
    deltas = [(np.array([r]), np.array([c]), np.array([1.0])) for r, c in zip(rows, cols)]
    basis = expand_sparse(deltas, pl)                                    # [D, p_half]
    return weights @ basis


# ----------------------------------------------------------------------------
# Algorithm 2, steps 1, 3, 4
# ----------------------------------------------------------------------------
def mean_and_covariance(a: np.ndarray, pl: Plan):
    """Mean of the k = 0 coefficients and the blocks C^(k).

    Algorithm 2 step 1: a_mean_{0,q} = (1/n) sum_i a^i_{0,q}, subtracted from k = 0 only.
    Eq.(ck_0): C^(0) = (1/n) A^(0) A^(0)^T.  Eq.(ck): C^(k) = (1/n) Re{A^(k) A^(k)^*}.
    """
    n = a.shape[0]
    p0 = pl.p[0]
    mean0 = a[:, :p0].real.mean(axis=0)
    C = []
    for k in range(pl.k_max + 1):
        o = pl.coef_off[k]
        A = a[:, o:o + pl.p[k]].T                                       # p_k x n
        if k == 0:
            A0 = A.real - mean0[:, None]
            C.append(A0 @ A0.T / n)
        else:
            C.append((A @ A.conj().T).real / n)
    return mean0, C


def hermitian_covariance(a: np.ndarray, pl: Plan):
    """Blocks of the covariance of the data augmented by rotations only (Sec. III: Eq.(cov)
    before the reflections make it real): C_H^(k) = (1/n) A^(k) A^(k)^*, complex Hermitian,
    for k > 0, and C^(0) as in `mean_and_covariance` for k = 0 (the mean removed; real).
    Its real part is the C^(k) of Eq.(ck); its imaginary part is (1/n)(Ai Ar^T - Ar Ai^T)."""
    n = a.shape[0]
    mean0, C = mean_and_covariance(a, pl)
    out = [C[0].astype(np.complex128)]
    for k in range(1, pl.k_max + 1):
        o = pl.coef_off[k]
        A = a[:, o:o + pl.p[k]].T
        out.append(A @ A.conj().T / n)
    return mean0, out


def covariance_blocks(a: np.ndarray, pl: Plan):
    return mean_and_covariance(a, pl)[1]


def eig_blocks(C: list):
    """Eigenpairs of each C^(k), eigenvalues descending (Algorithm 2, step 4).

    Eigenvectors are columns, sign-normalised so that the entry of largest
    magnitude is positive (lowest index on ties).
    """
    lam, U = [], []
    for Ck in C:
        wv, V = np.linalg.eigh(Ck)
        order = np.argsort(-wv, kind="stable")
        wv = wv[order]
        V = V[:, order]
        for col in range(V.shape[1]):
            i = int(np.argmax(np.abs(V[:, col])))
            if V[i, col] < 0:
                V[:, col] = -V[:, col]
        lam.append(wv)
        U.append(V)
    return lam, U


def coefficient_rows(a: np.ndarray, pl: Plan, k: int, mean0: np.ndarray | None = None) -> np.ndarray:
    """The real data matrix of angular frequency k whose Gram matrix is n C^(k): for k > 0
    the rows are Re a^i_{k,.} (i = 1..n) followed by Im a^i_{k,.}, so that
    X^T X = Re(A^(k) A^(k)*) (Eq.(ck)); for k = 0 the rows are a^i_{0,.} - mean (Eq.(ck_0)
    with the mean of Algorithm 2, step 1)."""
    o = pl.coef_off[k]
    A = a[:, o:o + pl.p[k]]
    if k == 0:
        m = A.real.mean(axis=0) if mean0 is None else mean0
        return A.real - m[None, :]
    return np.concatenate([A.real, A.imag], axis=0)


def svd_blocks(a: np.ndarray, pl: Plan):
    """Principal components from the SVD of the coefficient matrices (Sec. III-C: the left
    singular vectors of A^(k), taken here as the right singular vectors of the real row
    matrix X^(k) = [Re A^(k)^T; Im A^(k)^T], whose Gram matrix is n C^(k)), by LAPACK's SVD.
    Eigenvalues of C^(k) are sigma^2 / n, descending; vectors sign-normalised as in
    eig_blocks.  Returns (mean0, lam, U) like mean_and_covariance + eig_blocks."""
    n = a.shape[0]
    mean0 = a[:, :pl.p[0]].real.mean(axis=0)
    lam, U = [], []
    for k in range(pl.k_max + 1):
        X = coefficient_rows(a, pl, k, mean0)
        _, s, Vt = np.linalg.svd(X, full_matrices=False)
        V = Vt.T.copy()
        for col in range(V.shape[1]):
            i = int(np.argmax(np.abs(V[:, col])))
            if V[i, col] < 0:
                V[:, col] = -V[:, col]
        lam.append(s ** 2 / n)
        U.append(V)
    return mean0, lam, U


# ----------------------------------------------------------------------------
# The adjoint T of T* (Eq.(transf)), used for synthesis and differentiation
# ----------------------------------------------------------------------------
def coeff_inner(a: np.ndarray, b: np.ndarray, pl: Plan) -> np.ndarray:
    """<a, b> over all k = -k_max..k_max with a_{-k} = conj(a_k) (Sec. II-B):
    sum_q a_{0q} b_{0q} + 2 Re sum_{k>0,q} conj(a_{kq}) b_{kq}, per image."""
    p0 = pl.p[0]
    s0 = np.sum((np.conj(a[..., :p0]) * b[..., :p0]).real, axis=-1)
    s1 = np.sum((np.conj(a[..., p0:]) * b[..., p0:]).real, axis=-1)
    return s0 + 2.0 * s1


def adjoint_polar(b: np.ndarray, pl: Plan, ring_filter=None) -> np.ndarray:
    """The transposes of Eq.(a) and Eq.(1DFFT) applied to coefficients b: the values on the
    polar nodes, complex128 [n, n_xi * n_theta] (rings outer), that the type-1 sum of
    ``adjoint`` takes to pixels.  Folding +-k gives weight 1 for k = 0 and 2 for k > 0;
    ring_filter as in ``adjoint``."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    K = pl.k_max
    D = np.zeros((n, pl.n_xi, K + 1), dtype=np.complex128)
    for k in range(K + 1):
        o = pl.coef_off[k]
        wk = 1.0 if k == 0 else 2.0
        D[:, :, k] = wk * (b[:, o:o + pl.p[k]] @ pl.B[k])              # sum_q B_qj b_kq
    if ring_filter is not None:
        D *= np.asarray(ring_filter, dtype=np.float64)[None, :, None]
    l = np.arange(pl.n_theta)
    kk = np.arange(K + 1)
    phase = (np.outer(l, kk) % pl.n_theta) / pl.n_theta
    Wp = np.exp(+1j * TWO_PI * phase)                                    # [n_theta, K+1]
    P = (TWO_PI / pl.n_theta) * (D @ Wp.T)                               # [n, n_xi, n_theta]: sum over k
    return P.reshape(n, -1)


def adjoint(b: np.ndarray, pl: Plan, node_block: int = 4096, ring_filter=None) -> np.ndarray:
    """(T b)(x) = Re sum_{k=-kmax..kmax} sum_q b_{kq} conj(M_{kq}(x)), with b_{-k} = conj(b_k).

    M_{kq}(x) is the row of T* for coefficient (k, q): Eq.(nufft), Eq.(1DFFT)
    and Eq.(a) composed.  Folding +-k gives weight 1 for k = 0 and 2 for k > 0.
    Computed as the transpose of each step in turn: the radial sum, the angular
    sum, then the direct type-1 sum over the polar nodes.

    ring_filter (optional, [n_xi]) multiplies the spectrum on ring j by H(xi_j) after the
    radial sum: the image of a radially symmetric Fourier filter H applied to the
    band-limited synthesis (the convolution of Sec. VI-C's CTF workload).
    """
    P = adjoint_polar(b, pl, ring_filter)
    n = P.shape[0]
    x = pixel_coords(pl.L)
    xi1, xi2 = polar_nodes(pl)
    xi1 = xi1.ravel()
    xi2 = xi2.ravel()
    out = np.zeros((n, pl.L, pl.L), dtype=np.float64)
    for s in range(0, xi1.size, node_block):
        e1 = np.exp(+1j * TWO_PI * np.outer(xi1[s:s + node_block], x))  # [nb, L] over i1
        e2 = np.exp(+1j * TWO_PI * np.outer(xi2[s:s + node_block], x))  # [nb, L] over i2
        for i in range(n):
            # sum over the nodes b of e1[b, i1] P[b] e2[b, i2], as one matrix product
            out[i] += ((e1 * P[i, s:s + node_block, None]).T @ e2).real
    return out


def adjoint_pixels(b: np.ndarray, pl: Plan, rows, cols) -> np.ndarray:
    """The same (T b)(x) as ``adjoint``, evaluated only at the pixels (rows[t], cols[t])
    (array indices, axis 0 then axis 1): the type-1 sum over every polar node, term by
    node, at each listed pixel.  Returns float64 [n, len(rows)]."""
    P = adjoint_polar(b, pl)
    x = pixel_coords(pl.L)
    xi1, xi2 = polar_nodes(pl)
    xi1 = xi1.ravel()
    xi2 = xi2.ravel()
    out = np.empty((P.shape[0], len(rows)), dtype=np.float64)
    for t, (r, c) in enumerate(zip(rows, cols)):
        e = np.exp(+1j * TWO_PI * (xi1 * x[r] + xi2 * x[c]))            # [nodes]
        out[:, t] = (P @ e).real
    return out
