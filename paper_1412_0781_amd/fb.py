"""Python binding of the MI355X Fourier-Bessel steerable PCA library.

Argument marshalling only: every step of the expansion, adjoint, covariance and
eigendecomposition runs in the HIP kernels of libffbspca.so.  torch provides
device memory and the current HIP stream.

Layouts (Sec. II of the paper): images are float32 [n, L, L] with axis 0 = x;
coefficients are float32 [n, p_half, 2] = (Re, Im) of a_{k,q}, k = 0..k_max,
q = 1..p_k, k-major.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import FB_BF16X3, FB_FP32, FBInfo, check, lib

PRECISIONS = {"fp32": FB_FP32, "bf16x3": FB_BF16X3}


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, dtype, shape, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


@dataclass
class CovState:
    """Accumulators of fb_covariance: G (FP64 packed p_k x p_k blocks), S0 (FP64 k = 0 sums of
    a_0 - shift), count; shift (FP32 [p0], filled by fb_covariance_shift from the first call's
    coefficients unless shift_set; None: no shift) and Gi (FP64, the imaginary parts of the
    Hermitian blocks; None: not accumulated)."""
    G: torch.Tensor
    S0: torch.Tensor
    count: int = 0
    shift: torch.Tensor | None = None
    Gi: torch.Tensor | None = None
    shift_set: bool = False


class Plan:
    """A plan for L x L images with band limit c and support radius R (Algorithm 1, steps 1-2).

    device=False builds the host tables only (sizes and index tables can be read
    without a GPU; compute calls then raise)."""

    def __init__(self, L: int, c: float, R: float, device: bool = True):
        h = ctypes.c_void_p()
        fn = lib().fb_plan if device else lib().fb_plan_host
        check(fn(int(L), float(c), float(R), ctypes.byref(h)))
        self._h = h
        info = FBInfo()
        check(lib().fb_plan_info(h, ctypes.byref(info)))
        self.info = info
        self.L, self.c, self.R = info.L, info.c, info.R
        self.n_xi, self.n_theta, self.k_max, self.p0 = info.n_xi, info.n_theta, info.k_max, info.p0
        self.p_half, self.p_total, self.cov_size = info.p_half, info.p_total, info.cov_size
        self.grid_n, self.kernel_w = info.grid_n, info.kernel_w
        K = self.k_max
        self.k = np.zeros(self.p_half, np.int32)
        self.q = np.zeros(self.p_half, np.int32)
        self.p = np.zeros(K + 1, np.int32)
        self.coef_off = np.zeros(K + 2, np.int64)
        self.cov_off = np.zeros(K + 2, np.int64)
        check(lib().fb_plan_tables(h, self.k.ctypes.data, self.q.ctypes.data, self.p.ctypes.data,
                                   self.coef_off.ctypes.data, self.cov_off.ctypes.data))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device else None
        self._ws = None

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().fb_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host tables -----------------------------------------------------------
    def host_tables(self):
        """FP64 roots R_{k,q}, norms N_{k,q}, Gauss-Legendre xi and w, and the radial table [p_half, n_xi]."""
        roots = np.zeros(self.p_half)
        norms = np.zeros(self.p_half)
        xi = np.zeros(self.n_xi)
        w = np.zeros(self.n_xi)
        radial = np.zeros((self.p_half, self.n_xi))
        check(lib().fb_plan_host_tables(self._h, roots.ctypes.data, norms.ctypes.data, xi.ctypes.data,
                                        w.ctypes.data, radial.ctypes.data))
        return roots, norms, xi, w, radial

    # -- workspace -----------------------------------------------------------
    def workspace_bytes(self, batch: int) -> int:
        return int(lib().fb_workspace_bytes(self._h, int(batch), 0))

    def workspace(self, batch: int) -> torch.Tensor:
        need = self.workspace_bytes(batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _ws_for(self, n: int, batch: int | None):
        b = max(1, min(int(n), int(batch) if batch else 2048))
        ws = self.workspace(b)
        return ws, self.workspace_bytes(b)

    # -- compute -----------------------------------------------------------
    def expand(self, images: torch.Tensor, precision="fp32", out: torch.Tensor | None = None,
               batch: int | None = None, weight_mode: int = 1) -> torch.Tensor:
        """a = T* I (Algorithm 1, steps 3-4).  images float32 [n, L, L] -> float32 [n, p_half, 2].
        weight_mode 0 multiplies the k > 0 coefficients by 2 (the +-k fold weight)."""
        n = images.shape[0]
        _need(images, torch.float32, (n, self.L, self.L), "images")
        if out is None:
            out = torch.empty((n, self.p_half, 2), dtype=torch.float32, device=images.device)
        _need(out, torch.float32, (n, self.p_half, 2), "out")
        ws, wsb = self._ws_for(n, batch)
        check(lib().fb_expand_weighted(self._h, images.data_ptr(), n, out.data_ptr(), _prec(precision),
                                       int(weight_mode), ws.data_ptr(), wsb, _stream_ptr(images.device)), self._h)
        return out

    def expand_noalloc(self, images: torch.Tensor, out: torch.Tensor, precision="fp32") -> torch.Tensor:
        """expand() through fb_expand_noalloc: the pass buffers are the library's fixed device
        array, so neither the library nor this call allocates (out must be given)."""
        n = images.shape[0]
        _need(images, torch.float32, (n, self.L, self.L), "images")
        _need(out, torch.float32, (n, self.p_half, 2), "out")
        check(lib().fb_expand_noalloc(self._h, images.data_ptr(), n, out.data_ptr(), _prec(precision),
                                      _stream_ptr(images.device)), self._h)
        return out

    def adjoint(self, coeffs: torch.Tensor, weight_mode: int = 0, out: torch.Tensor | None = None,
                batch: int | None = None, ring_filter: torch.Tensor | None = None) -> torch.Tensor:
        """I = T b: synthesis, the transpose of expand (weight_mode 0: +-k folded; 1: plain transpose).
        ring_filter (float32 [n_xi]) applies a radial Fourier filter H(xi_j) on the way."""
        n = coeffs.shape[0]
        _need(coeffs, torch.float32, (n, self.p_half, 2), "coeffs")
        if out is None:
            out = torch.empty((n, self.L, self.L), dtype=torch.float32, device=coeffs.device)
        _need(out, torch.float32, (n, self.L, self.L), "out")
        ws, wsb = self._ws_for(n, batch)
        if ring_filter is None:
            check(lib().fb_adjoint(self._h, coeffs.data_ptr(), n, out.data_ptr(), int(weight_mode), ws.data_ptr(),
                                   wsb, _stream_ptr(coeffs.device)), self._h)
        else:
            _need(ring_filter, torch.float32, (self.n_xi,), "ring_filter")
            check(lib().fb_adjoint_filtered(self._h, coeffs.data_ptr(), n, out.data_ptr(), int(weight_mode),
                                            ring_filter.data_ptr(), ws.data_ptr(), wsb,
                                            _stream_ptr(coeffs.device)), self._h)
        return out

    # -- estimation of R and c (Sec. VI-C) ---------------------------------------
    def pixel_moments(self, images: torch.Tensor, sum: torch.Tensor | None = None,
                      sumsq: torch.Tensor | None = None):
        """Accumulate per-pixel sums and sums of squares (FP64 [L*L] each); returns (sum, sumsq)."""
        n = images.shape[0]
        _need(images, torch.float32, (n, self.L, self.L), "images")
        dev = images.device
        if sum is None:
            sum = torch.zeros(self.L * self.L, dtype=torch.float64, device=dev)
        if sumsq is None:
            sumsq = torch.zeros(self.L * self.L, dtype=torch.float64, device=dev)
        _need(sum, torch.float64, (self.L * self.L,), "sum")
        _need(sumsq, torch.float64, (self.L * self.L,), "sumsq")
        wsb = int(lib().fb_moments_workspace_bytes(self._h))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        check(lib().fb_pixel_moments(self._h, images.data_ptr(), n, sum.data_ptr(), sumsq.data_ptr(), ws.data_ptr(),
                                     wsb, _stream_ptr(dev)), self._h)
        return sum, sumsq

    def polar_power(self, images: torch.Tensor, pixel_sum: torch.Tensor | None = None, count: int = 0,
                    power: torch.Tensor | None = None, batch: int | None = None) -> torch.Tensor:
        """Accumulate sum_i sum_l |F(I_i - mean)(xi_j, theta_l)|^2 per ring (FP64 [n_xi]); the mean
        image is pixel_sum / count when pixel_sum is given."""
        n = images.shape[0]
        _need(images, torch.float32, (n, self.L, self.L), "images")
        dev = images.device
        if power is None:
            power = torch.zeros(self.n_xi, dtype=torch.float64, device=dev)
        _need(power, torch.float64, (self.n_xi,), "power")
        if pixel_sum is not None:
            _need(pixel_sum, torch.float64, (self.L * self.L,), "pixel_sum")
        b = max(1, min(int(n), int(batch) if batch else 2048))
        wsb = int(lib().fb_polar_power_workspace_bytes(self._h, b))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        check(lib().fb_polar_power(self._h, images.data_ptr(), n,
                                   pixel_sum.data_ptr() if pixel_sum is not None else None, int(count),
                                   power.data_ptr(), ws.data_ptr(), wsb, _stream_ptr(dev)), self._h)
        return power

    def ctf_filter(self, pixel_size: float, lam: float, defocus: float, phase: float, bfactor: float,
                   out: torch.Tensor | None = None) -> torch.Tensor:
        """Eq.(CTFenv) on the plan's rings (float32 [n_xi] on the device), for adjoint(ring_filter=...)."""
        if out is None:
            out = torch.empty(self.n_xi, dtype=torch.float32, device=self.device)
        _need(out, torch.float32, (self.n_xi,), "out")
        check(lib().fb_ctf_filter(self._h, float(pixel_size), float(lam), float(defocus), float(phase),
                                  float(bfactor), out.data_ptr(), _stream_ptr(out.device)), self._h)
        return out

    def estimate_support(self, sum: torch.Tensor, sumsq: torch.Tensor, n: int, power: torch.Tensor,
                         noise_var: float, frac: float = 0.999):
        """(R, c) from the accumulated moments and ring power (the cumulative-fraction rule)."""
        _need(sum, torch.float64, (self.L * self.L,), "sum")
        _need(sumsq, torch.float64, (self.L * self.L,), "sumsq")
        _need(power, torch.float64, (self.n_xi,), "power")
        out = torch.empty(2, dtype=torch.float64, device=sum.device)
        check(lib().fb_estimate_support(self._h, sum.data_ptr(), sumsq.data_ptr(), int(n), power.data_ptr(),
                                        float(noise_var), float(frac), out.data_ptr(), _stream_ptr(sum.device)),
              self._h)
        R, c = out.cpu().tolist()
        return int(R), c

    def new_covariance(self, shift: bool = True, hermitian: bool = False) -> CovState:
        """Zeroed accumulators; shift=True lets the first call centre the k = 0 sums on its
        mean, hermitian=True also accumulates the imaginary parts Gi."""
        dev = self.device
        return CovState(G=torch.zeros(self.cov_size, dtype=torch.float64, device=dev),
                        S0=torch.zeros(self.p0, dtype=torch.float64, device=dev), count=0,
                        shift=torch.zeros(self.p0, dtype=torch.float32, device=dev) if shift else None,
                        Gi=torch.zeros(self.cov_size, dtype=torch.float64, device=dev) if hermitian else None)

    def covariance(self, coeffs: torch.Tensor, state: CovState | None = None, precision="fp32",
                   ws: torch.Tensor | None = None) -> CovState:
        """Accumulate G^(k) += Re(A A^*), the k = 0 sums and, if the state holds Gi,
        Gi^(k) += Im(A A^*) (Eqs.(ck),(ck_0); Eq.(cov) before the real part)."""
        n = coeffs.shape[0]
        _need(coeffs, torch.float32, (n, self.p_half, 2), "coeffs")
        if state is None:
            state = self.new_covariance()
        if n > 0 and state.shift is not None and not state.shift_set:
            check(lib().fb_covariance_shift(self._h, coeffs.data_ptr(), n, state.shift.data_ptr(),
                                            _stream_ptr(coeffs.device)), self._h)
            state.shift_set = True
        cnt = ctypes.c_int64(state.count)
        wsb = int(lib().fb_covariance_workspace_bytes(self._h, n, 1 if state.Gi is not None else 0))
        if ws is None or ws.numel() * ws.element_size() < wsb:
            ws = torch.empty(max(wsb, 8), dtype=torch.uint8, device=coeffs.device)
        check(lib().fb_covariance(self._h, coeffs.data_ptr(), n, state.G.data_ptr(), state.S0.data_ptr(),
                                  state.Gi.data_ptr() if state.Gi is not None else None,
                                  state.shift.data_ptr() if state.shift is not None else None,
                                  ctypes.byref(cnt), _prec(precision), ws.data_ptr(), wsb,
                                  _stream_ptr(coeffs.device)), self._h)
        state.count = int(cnt.value)
        return state

    def covariance_workspace(self, n: int, hermitian: bool = False) -> torch.Tensor:
        wsb = int(lib().fb_covariance_workspace_bytes(self._h, int(n), 1 if hermitian else 0))
        return torch.empty(max(wsb, 8), dtype=torch.uint8, device=self.device)

    def eig(self, state: CovState):
        """Finalise C^(k) and diagonalise (Algorithm 2, steps 1 and 4).

        Returns (evals [p_half], evecs [cov_size], C [cov_size], mean [p0]), FP64 device tensors."""
        dev = state.G.device
        evals = torch.empty(self.p_half, dtype=torch.float64, device=dev)
        evecs = torch.empty(self.cov_size, dtype=torch.float64, device=dev)
        C = torch.empty(self.cov_size, dtype=torch.float64, device=dev)
        mean = torch.empty(self.p0, dtype=torch.float64, device=dev)
        wsb = int(lib().fb_eig_workspace_bytes(self._h))
        ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        check(lib().fb_eig(self._h, state.G.data_ptr(), state.S0.data_ptr(),
                           state.shift.data_ptr() if state.shift is not None else None, state.count, evals.data_ptr(),
                           evecs.data_ptr(), C.data_ptr(), mean.data_ptr(), ws.data_ptr(), wsb,
                           _stream_ptr(dev)), self._h)
        return evals, evecs, C, mean

    def svd_workspace_bytes(self, n: int) -> int:
        return int(lib().fb_svd_workspace_bytes(self._h, int(n)))

    def svd(self, coeffs: torch.Tensor, ws: torch.Tensor | None = None):
        """Principal components by the SVD of the coefficient matrices (Sec. III-C), without
        forming C^(k).  Returns (evals [p_half], evecs [cov_size], mean [p0]), FP64 device
        tensors laid out like eig's."""
        n = coeffs.shape[0]
        _need(coeffs, torch.float32, (n, self.p_half, 2), "coeffs")
        dev = coeffs.device
        evals = torch.empty(self.p_half, dtype=torch.float64, device=dev)
        evecs = torch.empty(self.cov_size, dtype=torch.float64, device=dev)
        mean = torch.empty(self.p0, dtype=torch.float64, device=dev)
        wsb = self.svd_workspace_bytes(n)
        if ws is None or ws.numel() * ws.element_size() < wsb:
            ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        check(lib().fb_svd(self._h, coeffs.data_ptr(), n, evals.data_ptr(), evecs.data_ptr(), mean.data_ptr(),
                           ws.data_ptr(), ws.numel() * ws.element_size(), _stream_ptr(dev)), self._h)
        return evals, evecs, mean

    # -- steerable PCA back end (Algorithm 2 steps 5-6, Sec. V) ------------------
    def spca_select(self, evals: torch.Tensor, count: int, sigma2: float):
        """Components above the Marcenko-Pastur edge per k (Eq.(compselect)) and the coefficient
        filter ell / (ell + sigma2), ell = (lambda - sigma2)_+.  Returns (n_sel int32 [k_max+1],
        weights FP64 [p_half]) on the device."""
        _need(evals, torch.float64, (self.p_half,), "evals")
        n_sel = torch.empty(self.k_max + 1, dtype=torch.int32, device=evals.device)
        w = torch.empty(self.p_half, dtype=torch.float64, device=evals.device)
        check(lib().fb_spca_select(self._h, evals.data_ptr(), int(count), float(sigma2), n_sel.data_ptr(),
                                   w.data_ptr(), _stream_ptr(evals.device)), self._h)
        return n_sel, w

    def spca_coeffs(self, coeffs: torch.Tensor, evecs: torch.Tensor, mean: torch.Tensor) -> torch.Tensor:
        """c_{k,.} = (a_{k,.} - m [k = 0]) U^(k) (Eq.(sPCAcoeff)); float32 [n, p_half, 2]."""
        n = coeffs.shape[0]
        _need(coeffs, torch.float32, (n, self.p_half, 2), "coeffs")
        _need(evecs, torch.float64, (self.cov_size,), "evecs")
        _need(mean, torch.float64, (self.p0,), "mean")
        out = torch.empty_like(coeffs)
        check(lib().fb_spca_coeffs(self._h, coeffs.data_ptr(), n, evecs.data_ptr(), mean.data_ptr(), out.data_ptr(),
                                   _stream_ptr(coeffs.device)), self._h)
        return out

    def spca_reconstruct(self, c: torch.Tensor, evecs: torch.Tensor, mean: torch.Tensor,
                         weights: torch.Tensor | None = None) -> torch.Tensor:
        """a_{k,.} = U^(k) (w_k c_{k,.}) + m [k = 0]; float32 [n, p_half, 2]."""
        n = c.shape[0]
        _need(c, torch.float32, (n, self.p_half, 2), "c")
        _need(evecs, torch.float64, (self.cov_size,), "evecs")
        _need(mean, torch.float64, (self.p0,), "mean")
        if weights is not None:
            _need(weights, torch.float64, (self.p_half,), "weights")
        out = torch.empty_like(c)
        check(lib().fb_spca_reconstruct(self._h, c.data_ptr(), n, evecs.data_ptr(), mean.data_ptr(),
                                        weights.data_ptr() if weights is not None else None, out.data_ptr(),
                                        _stream_ptr(c.device)), self._h)
        return out

    def spca_radial(self, evecs: torch.Tensor) -> torch.Tensor:
        """Radial parts f^{k,l}(xi_j) of the steerable principal components (Eq.(sPCArad)), float32
        [n_xi * p_half]: block k at n_xi * coef_off[k], [n_xi][p_k]."""
        _need(evecs, torch.float64, (self.cov_size,), "evecs")
        f = torch.empty(self.n_xi * self.p_half, dtype=torch.float32, device=evecs.device)
        check(lib().fb_spca_radial(self._h, evecs.data_ptr(), f.data_ptr(), _stream_ptr(evecs.device)), self._h)
        return f

    def eigenimages(self, evecs: torch.Tensor, k: int, l0: int = 0, nl: int | None = None,
                    out: torch.Tensor | None = None) -> torch.Tensor:
        """Real-space steerable principal components l0 .. l0 + nl - 1 of angular frequency k
        on the pixel grid (Eq.(IFT_FB) combinations, Sec. VI-B): complex128 [nl][L][L]."""
        _need(evecs, torch.float64, (self.cov_size,), "evecs")
        if nl is None:
            nl = self.p[k] - l0
        if out is None:
            out = torch.empty((nl, self.L, self.L), dtype=torch.complex128, device=evecs.device)
        if out.dtype != torch.complex128 or tuple(out.shape) != (nl, self.L, self.L) or not out.is_contiguous() \
                or out.device != evecs.device:
            raise ValueError("out must be contiguous complex128 [nl][L][L] on the device of evecs")
        check(lib().fb_eigenimages(self._h, evecs.data_ptr(), int(k), int(l0), int(nl), out.data_ptr(),
                                   _stream_ptr(evecs.device)), self._h)
        return out

    def radial_blocks(self, f: torch.Tensor | np.ndarray):
        return [f[self.n_xi * self.coef_off[k]:self.n_xi * self.coef_off[k + 1]].reshape(self.n_xi, self.p[k])
                for k in range(self.k_max + 1)]

    # -- per-kernel timing ---------------------------------------------------
    def profile(self, enable: bool = True):
        check(lib().fb_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset: bool = True) -> dict:
        """{stage name: (total ms, launches)} of the kernels launched while profiling was on."""
        ms = np.zeros(32)
        n = np.zeros(32, np.int64)
        ns = lib().fb_profile_read(self._h, ms.ctypes.data, n.ctypes.data, 32, 1 if reset else 0)
        if ns < 0:
            check(ns, self._h)
        return {lib().fb_stage_name(s).decode(): (float(ms[s]), int(n[s])) for s in range(ns) if n[s] > 0}

    # -- helpers -----------------------------------------------------------
    def blocks(self, packed: torch.Tensor | np.ndarray):
        """Split a packed [cov_size] array into its p_k x p_k blocks."""
        return [packed[self.cov_off[k]:self.cov_off[k + 1]].reshape(self.p[k], self.p[k])
                for k in range(self.k_max + 1)]

    def to_complex(self, coeffs: torch.Tensor) -> torch.Tensor:
        return torch.view_as_complex(coeffs)


def synth_normals(seed: int, rng_stream: int, first: int, n: int, n_per: int, scale: float = 1.0,
                  device=None) -> torch.Tensor:
    """Philox-4x32-10 + Box-Muller normals on the device, float32 [n, n_per] (seeded inputs)."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((n, n_per), dtype=torch.float32, device=device)
    check(lib().fb_synth_normals(int(seed), int(rng_stream), int(first), int(n), int(n_per), float(scale),
                                 out.data_ptr(), _stream_ptr(device)))
    return out


def synth_words(seed: int, rng_stream: int, first: int, n: int, n_per: int, device=None) -> torch.Tensor:
    device = device or torch.device("cuda", torch.cuda.current_device())
    out = torch.empty((n, n_per), dtype=torch.int32, device=device)
    check(lib().fb_synth_words(int(seed), int(rng_stream), int(first), int(n), int(n_per), out.data_ptr(),
                               _stream_ptr(device)))
    return out


# ----------------------------------------------------------------------------
# autograd
# ----------------------------------------------------------------------------
class FBExpand(torch.autograd.Function):
    """a = T* I with gradient T g (plain transpose, weight 1 for every k; k = 0 imaginary parts ignored)."""

    @staticmethod
    def forward(ctx, images, plan: Plan, precision="fp32"):
        ctx.plan = plan
        return plan.expand(images.contiguous(), precision=precision)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adjoint(g.contiguous(), weight_mode=1), None, None


class FBSynth(torch.autograd.Function):
    """I = T b (+-k folded) with gradient w * (T* g), w = 1 for k = 0 and 2 for k > 0."""

    @staticmethod
    def forward(ctx, coeffs, plan: Plan):
        ctx.plan = plan
        return plan.adjoint(coeffs.contiguous(), weight_mode=0)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.expand(g.contiguous(), precision="fp32", weight_mode=0), None


def fb_expand(images, plan: Plan, precision="fp32"):
    return FBExpand.apply(images, plan, precision)


def fb_synth(coeffs, plan: Plan):
    return FBSynth.apply(coeffs, plan)
