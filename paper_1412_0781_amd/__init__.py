"""MI355X (gfx950) fast Fourier-Bessel steerable PCA: the per-image Fourier-Bessel
expansion (polar non-uniform FFT, angular FFT, radial quadrature), the steerable
covariance and its eigendecomposition, and the adjoint synthesis, as HIP kernels
behind the C ABI of include/ffbspca.h."""

from .fb import (  # noqa: F401
    FBExpand,
    FBSynth,
    CovState,
    Plan,
    fb_expand,
    fb_synth,
    synth_normals,
    synth_words,
)
from ._lib import FB_BF16X3, FB_FP32, FBError  # noqa: F401
