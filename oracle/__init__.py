"""FP64 CPU oracle for the fast Fourier-Bessel expansion and steerable covariance.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the paper (Zhao, Shkolnisky, Singer, "Fast Steerable
Principal Component Analysis", arXiv:1412.0781) computes.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and this package never imports the
product.  The two share no code, tables or constants.

Every function states the passage of the paper it follows.  Where the paper is
silent or garbled the reading taken is stated beside the code (and listed in
the design notes of the repository):

* The normalisation of the polar Fourier transform Eq.(nufft) is taken as 1
  (a Riemann sum of the continuous transform with unit pixel), not the printed
  1/(2R)^2, because only s = 1 makes T*T close to the identity as Sec. II-B and
  the Marcenko-Pastur statements of Sec. V require.
* The double sum of Eq.(nufft) runs over the whole L x L grid of Sec. II.
* Array axis 0 is i1 (the x coordinate), axis 1 is i2 (y).
* Eq.(IFT_FB) is used with i^{+k} in the numerator (the printed 1/i^k has the
  wrong sign for odd k; the Jacobi-Anger expansion fixes it).
* The covariance normaliser is 1/n (Eq.(cov)), the mean is removed from k = 0
  only (Algorithm 2, step 1), and eigenvectors are sign-normalised so that the
  entry of largest magnitude is positive (lowest index on ties).

Parity status: every function here is pinned by a test that does not re-type
its formula (see ``tests/test_oracle_*.py``).
"""

from .fb import (  # noqa: F401
    Plan,
    plan,
    pixel_coords,
    polar_nodes,
    nudft_polar,
    nudft_polar_sparse,
    angular_dft,
    radial_quadrature,
    expand,
    expand_sparse,
    expand_pixel_combinations,
    expand_stages,
    hermitian_covariance,
    mean_and_covariance,
    covariance_blocks,
    eig_blocks,
    coefficient_rows,
    svd_blocks,
    adjoint,
    adjoint_polar,
    adjoint_pixels,
    coeff_inner,
)
from . import spca  # noqa: F401,E402
from . import estimate  # noqa: F401,E402
