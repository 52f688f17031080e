/*
 * ffbspca.h - C ABI of the MI355X (gfx950) fast Fourier-Bessel steerable PCA library.
 *
 * Method: Zhao, Shkolnisky, Singer, "Fast Steerable Principal Component
 * Analysis" (arXiv:1412.0781).  The library computes
 *   - the Fourier-Bessel expansion a = T* I of each image (Algorithm 1:
 *     polar Fourier samples Eq.(nufft) by a non-uniform FFT, the angular sum
 *     Eq.(1DFFT) by an FFT on each ring, the radial Gauss-Legendre sum Eq.(a));
 *   - the steerable covariance blocks C^(k) (Eqs.(ck),(ck_0)) with the mean
 *     removed from k = 0 (Algorithm 2, step 1) and their eigenpairs
 *     (Algorithm 2, step 4);
 *   - the adjoint T (synthesis of images from coefficients), the transpose of T*.
 *
 * Conventions (all calls):
 *   images   float32 [n][L][L], C-contiguous, device memory.  Axis 0 is i1 (the
 *            x coordinate), axis 1 is i2 (y); pixel indices run over
 *            -ceil((L-1)/2) .. floor((L-1)/2) (Sec. II).
 *   coeffs   float32 [n][p_half][2] (real, imaginary), device memory: a_{k,q}
 *            for k = 0..k_max, q = 1..p_k, ordered k ascending then q ascending
 *            (a_{-k,q} = conj(a_{k,q}) is implied, Sec. II-B).  The imaginary
 *            part of every k = 0 entry is written as exactly 0.
 *   The polar transform Eq.(nufft) is taken with normalisation 1 (a Riemann
 *   sum of the continuous Fourier transform with unit pixel); the printed
 *   1/(2R)^2 would scale a by 1/(2R)^2 and C, lambda by 1/(2R)^4.
 *
 * Ownership: the library owns a plan and the device tables inside it.  The
 * caller owns every image, coefficient, accumulator and workspace buffer.
 * Compute calls are asynchronous on the given HIP stream, allocate nothing and
 * never synchronise the host.  A plan is immutable once built and may be used
 * from several streams at once, provided the workspaces differ.
 *
 * Errors: every call returns 0 on success or a negative FB_ERR_* code; no
 * exception crosses the ABI.  Argument errors are detected before any work is
 * enqueued.  FB_ERR_HIP means a HIP runtime call failed; fb_plan_last_hip_error
 * returns that HIP error code.
 */
#ifndef FFBSPCA_H
#define FFBSPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fb_plan_s* fb_plan_t;

/* Return codes */
#define FB_OK 0
#define FB_ERR_INVALID_ARG (-1)        /* a size, pointer or parameter is out of range */
#define FB_ERR_ALLOC (-2)              /* host or device allocation failed (plan creation only) */
#define FB_ERR_HIP (-3)                /* a HIP runtime call failed */
#define FB_ERR_UNSUPPORTED (-4)        /* e.g. odd n_theta, FFT length with a prime factor > 31 */
#define FB_ERR_NO_DEVICE (-5)          /* compute call on a plan built with fb_plan_host */
#define FB_ERR_WORKSPACE (-6)          /* workspace too small for even one image */
#define FB_ERR_SCRATCH_LIMIT (-7)      /* fb_expand_noalloc: a pass of 16 images exceeds its fixed scratch */

/* Arithmetic of the two dense contractions (radial quadrature Eq.(a) and covariance Eq.(ck)). */
#define FB_FP32 0    /* FP32 matrix-core products, FP32 accumulation */
#define FB_BF16X3 1  /* split-BF16 operands x = hi + lo, products hi*hi + hi*lo + lo*hi, FP32 accumulation */

typedef struct fb_info {
  int32_t L;          /* image side */
  double c;           /* band limit, 0 < c <= 1/2 (Sec. II) */
  double R;           /* support radius, 0 < R <= L/2 (Sec. II-A) */
  int32_t n_xi;       /* ceil(4 c R), radial Gauss-Legendre nodes (Algorithm 1, step 1) */
  int32_t n_theta;    /* ceil(16 c R), angular nodes per ring (Algorithm 1, step 1) */
  int32_t k_max;      /* largest admissible angular frequency (Eq.(criterion1)) */
  int32_t p0;         /* p_0 */
  int64_t p_half;     /* sum_{k=0}^{k_max} p_k: complex coefficients stored per image */
  int64_t p_total;    /* the paper's p = p_0 + 2 sum_{k>0} p_k (Sec. II-A) */
  int64_t cov_size;   /* sum_k p_k^2: doubles in a packed covariance / eigenvector array */
  int32_t grid_n;     /* side of the oversampled Cartesian grid of the non-uniform FFT */
  int32_t kernel_w;   /* spreading kernel width, in grid points */
  double kernel_beta; /* shape of the Kaiser-Bessel kernel I_0(beta sqrt(1-z^2)) / I_0(beta) */
  int32_t has_device; /* 1 for fb_plan, 0 for fb_plan_host */
} fb_info;

/* Build a plan for L x L images with band limit c and support radius R
 * (Algorithm 1, steps 1-2): the (k,q) selection of Eq.(criterion1), n_xi and
 * n_theta, Gauss-Legendre nodes on [0, c], the radial table
 * N_{k,q} J_k(R_{k,q} xi_j / c) xi_j w_j in FP64 (with FP32 and BF16 hi/lo
 * copies), and the non-uniform FFT tables; uploads them to the current HIP
 * device.  Synchronous.  Errors: FB_ERR_INVALID_ARG if L < 2, c not in
 * (0, 1/2], R not in (0, L/2], or no (k,q) is admissible; FB_ERR_UNSUPPORTED
 * if n_theta is odd or an FFT length has a prime factor above 31. */
int fb_plan(int L, double c, double R, fb_plan_t* out);

/* Same tables, host side only (no HIP call): for inspection of sizes and index
 * tables on a machine without a GPU.  Compute calls on it return FB_ERR_NO_DEVICE. */
int fb_plan_host(int L, double c, double R, fb_plan_t* out);

/* Free a plan and its device tables.  NULL is accepted. */
int fb_plan_destroy(fb_plan_t plan);

/* Sizes of a plan. */
int fb_plan_info(fb_plan_t plan, fb_info* out);

/* Host copies of the index tables (any pointer may be NULL to skip it):
 *   k, q      int32 [p_half]: the (k, q) of each stored coefficient, q from 1
 *   p         int32 [k_max+1]: p_k
 *   coef_off  int64 [k_max+2]: first coefficient of block k (coef_off[k_max+1] = p_half)
 *   cov_off   int64 [k_max+2]: first entry of the p_k x p_k block k in packed arrays */
int fb_plan_tables(fb_plan_t plan, int32_t* k, int32_t* q, int32_t* p, int64_t* coef_off, int64_t* cov_off);

/* Host copies of FP64 tables (NULL skips):
 *   roots   [p_half]  R_{k,q}, the Bessel zeros (Eq.(FB))
 *   norms   [p_half]  N_{k,q} = 1 / (c sqrt(pi) |J_{k+1}(R_{k,q})|)
 *   xi, w   [n_xi]    Gauss-Legendre nodes and weights on [0, c]
 *   radial  [p_half * n_xi]  row (k,q): N_{k,q} J_k(R_{k,q} xi_j / c) xi_j w_j (Eq.(a)) */
int fb_plan_host_tables(fb_plan_t plan, double* roots, double* norms, double* xi, double* w, double* radial);

/* Workspace bytes that make fb_expand / fb_adjoint process up to `batch` images
 * per internal pass (any workspace of at least fb_workspace_bytes(plan, 1, ...)
 * works; larger ones let the library use larger passes).  Pass buffers hold
 * images in groups of 16, so the size is that of ceil(batch / 16) * 16 images. */
size_t fb_workspace_bytes(fb_plan_t plan, int64_t batch, int precision);

/* a = T* I (Algorithm 1, steps 3-4) for n images.  images and coeffs as in
 * the conventions above; ws is device memory of ws_bytes bytes.  Asynchronous
 * on `stream` (a hipStream_t; NULL is the null stream).  n = 0 is a no-op.
 * Errors: FB_ERR_INVALID_ARG (NULL pointer with n > 0, n < 0, bad precision),
 * FB_ERR_WORKSPACE, FB_ERR_NO_DEVICE, FB_ERR_HIP (launch failure). */
int fb_expand(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision,
              void* ws, size_t ws_bytes, void* stream);
/* fb_expand with a weight on the output: weight_mode 1 is fb_expand itself; weight_mode 0
 * multiplies every k > 0 coefficient by 2, the +-k fold weight of the coefficient inner
 * product below (w * T* g is the gradient of the synthesis fb_adjoint with respect to its
 * coefficients; the multiplication is exact).  Same arguments and errors as fb_expand, plus
 * FB_ERR_INVALID_ARG for a weight_mode other than 0 or 1. */
int fb_expand_weighted(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision,
                       int weight_mode, void* ws, size_t ws_bytes, void* stream);

/* fb_expand without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The pass buffers live in a fixed array of FB_NOALLOC_SCRATCH_BYTES bytes inside the
 * library (256 MiB: passes of 112 images at L = 256, 48 at L = 360), one copy per device,
 * loaded with the library and held by each device it runs on until the process ends.
 * Same arguments, layout and result as fb_expand with that array as ws; nothing is
 * allocated (no hipMalloc, hipFree or allocating library call) and nothing needs to be
 * cleared first (every pass writes what it later reads).  Calls on one device share that
 * device's array: two calls that overlap in time on one device (different streams, or
 * different host threads without ordering) race on it and give wrong results; calls
 * ordered on one stream are safe.  The current device must be the plan's device.
 * Errors: those of fb_expand; FB_ERR_SCRATCH_LIMIT (checked first) when one pass of 16 images
 * does not fit the array (above about 16.7 MB of pass buffers per image, e.g. L = 1024, whose
 * oversampled grid side is 2048); FB_ERR_INVALID_ARG also when the plan was built on another
 * device or its per-kernel timer is enabled (the timer creates HIP events). */
#define FB_NOALLOC_SCRATCH_BYTES (256ull << 20)
int fb_expand_noalloc(fb_plan_t plan, const float* images, int64_t n, float* coeffs, int precision, void* stream);

/* Synthesis I = T b, the transpose of fb_expand with respect to the coefficient
 * inner product sum_q b_{0q} c_{0q} + 2 Re sum_{k>0,q} conj(b_{kq}) c_{kq}
 * (the +-k terms folded together, Sec. II-B), i.e.
 *   (T b)(x) = Re sum_{k=-kmax}^{kmax} sum_q b_{kq} conj(M_{kq}(x)),  b_{-k} = conj(b_k),
 * where M_{kq} is row (k,q) of T*.  The imaginary parts of the k = 0 inputs
 * are ignored.  `weight_mode` 0 applies the fold weights (1 for k = 0, 2 for
 * k > 0); 1 applies weight 1 to every k (the plain real transpose of
 * fb_expand, used for gradients).  Asynchronous; same errors as fb_expand. */
int fb_adjoint(fb_plan_t plan, const float* coeffs, int64_t n, float* images, int weight_mode,
               void* ws, size_t ws_bytes, void* stream);
/* fb_adjoint with a radially symmetric Fourier filter: ring_filter (device FP32 [n_xi],
 * nullable = no filter) multiplies the spectrum on ring xi_j by H(xi_j) before the
 * angular and polar steps, i.e. the synthesised image is convolved with the inverse
 * transform of H restricted to the band (the CTF-filtered workload of Sec. VI-C,
 * Eq.(CTFenv), with H evaluated at the plan's xi_j by the caller).  Same errors. */
int fb_adjoint_filtered(fb_plan_t plan, const float* coeffs, int64_t n, float* images, int weight_mode,
                        const float* ring_filter, void* ws, size_t ws_bytes, void* stream);
/* The CTF envelope of Sec. VI-C, Eq.(CTFenv), on the plan's rings:
 *   filter[j] = min(pi lambda z f^2 + a, 1) exp(-B f^2),  f = xi_j / pixel_size,
 * in FP64, stored as FP32 (device [n_xi], caller-owned), for fb_adjoint_filtered.
 * lambda: electron wavelength, z: defocus (both in the units of pixel_size, e.g. Angstrom),
 * a: amplitude contrast phase (rad), B: B-factor (pixel_size units squared).  Asynchronous
 * on `stream`; allocates nothing.  Errors: FB_ERR_INVALID_ARG (NULL filter, pixel_size
 * <= 0, a non-finite parameter), FB_ERR_NO_DEVICE, FB_ERR_HIP. */
int fb_ctf_filter(fb_plan_t plan, double pixel_size, double lambda, double defocus, double phase, double bfactor,
                  float* filter, void* stream);

/* Accumulate the steerable covariance of n coefficient vectors (Eqs.(ck),(ck_0)):
 *   G[cov_off[k] + q p_k + q'] += sum_i Re(b^i_{kq} conj(b^i_{kq'}))  (FP64, full p_k x p_k blocks)
 *   S0[q] += sum_i b^i_{0q}                                          (FP64 [p_0])
 *   Gi[cov_off[k] + q p_k + q'] += sum_i Im(a^i_{kq} conj(a^i_{kq'})) (FP64, nullable; k > 0)
 *   *count += n                                                      (host int64)
 * with b = a, except that the k = 0 coefficients enter as b_{0q} = a_{0q} - shift[q] when
 * `shift` is given.  `shift` (device FP32 [p_0], nullable, read only) keeps the k = 0 sums of
 * the order of the spread of the data instead of its mean, so that the FP32 (or BF16x3)
 * products lose no accuracy to a large mean image.  Any fixed vector near the mean serves
 * (fb_covariance_shift makes one from the first call's images); every call that adds into
 * one G must pass the same values, and fb_eig must receive them too: C^(0) = G^(0)/count -
 * d d^T with d = S0/count does not depend on the shift, and the mean is shift + d.
 * Gi (nullable) accumulates the imaginary part of the Hermitian matrix sum_i a a^* of each
 * k > 0 (the covariance of the data augmented by rotations only, before the reflections of
 * Sec. III make it real; Eq.(cov) without the real part), Im(A A^*) = Ai Ar^T - Ar Ai^T:
 * antisymmetric blocks; the k = 0 block is left unchanged (a_0 is real).  The SO(2)
 * Hermitian covariance is (G + i Gi)/count for k > 0.
 * G, S0 and Gi are device memory owned by the caller (zero them before the first call).
 * The n images are cut into at most 16 runs of consecutive images; within a run, partial
 * sums are formed in FP32 over at most 256 images and added to FP64 in a fixed order, and
 * the runs' FP64 sums are added into G in run order, so results are bitwise reproducible.
 * ws: device scratch of at least fb_covariance_workspace_bytes(plan, n, Gi != NULL) bytes,
 * 8-byte aligned, owned by the caller (contents on entry are ignored).  Asynchronous.
 * precision selects FB_FP32 or FB_BF16X3 products.
 * Errors: FB_ERR_INVALID_ARG (NULL or misaligned pointers, n < 0, *count < 0, bad
 * precision), FB_ERR_WORKSPACE (ws too small), FB_ERR_NO_DEVICE (host-only plan). */
int fb_covariance(fb_plan_t plan, const float* coeffs, int64_t n, double* G, double* S0, double* Gi,
                  const float* shift, int64_t* count, int precision, void* ws, size_t ws_bytes, void* stream);
/* shift[q] = the mean of a^i_{0q} over the first min(n, 1024) of the n coefficient vectors
 * (FP64 sum in image order, rounded to FP32): a shift for fb_covariance.  shift is device
 * FP32 [p_0], caller-owned.  Asynchronous.  Errors: FB_ERR_INVALID_ARG (NULL pointers,
 * n <= 0), FB_ERR_NO_DEVICE, FB_ERR_HIP. */
int fb_covariance_shift(fb_plan_t plan, const float* coeffs, int64_t n, float* shift, void* stream);
/* Scratch bytes fb_covariance needs for n images, with (hermitian != 0) or without the
 * imaginary parts (0 for n <= 0 or a NULL plan). */
size_t fb_covariance_workspace_bytes(fb_plan_t plan, int64_t n, int hermitian);

/* Finalise and diagonalise (Algorithm 2, steps 1 and 4), all FP64 on the device:
 *   d = S0 / count;  C^(0) = G^(0)/count - d d^T;  C^(k) = G^(k)/count (k > 0);
 *   m = shift + d (the k = 0 mean; shift as passed to fb_covariance, NULL meaning 0);
 *   evals [p_half]: eigenvalues of each C^(k), descending within block k (at coef_off[k]);
 *   evecs [cov_size]: block k at cov_off[k], p_k x p_k row-major, column l = u_l,
 *         sign-normalised so that its entry of largest magnitude is positive;
 *   C_out [cov_size] (nullable): the finalised C^(k) blocks;
 *   mean_out [p_0] (nullable): m.
 * ws must hold fb_eig_workspace_bytes(plan) bytes.  When the plan's largest block fits
 * in LDS (max p_k <= 138, p_k^2 + p_k doubles): one-sided Jacobi on the columns of each
 * C^(k) with the rotations accumulated into V, until every column pair is orthogonal to
 * 1e-15 of the product of their norms; eigenvalues are the Rayleigh quotients u_l^T C u_l.
 * Otherwise: cyclic two-sided Jacobi until the off-diagonal norm is below 1e-15 of the
 * block norm.
 * Asynchronous.
 * Errors: FB_ERR_INVALID_ARG if count <= 0 or a required pointer is NULL. */
int fb_eig(fb_plan_t plan, const double* G, const double* S0, const float* shift, int64_t count, double* evals,
           double* evecs, double* C_out, double* mean_out, void* ws, size_t ws_bytes, void* stream);
size_t fb_eig_workspace_bytes(fb_plan_t plan);

/* Steerable PCA back end (Algorithm 2, steps 5-6, and Sec. V), on the eigenpairs of
 * fb_eig.  All arrays are device memory owned by the caller; asynchronous on `stream`.
 *
 * fb_spca_select: component selection of Eq.(compselect) and the coefficient filter.
 *   For each k, component l is selected when lambda_l^(k) > sigma2 (1 + sqrt(gamma_k))^2
 *   with gamma_0 = p_0 / count and gamma_k = p_k / (2 count) (the Marcenko-Pastur edge);
 *   n_sel [k_max + 1] (int32) receives the number selected per k; weights [p_half] (FP64,
 *   at coef_off[k] + l) receives ell / (ell + sigma2), ell = (lambda - sigma2)_+ (the
 *   first-order soft threshold of the eigenvalues), for selected components and 0 for
 *   the others.  evals as written by fb_eig; count = the number of images; sigma2 >= 0
 *   the noise variance (estimated by the caller).
 * fb_spca_coeffs: c^i_{k,l} = sum_q (a^i_{k,q} - m_q [k = 0]) u_l^(k)(q) (Eq.(sPCAcoeff)
 *   with the mean of Algorithm 2 step 1 removed); coeffs and out float32 [n][p_half][2]
 *   (l in place of q, same layout), evecs and mean as written by fb_eig.  FP32 products.
 * fb_spca_reconstruct: a^i_{k,q} = sum_l u_l^(k)(q) w_{k,l} c^i_{k,l} + m_q [k = 0]; weights
 *   nullable (then w = 1, the inverse of fb_spca_coeffs).  With the weights of
 *   fb_spca_select, fb_adjoint of the result gives the denoised images.
 * fb_spca_radial: f^{k,l}(xi_j) = sum_q N_{k,q} J_k(R_{k,q} xi_j / c) u_l^(k)(q)
 *   (Eq.(sPCArad)) at the Gauss-Legendre nodes; f float32, block k at n_xi * coef_off[k],
 *   [n_xi][p_k] row-major.
 * fb_eigenimages: the real-space steerable principal components of Sec. VI-B on the
 *   L x L pixel grid (axis 0 = x, axis 1 = y, pixel coordinates -floor(L/2) ..), as the
 *   linear combinations E^{k,l}(x) = sum_q u_l^(k)(q) F^{-1}(psi_c^{k,q})(x) of the closed
 *   forms of Eq.(IFT_FB) (with i^k in the numerator: the printed 1/i^k has the wrong
 *   sign for odd k), for components l = l0 .. l0 + nl - 1 of angular frequency k.
 *   evecs as written by fb_eig (device, FP64); out device FP64 [nl][L][L][2] (re, im),
 *   caller-owned.  FP64 throughout (Bessel functions by Miller's backward recurrence);
 *   within 1e-8 of a Bessel root the quotient J_k(z)/(z^2 - R^2) takes its limit.
 *   For k > 0, 2 Re E^{k,l} is the image that fb_adjoint gives for the coefficient
 *   vector u_l^(k) placed at k.  nl = 0 is a no-op.
 * Errors: FB_ERR_INVALID_ARG (NULL pointers, in-place out, count <= 0, sigma2 < 0;
 * k outside 0..k_max, l0 < 0, nl < 0 or l0 + nl > p_k), FB_ERR_NO_DEVICE, FB_ERR_HIP. */
int fb_spca_select(fb_plan_t plan, const double* evals, int64_t count, double sigma2, int32_t* n_sel,
                   double* weights, void* stream);
int fb_spca_coeffs(fb_plan_t plan, const float* coeffs, int64_t n, const double* evecs, const double* mean,
                   float* out, void* stream);
int fb_spca_reconstruct(fb_plan_t plan, const float* c, int64_t n, const double* evecs, const double* mean,
                        const double* weights, float* out, void* stream);
int fb_spca_radial(fb_plan_t plan, const double* evecs, float* f, void* stream);
int fb_eigenimages(fb_plan_t plan, const double* evecs, int k, int l0, int nl, double* out, void* stream);

/* Estimation of the support radius R and the band limit c from noisy images (Sec. VI-C).
 * fb_pixel_moments: sum[p] += sum_i I_i(p), sumsq[p] += sum_i I_i(p)^2 (device FP64 [L*L],
 *   caller-owned, zero them first); images device float32 [n][L][L]; ws of at least
 *   fb_moments_workspace_bytes(plan) bytes, 8-byte aligned.  Fixed summation order.
 * fb_polar_power: power[j] += sum_i sum_{l < n_theta/2} |F(I_i - mean)(xi_j, theta_l)|^2
 *   (device FP64 [n_xi], caller-owned; Eq.(nufft) with unit normalisation at the plan's
 *   polar nodes; a plan with c = 1/2 covers the band up to Nyquist).  The mean image is
 *   pixel_sum / count (pixel_sum device FP64 [L*L], e.g. from fb_pixel_moments; NULL: no
 *   subtraction).  ws of at least fb_polar_power_workspace_bytes(plan, batch) bytes.
 * fb_estimate_support: out[0] = R, out[1] = c (device FP64 [2]).  The mean radial variance
 *   v_r averages sumsq/n - (sum/n)^2 over the pixels with round(|x|) = r, r = 0 .. L/2;
 *   R is the smallest r at which sum_{r' <= r} (v_r' - noise_var) r' reaches frac of its
 *   total.  The mean radial power spectrum is p_j = power[j] / (n (n_theta/2) L^2); c is the
 *   smallest xi_j at which sum_{j' <= j} (p_j' - noise_var) xi_j' w_j' reaches frac of its
 *   total (w_j the Gauss-Legendre weights).  One workgroup; FP64, sums in pixel and ring
 *   order.  frac in (0, 1] (the paper's 0.999).
 * Asynchronous on `stream`; allocate nothing.  Errors: FB_ERR_INVALID_ARG (NULL pointers,
 * n < 0 (n <= 0 for the estimate), pixel_sum with count <= 0, frac outside (0, 1],
 * misaligned ws), FB_ERR_WORKSPACE, FB_ERR_NO_DEVICE, FB_ERR_HIP. */
size_t fb_moments_workspace_bytes(fb_plan_t plan);
int fb_pixel_moments(fb_plan_t plan, const float* images, int64_t n, double* sum, double* sumsq, void* ws,
                     size_t ws_bytes, void* stream);
size_t fb_polar_power_workspace_bytes(fb_plan_t plan, int64_t batch);
int fb_polar_power(fb_plan_t plan, const float* images, int64_t n, const double* pixel_sum, int64_t count,
                   double* power, void* ws, size_t ws_bytes, void* stream);
int fb_estimate_support(fb_plan_t plan, const double* sum, const double* sumsq, int64_t n, const double* power,
                        double noise_var, double frac, double* out, void* stream);

/* Principal components by the SVD of the coefficient matrices (Sec. III-C: the left
 * singular vectors of A^(k) in place of the eigenvectors of C^(k), same complexity,
 * better conditioning).  For each k the real matrix X^(k) = [Re A^(k)^T; Im A^(k)^T]
 * (2n x p_k; for k = 0, the n x p_0 matrix A^(0)^T minus the mean of Algorithm 2 step 1)
 * has Gram matrix n C^(k).  The library reduces it to a triangular factor by Householder
 * reflections (tall-skinny QR over row ranges, then a merge per k) and takes the SVD of
 * that factor by one-sided Jacobi sweeps, in FP64 without forming any Gram matrix.
 *   coeffs   device float32 [n][p_half][2] as written by fb_expand (k = 0 imaginary parts
 *            are ignored).
 *   evals    device FP64 [p_half]: lambda_l = sigma_l^2 / n at coef_off[k] + l, descending
 *            within each k (the eigenvalues of C^(k)).
 *   evecs    device FP64 [sum p_k^2], packed like fb_eig's: block k at cov_off[k],
 *            p_k x p_k row-major, column l = the right singular vector for sigma_l, the
 *            entry of largest magnitude positive (lowest index on ties).  A column with
 *            sigma_l = 0 (fewer data rows than p_k) is written as zeros.
 *   mean_out nullable device FP64 [p_0]: the k = 0 mean.
 *   ws       device workspace of at least fb_svd_workspace_bytes(plan, n) bytes,
 *            8-byte aligned, caller-owned (mean, per-range factors, p_k x p_k blocks).
 * Asynchronous on `stream`; allocates nothing.  Errors: FB_ERR_INVALID_ARG (NULL
 * pointers, n <= 0, misaligned ws), FB_ERR_WORKSPACE, FB_ERR_UNSUPPORTED (max p_k above
 * 199: the packed triangular factor of the largest block is kept in LDS; two threads per
 * column, in workgroups of 512 threads when max p_k > 128; blocks whose p_k x p_k rotation
 * matrix does not fit in LDS (p_k > 141) are rotated in global memory), FB_ERR_NO_DEVICE,
 * FB_ERR_HIP. */
size_t fb_svd_workspace_bytes(fb_plan_t plan, int64_t n);
int fb_svd(fb_plan_t plan, const float* coeffs, int64_t n, double* evals, double* evecs, double* mean_out, void* ws,
           size_t ws_bytes, void* stream);

/* Seeded synthetic inputs on the device (not part of the method): Philox-4x32-10
 * (Salmon et al., SC'11) words with counter (word_block, index_lo, index_hi,
 * stream) and key (seed_lo, seed_hi), Box-Muller normals on word pairs.
 *   fb_synth_normals: out[i][t] = scale * z_t(seed, stream, first_index + i), t < n_per
 *   fb_synth_words:   out[i][t] = 32-bit word t of image first_index + i
 * Asynchronous on `stream` (the HIP stream); `rng_stream` is the Philox stream id. */
int fb_synth_normals(uint64_t seed, uint32_t rng_stream, int64_t first_index, int64_t n, int64_t n_per,
                     float scale, float* out, void* stream);
int fb_synth_words(uint64_t seed, uint32_t rng_stream, int64_t first_index, int64_t n, int64_t n_per,
                   uint32_t* out, void* stream);

/* Per-kernel timing (instrumentation, not part of the method).  While enabled,
 * the library records a pair of HIP events on the caller's stream around every
 * kernel it launches for this plan.  fb_profile_read waits for the recorded
 * events, adds their elapsed times to per-stage totals and returns, for stage
 * s < min(max_stages, FB_NUM_STAGES): total_ms[s] (milliseconds summed over
 * launches) and launches[s]; reset = 1 clears the totals afterwards.  Returns
 * the number of stages (FB_NUM_STAGES) or a negative FB_ERR_* code.  Stage
 * names come from fb_stage_name.  Not for concurrent use of one plan from
 * several streams while enabled. */
#define FB_NUM_STAGES 15
int fb_profile_enable(fb_plan_t plan, int enable);
int fb_profile_read(fb_plan_t plan, double* total_ms, int64_t* launches, int max_stages, int reset);
const char* fb_stage_name(int stage);

/* Human-readable text for a return code. */
const char* fb_error_string(int code);

/* HIP error code of the last failing HIP call made for this plan (0 if none). */
int fb_plan_last_hip_error(fb_plan_t plan);

#ifdef __cplusplus
}
#endif
#endif /* FFBSPCA_H */
