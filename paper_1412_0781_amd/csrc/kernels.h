// Launchers of the gfx950 kernels (all asynchronous on the given stream).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace fb {

// Largest p_k the device eigensolver handles (one workgroup per block C^(k)).
constexpr int EIG_MAX_P = 256;
constexpr int kEigLdsLimit = 152 * 1024;  // dynamic LDS of the one-sided eigendecomposition (its static arrays need ~5 KB more)
hipError_t configure_eig_kernels();

// Raise the dynamic-LDS limit of the FFT kernels (called once per plan upload).
hipError_t configure_kernels();

// Eq.(nufft) for nimg images: images -> polar half-ring samples in bufA (bufB is scratch).
hipError_t launch_forward_nufft(const Plan& pl, const float* images, int nimg, float2* bufA, float2* bufB,
                                hipStream_t st);
// Eq.(1DFFT): polar samples P -> angular spectrum Fh [k][j][image] (complex).
hipError_t launch_forward_angular(const Plan& pl, const float2* P, float2* Fh, int nimg, hipStream_t st);
// Eq.(a): Fh -> coefficients [image][p_half][2].
// weight_mode 0 multiplies the k > 0 coefficients by 2 (the +-k fold), 1 leaves them as they are
hipError_t launch_radial_forward(const Plan& pl, const float2* Fh, float* coeffs, int nimg, int precision,
                                 int weight_mode, hipStream_t st);

// transposes
hipError_t launch_radial_adjoint(const Plan& pl, const float* coeffs, float2* D, int nimg, int weight_mode,
                                 const float* ring_filter, hipStream_t st);
hipError_t launch_adjoint_angular(const Plan& pl, const float2* D, float2* Q, int nimg, hipStream_t st);
// largest pass the adjoint spread takes (its node value offsets are 32-bit)
int64_t spread_max_images(const Plan& pl);
hipError_t launch_adjoint_nufft(const Plan& pl, const float2* Q, int nimg, float2* bufA, float2* bufB,
                                float* images, hipStream_t st);

// Eqs.(ck),(ck_0) accumulation and the k = 0 sums.  The images are split into
// `slices` runs of `per` images; each run's FP64 partial G (and S0) goes to the
// workspace and the runs are then added into G in order.
constexpr int kCovMaxSlices = 16;
constexpr int kCovSliceImages = 4096;  // images per slice at least, until kCovMaxSlices
constexpr int kCovShiftImages = 1024;  // images whose k = 0 mean becomes the shift
struct CovSplit {
  long long per = 0;
  int slices = 0;
  size_t bytes_g = 0;   // slices * cov_size doubles
  size_t bytes_gi = 0;  // the same again for the imaginary parts (Hermitian form), else 0
  size_t bytes = 0;     // + slices * p0 doubles
};
CovSplit cov_split(const Plan& pl, long long n, bool hermitian);
// shift = mean of the k = 0 coefficients of the first min(n, kCovShiftImages) images
hipError_t launch_cov_shift(const Plan& pl, const float* coeffs, long long n, float* shift, hipStream_t st);
// Gi (nullable): accumulate Im(A A^*) too; shift (nullable): FP32 [p_0] subtracted from a_0
hipError_t launch_covariance(const Plan& pl, const float* coeffs, long long n, double* G, double* S0, double* Gi,
                             const float* shift, int precision, void* ws, hipStream_t st);

// Algorithm 2, steps 1 and 4 (FP64).
hipError_t launch_eig(const Plan& pl, const double* G, const double* S0, const float* shift, long long count,
                      double* evals, double* evecs, double* C_out, double* mean_out, double* work, hipStream_t st);
size_t eig_workspace_bytes(const Plan& pl);

// Steerable PCA back end (Algorithm 2 steps 5-6; Sec. V selection and shrinkage).
hipError_t launch_spca_select(const Plan& pl, const double* evals, long long count, double sigma2, int* n_sel,
                              double* weights, hipStream_t st);
// mode 0: c = (a - m) U per k; mode 1: a = U (w c) + m per k (weights may be null only in mode 0)
hipError_t launch_spca_apply(const Plan& pl, int mode, const float* in, long long n, const double* evecs,
                             const double* mean, const double* weights, float* out, hipStream_t st);
hipError_t launch_spca_radial(const Plan& pl, const double* evecs, float* f, hipStream_t st);
// SVD route (Sec. III-C): rows per level-1 workgroup, LDS ceiling of the two SVD kernels.
constexpr int kSvdRowsPerGroup = 8192;
constexpr int kSvdLdsLimit = 160 * 1024 - 1024;
constexpr int kSvdMaxP = 256;  // two threads per column in a workgroup of at most 512 threads
int svd_max_p(const Plan& pl);
struct SvdSplit {
  int W0, W1;                 // level-1 workgroups for k = 0 and for each k > 0
  long long base1;            // doubles of the k = 0 level-1 factors
  long long r_doubles;        // doubles of all level-1 factors
  long long mean_doubles;     // doubles reserved for the k = 0 mean
  long long total_doubles;    // workspace: mean, level-1 factors, p_k x p_k blocks
};
SvdSplit svd_split(const Plan& pl, long long n);
size_t svd_finish_lds_bytes(const Plan& pl);
size_t svd_qr_lds_bytes(const Plan& pl);
hipError_t configure_svd_kernels();
hipError_t launch_svd(const Plan& pl, const float* coeffs, long long n, double* evals, double* evecs,
                      double* mean_out, double* ws, hipStream_t st);
// Estimation of R and c (Sec. VI-C)
constexpr int kMomentSlices = 64;  // image slices of the per-pixel moments
size_t moments_workspace_bytes(const Plan& pl);
hipError_t launch_pixel_moments(const Plan& pl, const float* images, long long n, double* sum, double* sumsq,
                                double* ws, hipStream_t st);
hipError_t launch_mean_image(const Plan& pl, const double* sum, long long count, float* mean, hipStream_t st);
hipError_t launch_polar_power(const Plan& pl, const float2* P, const float2* Pmean, int nimg, double* power,
                              hipStream_t st);
hipError_t launch_copy_polar(const Plan& pl, const float2* P, float2* dst, hipStream_t st);
hipError_t launch_estimate_support(const Plan& pl, const double* sum, const double* sumsq, long long n,
                                   const double* power, double noise_var, double frac, double* out, hipStream_t st);
hipError_t launch_ctf_filter(const Plan& pl, double pixel_size, double lambda, double defocus, double phase,
                             double bfactor, float* filter, hipStream_t st);
hipError_t launch_eigenimages(const Plan& pl, const double* evecs, int k, int l0, int nl, double* out,
                              hipStream_t st);

// seeded inputs
hipError_t launch_synth_normals(unsigned long long seed, unsigned rng_stream, long long first, long long n,
                                long long n_per, float scale, float* out, hipStream_t st);
hipError_t launch_synth_words(unsigned long long seed, unsigned rng_stream, long long first, long long n,
                              long long n_per, unsigned* out, hipStream_t st);

}  // namespace fb
