// Estimation of the support radius R and the band limit c from a set of noisy images
// (Sec. VI-C): the per-pixel variance of the mean-subtracted images averaged over
// integer-radius bins (the mean radial variance), and the power of the mean-subtracted
// images on the polar rings of a plan (the mean radial power spectrum); after the noise
// variance is subtracted, R and c are where the cumulative variance (weight r dr) and the
// cumulative power (weight xi dxi, the Gauss-Legendre weights of the rings) reach a given
// fraction of their totals.  The ring power comes from the polar samples of the NUFFT
// (Eq.(nufft) with unit normalisation), so white noise of variance sigma^2 has
// E|F|^2 / L^2 = sigma^2 on every ring.  All sums are FP64 in a fixed order.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fb {

// partial per-pixel sums over image slices: part[s][p] = sum_i I_i(p), part[S + s][p] =
// sum_i I_i(p)^2 over slice s (images [s per, (s + 1) per)), images in order
__global__ __launch_bounds__(256) void k_pixel_moments_part(const float* __restrict__ img, long long n, int npix,
                                                           long long per, double* __restrict__ part) {
  const int p = blockIdx.x * 256 + threadIdx.x, s = blockIdx.y, S = gridDim.y;
  if (p >= npix) return;
  const long long i0 = (long long)s * per, i1 = min(n, i0 + per);
  double a = 0.0, b = 0.0;
#pragma unroll 8
  for (long long i = i0; i < i1; ++i) {
    const double v = (double)img[i * npix + p];
    a += v;
    b = fma(v, v, b);
  }
  part[(size_t)s * npix + p] = a;
  part[((size_t)S + s) * npix + p] = b;
}

// sum[p] += sum_s part[s][p], sumsq[p] += sum_s part[S + s][p], slices in order
__global__ __launch_bounds__(256) void k_pixel_moments_reduce(const double* __restrict__ part, int npix, int S,
                                                             double* __restrict__ sum, double* __restrict__ sumsq) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  double a = 0.0, b = 0.0;
  for (int s = 0; s < S; ++s) {
    a += part[(size_t)s * npix + p];
    b += part[((size_t)S + s) * npix + p];
  }
  sum[p] += a;
  sumsq[p] += b;
}

__global__ __launch_bounds__(256) void k_mean_image(const double* __restrict__ sum, long long count, int npix,
                                                   float* __restrict__ mean) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < npix) mean[p] = (float)(sum[p] / (double)count);
}

// one image's polar samples P [n_xi][1][H][16] (slot 0) -> dst [n_xi][H]
__global__ __launch_bounds__(256) void k_copy_polar(const float2* __restrict__ P, int total, float2* __restrict__ dst) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < total) dst[e] = P[(size_t)e * kImgGroup];
}

// power[j] += sum over the images of the pass and the angles l < H of |P - Pmean|^2 (one
// workgroup per ring, fixed order: lane-strided sums, then a tree)
__global__ __launch_bounds__(256) void k_polar_power(const float2* __restrict__ P, const float2* __restrict__ Pmean,
                                                    int H, int nimg, int ngrp, double* __restrict__ power) {
  __shared__ double s[256];
  const int j = blockIdx.x;
  const float2* Pj = P + (size_t)j * ngrp * H * kImgGroup;
  const long long tot = (long long)ngrp * H * kImgGroup;
  double acc = 0.0;
  for (long long e = threadIdx.x; e < tot; e += 256) {
    const int slot = (int)(e & (kImgGroup - 1));
    const long long gl = e >> 4;
    const int grp = (int)(gl / H), l = (int)(gl - (long long)grp * H);
    if (grp * kImgGroup + slot >= nimg) continue;
    float2 v = Pj[e];
    double dx = v.x, dy = v.y;
    if (Pmean) {
      const float2 m = Pmean[(size_t)j * H + l];
      dx -= m.x;
      dy -= m.y;
    }
    acc += dx * dx + dy * dy;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) power[j] += s[0];
}

// R and c by the cumulative-fraction rule; out[0] = R (pixels), out[1] = c.  Bin b of the
// radial variance collects the pixels with round(|x|) = b, b = 0 .. L/2, in pixel order;
// products and sums are written out unfused so that the decision follows the stated
// arithmetic step by step.
constexpr int kMaxRadialBins = 1024;
__global__ __launch_bounds__(256) void k_estimate_support(const double* __restrict__ sum,
                                                         const double* __restrict__ sumsq, long long n,
                                                         const double* __restrict__ power,
                                                         const double* __restrict__ xi, const double* __restrict__ wq,
                                                         int L, int n_xi, int H, double s2, double frac,
                                                         double* __restrict__ out) {
  __shared__ double vb[kMaxRadialBins];
  const int rmax = L / 2, h = L / 2;
  const double dn = (double)n;
  for (int b = threadIdx.x; b <= rmax; b += blockDim.x) {
    double tot = 0.0;
    long long cnt = 0;
    for (int p = 0; p < L * L; ++p) {
      const int a = p / L, c = p - a * L;
      const double x1 = (double)(a - h), x2 = (double)(c - h);
      if ((int)rint(sqrt(x1 * x1 + x2 * x2)) != b) continue;
      const double m = __ddiv_rn(sum[p], dn);
      const double v = __dsub_rn(__ddiv_rn(sumsq[p], dn), __dmul_rn(m, m));
      tot = __dadd_rn(tot, v);
      ++cnt;
    }
    vb[b] = __ddiv_rn(tot, (double)cnt);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double cv = 0.0;
  for (int b = 0; b <= rmax; ++b) cv = __dadd_rn(cv, __dmul_rn(__dsub_rn(vb[b], s2), (double)b));
  const double thr_r = __dmul_rn(frac, cv);
  double acc = 0.0;
  int R = 0;
  for (int b = 0; b <= rmax; ++b) {
    acc = __dadd_rn(acc, __dmul_rn(__dsub_rn(vb[b], s2), (double)b));
    if (acc >= thr_r) {
      R = b;
      break;
    }
  }
  const double den = (double)(n * (long long)H * L * L);
  double cp = 0.0;
  for (int j = 0; j < n_xi; ++j)
    cp = __dadd_rn(cp, __dmul_rn(__dmul_rn(__dsub_rn(__ddiv_rn(power[j], den), s2), xi[j]), wq[j]));
  const double thr_c = __dmul_rn(frac, cp);
  acc = 0.0;
  int jc = 0;
  for (int j = 0; j < n_xi; ++j) {
    acc = __dadd_rn(acc, __dmul_rn(__dmul_rn(__dsub_rn(__ddiv_rn(power[j], den), s2), xi[j]), wq[j]));
    if (acc >= thr_c) {
      jc = j;
      break;
    }
  }
  out[0] = (double)R;
  out[1] = xi[jc];
}

size_t moments_workspace_bytes(const Plan& pl) {
  return (size_t)2 * kMomentSlices * pl.L * pl.L * sizeof(double);
}

hipError_t launch_pixel_moments(const Plan& pl, const float* images, long long n, double* sum, double* sumsq,
                                double* ws, hipStream_t st) {
  const int npix = pl.L * pl.L;
  const int S = (int)std::min<long long>(kMomentSlices, n);
  const long long per = (n + S - 1) / S;
  const int S_used = (int)((n + per - 1) / per);
  pl.prof.begin(ST_ESTIMATE, st);
  hipLaunchKernelGGL(k_pixel_moments_part, dim3((unsigned)((npix + 255) / 256), (unsigned)S_used), dim3(256), 0, st,
                     images, n, npix, per, ws);
  hipLaunchKernelGGL(k_pixel_moments_reduce, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, ws, npix,
                     S_used, sum, sumsq);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_mean_image(const Plan& pl, const double* sum, long long count, float* mean, hipStream_t st) {
  const int npix = pl.L * pl.L;
  hipLaunchKernelGGL(k_mean_image, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, sum, count, npix, mean);
  return hipGetLastError();
}

hipError_t launch_copy_polar(const Plan& pl, const float2* P, float2* dst, hipStream_t st) {
  const int total = pl.n_xi * pl.H;
  hipLaunchKernelGGL(k_copy_polar, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, P, total, dst);
  return hipGetLastError();
}

hipError_t launch_polar_power(const Plan& pl, const float2* P, const float2* Pmean, int nimg, double* power,
                              hipStream_t st) {
  const int ngrp = (nimg + kImgGroup - 1) / kImgGroup;
  pl.prof.begin(ST_ESTIMATE, st);
  hipLaunchKernelGGL(k_polar_power, dim3((unsigned)pl.n_xi), dim3(256), 0, st, P, Pmean, pl.H, nimg, ngrp, power);
  pl.prof.end(st);
  return hipGetLastError();
}

// Eq.(CTFenv) at f = xi_j / pixel_size, one ring per thread, in FP64
__global__ void k_ctf_filter(const double* __restrict__ xi, int n_xi, double pixel_size, double lambda,
                             double defocus, double phase, double bfactor, float* __restrict__ filter) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n_xi) {
    const double f = xi[j] / pixel_size, f2 = f * f;
    const double env = fmin(3.14159265358979323846 * lambda * defocus * f2 + phase, 1.0);
    filter[j] = (float)(env * exp(-bfactor * f2));
  }
}

hipError_t launch_ctf_filter(const Plan& pl, double pixel_size, double lambda, double defocus, double phase,
                             double bfactor, float* filter, hipStream_t st) {
  hipLaunchKernelGGL(k_ctf_filter, dim3((unsigned)((pl.n_xi + 255) / 256)), dim3(256), 0, st, pl.d_xi, pl.n_xi,
                     pixel_size, lambda, defocus, phase, bfactor, filter);
  return hipGetLastError();
}

hipError_t launch_estimate_support(const Plan& pl, const double* sum, const double* sumsq, long long n,
                                   const double* power, double noise_var, double frac, double* out, hipStream_t st) {
  if (pl.L / 2 + 1 > kMaxRadialBins) return hipErrorInvalidValue;
  pl.prof.begin(ST_ESTIMATE, st);
  hipLaunchKernelGGL(k_estimate_support, dim3(1), dim3(256), 0, st, sum, sumsq, n, power, pl.d_xi, pl.d_wq, pl.L,
                     pl.n_xi, pl.H, noise_var, frac, out);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
