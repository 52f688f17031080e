// Steerable PCA back end on the device (Algorithm 2, steps 5-6, and the component
// selection and eigenvalue shrinkage of Sec. V), from the eigenpairs of fb_eig:
//   selection  lambda_l^(k) > sigma^2 (1 + sqrt(gamma_k))^2, gamma_0 = p_0/n,
//              gamma_k = p_k/(2n) (Eq.(compselect)); filter ell/(ell + sigma^2) with
//              ell = (lambda - sigma^2)_+ on the selected components, 0 elsewhere
//   project    c_{k,.} = (a_{k,.} - m delta_{k0}) U^(k)               (Eq.(sPCAcoeff))
//   rebuild    a_{k,.} = U^(k) (w_k * c_{k,.}) + m delta_{k0}
//   radial     f^{k,l}(xi_j) = sum_q N_{k,q} J_k(R_{k,q} xi_j / c) u_l^(k)(q)  (Eq.(sPCArad))
//   real space E^{k,l}(x) = sum_q u_l^(k)(q) F^{-1}(psi_c^{k,q})(x)  (Eq.(IFT_FB), i^k in the
//              numerator), the eigenimages of Sec. VI-B on the pixel grid, in FP64
// The two coefficient maps are per-k products of the complex coefficients (real and
// imaginary parts as separate rows) with the real p_k x p_k matrix U^(k), on
// v_mfma_f32_32x32x2f32 in 64 x 64 tiles (FP32 products and sums; U rounded to FP32).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace fb {

typedef float f32x16_s __attribute__((ext_vector_type(16)));

__global__ void k_spca_select(const double* __restrict__ evals, const int* __restrict__ coef_off,
                              const int* __restrict__ p, double n, double sigma2, int* __restrict__ n_sel,
                              double* __restrict__ weights) {
  const int k = blockIdx.x, pk = p[k], off = coef_off[k];
  const double gamma = (k == 0) ? pk / n : pk / (2.0 * n);
  const double edge = sigma2 * (1.0 + sqrt(gamma)) * (1.0 + sqrt(gamma));
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int l = threadIdx.x; l < pk; l += blockDim.x) {
    const double lam = evals[off + l];
    const bool sel = lam > edge;
    const double ell = lam > sigma2 ? lam - sigma2 : 0.0;
    weights[off + l] = sel ? ell / (ell + sigma2) : 0.0;
    if (sel) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) n_sel[k] = cnt;
}

// MODE 0 (project): out[i][off + l] = sum_q (a[i][off + q] - m_q [k = 0, re]) U[q][l]
// MODE 1 (rebuild): out[i][off + q] = sum_l U[q][l] w[off + l] c[i][off + l] + m_q [k = 0, re]
// grid: (runs of kSpcaBlocks image blocks of 32, work items (k, 64-wide output tile)); rows
// of a tile are (image, re/im) pairs.  PANEL: the item's whole B operand (p_k rows of its 64
// columns, rounded to FP32 once) sits in LDS for all the run's image blocks; otherwise it is
// read per chunk of 16 rows (blocks above the panel's capacity).  An image's coefficients of
// block k are one contiguous run, read as (re, im) pairs along q.
constexpr int kSpcaBlocks = 8;
constexpr int kSpcaTK = 16, kSpcaLd = 64 + 4;
template <int MODE, bool PANEL>
__global__ __launch_bounds__(256) void k_spca_apply(const float* __restrict__ in, float* __restrict__ out,
                                                    const double* __restrict__ evecs,
                                                    const double* __restrict__ mean,
                                                    const double* __restrict__ weights,
                                                    const GemmItem* __restrict__ items,
                                                    const int* __restrict__ coef_off, const int* __restrict__ p,
                                                    const long long* __restrict__ cov_off, long long n,
                                                    long long p_half) {
  constexpr int TM = 64, TK = kSpcaTK, LD = kSpcaLd;
  extern __shared__ float spca_lds[];
  float(*As)[LD] = (float(*)[LD])spca_lds;              // TK rows
  float(*Bs)[LD] = (float(*)[LD])(spca_lds + TK * LD);  // p_k rounded to TK rows (PANEL) or TK rows
  const GemmItem it = items[blockIdx.y];
  const int k = it.k, n0 = it.t0, pk = p[k], off = coef_off[k];
  const double* U = evecs + cov_off[k];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  // B rows r0 .. r0 + nr - 1 of this item's 64 columns into Bs[d0 + ...]
  auto load_b = [&](int r0, int nr, int d0) {
    for (int e = tid; e < nr * 64; e += 256) {
      const int kk = e >> 6, nn = e & 63;
      const int r = r0 + kk, c = n0 + nn;
      float v = 0.f;
      if (r < pk && c < pk) {
        if (MODE == 0)
          v = (float)U[(size_t)r * pk + c];                                     // U[q = r][l = c]
        else
          v = (float)(U[(size_t)c * pk + r] * (weights ? weights[off + r] : 1.0));  // U[q = c][l = r] w_l
      }
      Bs[d0 + kk][nn] = v;
    }
  };
  const int pk_pad = (pk + TK - 1) / TK * TK;
  if (PANEL) {
    load_b(0, pk_pad, 0);
    __syncthreads();
  }
  // the A chunk: thread t loads image t / 8 of the block, q = k0 + 2 (t % 8) + {0, 1}
  const int ai = tid >> 3, aq = 2 * (tid & 7);
  for (int blk = 0; blk < kSpcaBlocks; ++blk) {
    const long long i0 = ((long long)blockIdx.x * kSpcaBlocks + blk) * (TM / 2);
    if (i0 >= n) break;
    const long long img = i0 + ai;
    const float2* arow = (const float2*)(in + (size_t)min(img, n - 1) * 2 * p_half) + off;
    // the next chunk's pair of values is loaded while the current one is multiplied; the
    // loads are unconditional (clamped to the block), values outside it are replaced by 0
    float2 pa[2];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) pa[h] = arow[min(k0 + aq + h, pk - 1)];
    };
    fetch(0);
    f32x16_s acc = {};
    for (int k0 = 0; k0 < pk; k0 += TK) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = k0 + aq + h;
        float2 v = (img < n && q < pk) ? pa[h] : make_float2(0.f, 0.f);
        if (MODE == 0 && k == 0 && q < pk) v.x -= (float)mean[q];
        *(float2*)&As[aq + h][2 * ai] = v;
      }
      if (!PANEL) load_b(k0, TK, 0);
      __syncthreads();
      if (k0 + TK < pk) fetch(k0 + TK);
      const int b0 = PANEL ? k0 : 0;
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        const float a = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
        const float b = Bs[b0 + kk + (lane >> 5)][wn * 32 + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = wm * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
      const int c = n0 + wn * 32 + (lane & 31);
      const long long oi = i0 + (m >> 1);
      const int ri = m & 1;
      if (oi < n && c < pk) {
        float v = acc[i];
        if (MODE == 1 && k == 0 && ri == 0) v += (float)mean[c];
        out[(size_t)oi * 2 * p_half + 2 * (size_t)(off + c) + ri] = v;
      }
    }
  }
}

// f [sum_k n_xi p_k]: block k at n_xi * coef_off[k], [n_xi][p_k] row-major
__global__ void k_spca_radial(const float* __restrict__ radial, const float* __restrict__ xw,
                              const double* __restrict__ evecs, const int* __restrict__ coef_off,
                              const int* __restrict__ p, const long long* __restrict__ cov_off, int n_xi,
                              float* __restrict__ f) {
  const int k = blockIdx.x, pk = p[k], off = coef_off[k];
  const double* U = evecs + cov_off[k];
  for (int e = threadIdx.x; e < n_xi * pk; e += blockDim.x) {
    const int j = e / pk, l = e - j * pk;
    double s = 0.0;
    for (int q = 0; q < pk; ++q) s += (double)radial[(size_t)(off + q) * n_xi + j] * U[(size_t)q * pk + l];
    f[(size_t)n_xi * off + e] = (float)(s / (double)xw[j]);
  }
}

// J_k(z) and J_{k+1}(z), z >= 0, by Miller's backward recurrence J_{m-1} = (2m/z) J_m - J_{m+1}
// started well above max(k + 1, z) (the start-order rule of Abramowitz & Stegun 9.12),
// normalised with J_0 + 2 sum_{m>=1} J_{2m} = 1, rescaled whenever the values pass 1e250.
__device__ void bessel_jk_pair(int k, double z, double& jk, double& jk1) {
  if (z == 0.0) {
    jk = k == 0 ? 1.0 : 0.0;
    jk1 = 0.0;
    return;
  }
  const double top = fmax((double)(k + 1), z);
  const int m0 = 2 * ((int)(top + 20.0 + sqrt(60.0 * top)) / 2) + 2;
  const double tz = 2.0 / z;
  double jp = 0.0, j = 1e-300, sum = 0.0, a = 0.0, b = 0.0;
  for (int m = m0; m >= 1; --m) {
    const double jm = (double)m * tz * j - jp;  // J_{m-1}
    jp = j;
    j = jm;
    const int o = m - 1;
    if (o == k + 1) b = j;
    if (o == k) a = j;
    if (o > 0 && (o & 1) == 0) sum += 2.0 * j;
    if (fabs(j) > 1e250) {
      j *= 1e-250;
      jp *= 1e-250;
      sum *= 1e-250;
      a *= 1e-250;
      b *= 1e-250;
    }
  }
  sum += j;
  jk = a / sum;
  jk1 = b / sum;
}

// Eigenimages of components l0 .. l0 + nl - 1 at angular frequency k on the L x L grid,
// one pixel per lane:
//   E(x) = 2 c sqrt(pi) i^k e^{ik phi} J_k(z) sum_q (-1)^q R_q u_l(q) / (z^2 - R_q^2),
// z = 2 pi c r.  Within kEigRootGuard of a root R_q the quotient J_k(z) / (z^2 - R_q^2) takes
// its limit -J_{k+1}(z) / (z + R_q).  Components go in chunks of kEigChunk accumulators.
constexpr double kEigRootGuard = 1e-8;
constexpr int kEigChunk = 16;
__global__ __launch_bounds__(64) void k_spca_eigenimages(const double* __restrict__ evecs,
                                                         const double* __restrict__ roots, int k, int pk,
                                                         int l0, int nl, int L, double c,
                                                         double2* __restrict__ out) {
  const int pix = blockIdx.x * 64 + threadIdx.x;
  if (pix >= L * L) return;
  const int a = pix / L, b = pix - a * L;
  const double x1 = (double)(a - L / 2), x2 = (double)(b - L / 2);
  const double pi = 3.14159265358979323846;
  const double z = 2.0 * pi * c * sqrt(x1 * x1 + x2 * x2);
  double jk, jk1;
  bessel_jk_pair(k, z, jk, jk1);
  double sn, cs;
  sincos((double)k * atan2(x2, x1), &sn, &cs);
  double ar, ai;  // i^k e^{ik phi}
  switch (k & 3) {
    case 0: ar = cs; ai = sn; break;
    case 1: ar = -sn; ai = cs; break;
    case 2: ar = -cs; ai = -sn; break;
    default: ar = sn; ai = -cs; break;
  }
  const double pref = 2.0 * c * sqrt(pi);
  const size_t plane = (size_t)L * L;
  for (int c0 = 0; c0 < nl; c0 += kEigChunk) {
    const int nc = min(kEigChunk, nl - c0);
    double acc[kEigChunk];
#pragma unroll
    for (int t = 0; t < kEigChunk; ++t) acc[t] = 0.0;
    for (int q = 1; q <= pk; ++q) {
      const double R = roots[q - 1];
      const double d = z - R;
      const double tq = (fabs(d) < kEigRootGuard ? -jk1 / (z + R) : jk / (d * (z + R))) * ((q & 1) ? -R : R);
      const double* Uq = evecs + (size_t)(q - 1) * pk + l0 + c0;
#pragma unroll
      for (int t = 0; t < kEigChunk; ++t)
        if (t < nc) acc[t] = fma(Uq[t], tq, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kEigChunk; ++t)
      if (t < nc) {
        const double v = pref * acc[t];
        out[(size_t)(c0 + t) * plane + pix] = make_double2(v * ar, v * ai);
      }
  }
}

hipError_t launch_spca_select(const Plan& pl, const double* evals, long long count, double sigma2, int* n_sel,
                              double* weights, hipStream_t st) {
  pl.prof.begin(ST_SPCA, st);
  hipLaunchKernelGGL(k_spca_select, dim3((unsigned)(pl.k_max + 1)), dim3(256), 0, st, evals, pl.d_coef_off, pl.d_p,
                     (double)count, sigma2, n_sel, weights);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_spca_apply(const Plan& pl, int mode, const float* in, long long n, const double* evecs,
                             const double* mean, const double* weights, float* out, hipStream_t st) {
  const long long runs = (n + 32LL * kSpcaBlocks - 1) / (32LL * kSpcaBlocks);
  if (runs > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 g((unsigned)runs, (unsigned)pl.items_spca.size());
  int pmax = 0;
  for (int v : pl.p) pmax = std::max(pmax, v);
  const int rows = (pmax + kSpcaTK - 1) / kSpcaTK * kSpcaTK;
  // B panel resident while the kernel's LDS stays within 64 KB (p_k <= 224), otherwise
  // streamed by chunks
  const bool panel = (kSpcaTK + rows) * kSpcaLd * sizeof(float) <= 64u * 1024u;
  const size_t lds = (size_t)(kSpcaTK + (panel ? rows : kSpcaTK)) * kSpcaLd * sizeof(float);
  pl.prof.begin(ST_SPCA, st);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, g, dim3(256), lds, st, in, out, evecs, mean, weights, pl.d_items_spca, pl.d_coef_off,
                       pl.d_p, pl.d_cov_off, n, (long long)pl.p_half);
  };
  if (mode == 0)
    panel ? go(k_spca_apply<0, true>) : go(k_spca_apply<0, false>);
  else
    panel ? go(k_spca_apply<1, true>) : go(k_spca_apply<1, false>);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_spca_radial(const Plan& pl, const double* evecs, float* f, hipStream_t st) {
  pl.prof.begin(ST_SPCA, st);
  hipLaunchKernelGGL(k_spca_radial, dim3((unsigned)(pl.k_max + 1)), dim3(256), 0, st, pl.d_radial, pl.d_xw, evecs,
                     pl.d_coef_off, pl.d_p, pl.d_cov_off, pl.n_xi, f);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_eigenimages(const Plan& pl, const double* evecs, int k, int l0, int nl, double* out,
                              hipStream_t st) {
  const long long npix = (long long)pl.L * pl.L;
  pl.prof.begin(ST_SPCA, st);
  hipLaunchKernelGGL(k_spca_eigenimages, dim3((unsigned)((npix + 63) / 64)), dim3(64), 0, st,
                     evecs + pl.cov_off[k], pl.d_roots + pl.coef_off[k], k, pl.p[k], l0, nl, pl.L, pl.c,
                     (double2*)out);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
