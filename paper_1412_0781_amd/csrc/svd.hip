// Principal components from the SVD of the coefficient matrices (Sec. III-C: the left
// singular vectors of A^(k) instead of the eigenvectors of C^(k)).  For each k the real row
// matrix X^(k) = [Re A^(k)^T; Im A^(k)^T] (k > 0), or A^(0)^T minus the mean (k = 0), has
// Gram matrix n C^(k).  It is reduced to its triangular factor R^(k) by Householder
// reflections (a tall-skinny QR: workgroups stream disjoint row ranges into their own R, a
// second pass merges those R's per k), and the one-sided Jacobi method (Hestenes)
// orthogonalises the columns of R^(k)^T: their norms are the singular values sigma_l of
// X^(k) and their directions its right singular vectors, the principal components;
// lambda_l = sigma_l^2 / n.  FP64 throughout (the FP32 coefficients are exact in FP64) and
// no Gram matrix is formed, so the small singular values keep their relative accuracy.
#include <hip/hip_runtime.h>

#include "jacobi_dev.h"
#include "kernels.h"

namespace fb {

constexpr int kSvdChunk = 32;          // rows per Householder update
constexpr int kSvdHalf = kSvdChunk / 2;  // rows per thread: two threads per column
constexpr int kSvdThreadsMax = 2 * kSvdMaxP;  // two threads per matrix column; 256 threads when max p_k <= 128

__device__ __forceinline__ long long tri_row(int j, int p) { return (long long)j * p - (long long)j * (j - 1) / 2; }

// k = 0 mean: m_q = (1/n) sum_i Re a^i_{0,q}, in FP64 and a fixed order (grid: one
// workgroup per q).
__global__ __launch_bounds__(256) void k_svd_mean(const float* __restrict__ coeffs, long long n, long long p_half,
                                                  double* __restrict__ mean) {
  __shared__ double s[256];
  const int q = blockIdx.x;
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) acc += (double)coeffs[(i * p_half + q) * 2];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[q] = s[0] / (double)n;
}

// [R; Y] <- the triangular factor of the stack: R upper triangular p x p (rows packed,
// row j from tri_row(j, p); its diagonal kept apart, read from dA and written to dB), Y
// a chunk of kSvdChunk rows held in registers: thread (c = tid / 2, h = tid % 2) holds rows
// h * kSvdHalf .. of column c in y[], and only it changes them.  The reflector of column j
// follows LAPACK's convention (beta = -sign(x0) ||(x0, y)||, tau = (beta - x0) / beta,
// v = (1, y / (x0 - beta))).  The owners of column j + 1 publish it at the end of step j,
// once it is up to date: its values to yb and its scalars (tau, 1 / (x0 - beta)) to ref,
// both double-buffered by the parity of the column.  One barrier per column.
__device__ __forceinline__ void publish_column(const double (&y)[kSvdHalf], int h, double x0, int j, double* yb,
                                               double* ref, double* dB) {
  double* dst = yb + (j & 1) * kSvdChunk + h * kSvdHalf;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < kSvdHalf; ++r) {
    dst[r] = y[r];
    s[r & 3] = fma(y[r], y[r], s[r & 3]);
  }
  double s2 = (s[0] + s[1]) + (s[2] + s[3]);
  s2 += __shfl_xor(s2, 1);
  if (h == 0) {
    double tau = 0.0, inv_d = 0.0, beta = x0;
    if (s2 != 0.0) {
      const double nrm = sqrt(fma(x0, x0, s2));
      beta = x0 >= 0.0 ? -nrm : nrm;
      inv_d = 1.0 / (x0 - beta);
      tau = (beta - x0) / beta;
    }
    ref[2 * (j & 1)] = tau;
    ref[2 * (j & 1) + 1] = inv_d;
    dB[j] = beta;
  }
}

__device__ void householder_chunk(double* R, const double* dA, double* dB, double (&y)[kSvdHalf], double* yb,
                                  double* ref, int p) {
  const int c = threadIdx.x >> 1, h = threadIdx.x & 1;
  if (c == 0) publish_column(y, h, dA[0], 0, yb, ref, dB);
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    const double tau = ref[2 * (j & 1)], inv_d = ref[2 * (j & 1) + 1];
    if (c > j && c < p) {
      if (tau != 0.0) {
        const double* yj = yb + (j & 1) * kSvdChunk + h * kSvdHalf;
        double* rjc = R + tri_row(j, p) + (c - j);
        double w4[4] = {h == 0 ? *rjc : 0.0, 0.0, 0.0, 0.0};
        double v[kSvdHalf];
#pragma unroll
        for (int r = 0; r < kSvdHalf; ++r) {
          v[r] = yj[r] * inv_d;
          w4[r & 3] = fma(v[r], y[r], w4[r & 3]);
        }
        double w = (w4[0] + w4[1]) + (w4[2] + w4[3]);
        w += __shfl_xor(w, 1);
        const double tw = tau * w;
        if (h == 0) *rjc -= tw;
#pragma unroll
        for (int r = 0; r < kSvdHalf; ++r) y[r] = fma(-tw, v[r], y[r]);
      }
      if (c == j + 1) publish_column(y, h, dA[c], c, yb, ref, dB);
    }
    __syncthreads();
  }
}

// LDS of the streaming QR: packed R, two diagonals, the published column (two buffers)
// and its reflector scalars (two pairs).
__host__ __device__ inline long long svd_qr_lds_doubles(int p) {
  return (long long)p * (p + 1) / 2 + 2LL * p + 2LL * kSvdChunk + 4;
}

// Level 1: workgroup (k, w) reduces rows [w rows_per, (w + 1) rows_per) of X^(k) to a
// packed R at Rout + offset(k, w).  Blocks 0 .. W0-1 take k = 0, then W1 blocks per k > 0.
__global__ __launch_bounds__(kSvdThreadsMax) void k_svd_tsqr(const float* __restrict__ coeffs, long long n,
                                                          long long p_half, const double* __restrict__ mean,
                                                          const int* __restrict__ p_arr,
                                                          const int* __restrict__ coef_off,
                                                          const long long* __restrict__ tri_off, int W0, int W1,
                                                          long long base1, long long rows_per,
                                                          double* __restrict__ Rout) {
  extern __shared__ double sm[];
  int b = blockIdx.x, k, w;
  if (b < W0) {
    k = 0;
    w = b;
  } else {
    b -= W0;
    k = 1 + b / W1;
    w = b - (k - 1) * W1;
  }
  const int pk = p_arr[k], off = coef_off[k], tid = threadIdx.x;
  const long long nrows = k == 0 ? n : 2 * n;
  const long long r0 = (long long)w * rows_per, r1 = min(nrows, r0 + rows_per);
  const long long tp = (long long)pk * (pk + 1) / 2;
  double* R = sm;
  double* dA = R + tp;
  double* dB = dA + pk;
  double* yb = dB + pk;
  double* ref = yb + 2 * kSvdChunk;
  for (long long i = tid; i < tp; i += (int)blockDim.x) R[i] = 0.0;
  for (int i = tid; i < pk; i += (int)blockDim.x) dA[i] = dB[i] = 0.0;
  const int c = tid >> 1, h = tid & 1;
  double y[kSvdHalf];
  for (long long q0 = r0; q0 < r1; q0 += kSvdChunk) {
#pragma unroll
    for (int r = 0; r < kSvdHalf; ++r) {
      const long long row = q0 + h * kSvdHalf + r;
      double v = 0.0;
      if (c < pk && row < r1) {
        const long long img = row < n ? row : row - n;
        v = (double)coeffs[((size_t)img * p_half + off + c) * 2 + (row < n ? 0 : 1)];
        if (k == 0) v -= mean[c];
      }
      y[r] = v;
    }
    __syncthreads();
    householder_chunk(R, dA, dB, y, yb, ref, pk);
    double* t = dA;
    dA = dB;
    dB = t;
  }
  __syncthreads();
  for (int j = tid; j < pk; j += (int)blockDim.x) R[tri_row(j, pk)] = dA[j];
  __syncthreads();
  double* out = Rout + (k == 0 ? 0 : base1 + (long long)W1 * (tri_off[k] - tri_off[1])) + (long long)w * tp;
  for (long long i = tid; i < tp; i += (int)blockDim.x) out[i] = R[i];
}

// Level 2 and the small SVD, one workgroup per k: merge the W R's of k (their rows streamed
// through the same update), write M = R^T column by column to Mg (column l = row l of R),
// load M into LDS, run cyclic one-sided Jacobi sweeps over the column pairs (round-robin
// order: the P/2 disjoint pairs of a round go to the waves, one pair per wave), then write
// lambda_l = ||m_l||^2 / n in descending order and the columns m_l / ||m_l||, the entry of
// largest magnitude made positive (lowest index on ties), packed like the covariance.
__global__ __launch_bounds__(kSvdThreadsMax) void k_svd_finish(const double* __restrict__ Rin_all, long long n,
                                                            const int* __restrict__ p_arr,
                                                            const int* __restrict__ coef_off,
                                                            const long long* __restrict__ cov_off,
                                                            const long long* __restrict__ tri_off, int W0, int W1,
                                                            long long base1, double* __restrict__ Mg_all,
                                                            double* __restrict__ evals, double* __restrict__ evecs,
                                                            long long lds_doubles) {
  extern __shared__ double sm[];
  __shared__ int s_rot;
  const int k = blockIdx.x, pk = p_arr[k], tid = threadIdx.x;
  const int W = k == 0 ? W0 : W1;
  const long long tp = (long long)pk * (pk + 1) / 2;
  const double* Rin = Rin_all + (k == 0 ? 0 : base1 + (long long)W1 * (tri_off[k] - tri_off[1]));
  // ---- merge
  double* R = sm;
  double* dA = R + tp;
  double* dB = dA + pk;
  double* yb = dB + pk;
  double* ref = yb + 2 * kSvdChunk;
  for (long long i = tid; i < tp; i += (int)blockDim.x) R[i] = 0.0;
  for (int i = tid; i < pk; i += (int)blockDim.x) dA[i] = dB[i] = 0.0;
  const long long nrows = (long long)W * pk;
  const int c = tid >> 1, h = tid & 1;
  double y[kSvdHalf];
  for (long long g0 = 0; g0 < nrows; g0 += kSvdChunk) {
#pragma unroll
    for (int r = 0; r < kSvdHalf; ++r) {
      const long long g = g0 + h * kSvdHalf + r;
      double v = 0.0;
      if (c < pk && g < nrows) {
        const long long w = g / pk;
        const int j = (int)(g - w * pk);
        if (c >= j) v = Rin[w * tp + tri_row(j, pk) + (c - j)];
      }
      y[r] = v;
    }
    __syncthreads();
    householder_chunk(R, dA, dB, y, yb, ref, pk);
    double* t = dA;
    dA = dB;
    dB = t;
  }
  __syncthreads();
  for (int j = tid; j < pk; j += (int)blockDim.x) R[tri_row(j, pk)] = dA[j];
  __syncthreads();
  double* Mg = Mg_all + cov_off[k];
  for (int i = tid; i < pk * pk; i += (int)blockDim.x) {
    const int l = i / pk, c = i - l * pk;
    Mg[i] = c >= l ? R[tri_row(l, pk) + (c - l)] : 0.0;
  }
  __syncthreads();
  // the rotations run on M in LDS when it fits (the LDS of R is free now), else on Mg in
  // global memory (the waves of one workgroup meet at barriers, which order those accesses)
  const bool in_lds = (long long)pk * pk + pk <= lds_doubles;
  double* M = in_lds ? sm : Mg;
  if (in_lds)
    for (int i = tid; i < pk * pk; i += (int)blockDim.x) M[i] = Mg[i];
  double* sig2 = in_lds ? M + (long long)pk * pk : sm;
  // ---- one-sided Jacobi
  one_sided_jacobi(M, pk, &s_rot);
  // ---- singular values, order, sign, output
  for (int l = tid; l < pk; l += (int)blockDim.x) {
    double a = 0.0;
    for (int e = 0; e < pk; ++e) a = fma(M[(long long)l * pk + e], M[(long long)l * pk + e], a);
    sig2[l] = a;
  }
  __syncthreads();
  const long long eo = cov_off[k];
  const int co = coef_off[k];
  for (int l = tid; l < pk; l += (int)blockDim.x) {
    const double s2 = sig2[l];
    int rank = 0;
    for (int m = 0; m < pk; ++m) rank += (sig2[m] > s2 || (sig2[m] == s2 && m < l)) ? 1 : 0;
    const double* col = M + (long long)l * pk;
    int im = 0;
    double vm = fabs(col[0]);
    for (int e = 1; e < pk; ++e)
      if (fabs(col[e]) > vm) {
        vm = fabs(col[e]);
        im = e;
      }
    const double sg = col[im] < 0.0 ? -1.0 : 1.0;
    const double inv = s2 > 0.0 ? sg / sqrt(s2) : 0.0;
    evals[co + rank] = s2 / (double)n;
    for (int e = 0; e < pk; ++e) evecs[eo + (long long)e * pk + rank] = inv * col[e];
  }
}

int svd_max_p(const Plan& pl) { return *std::max_element(pl.p.begin(), pl.p.end()); }

size_t svd_finish_lds_bytes(const Plan& pl) {
  // the merge's LDS, and the p x p block of the rotations with its p norms when that fits
  const int pm = *std::max_element(pl.p.begin(), pl.p.end());
  long long need = std::max(svd_qr_lds_doubles(pm), (long long)pm);
  const long long block = (long long)pm * pm + pm;
  if (block * (long long)sizeof(double) <= kSvdLdsLimit) need = std::max(need, block);
  return (size_t)need * sizeof(double);
}

int svd_threads(const Plan& pl) { return svd_max_p(pl) > kSvdMaxP / 2 ? kSvdThreadsMax : kSvdThreadsMax / 2; }

size_t svd_qr_lds_bytes(const Plan& pl) {
  const int pm = *std::max_element(pl.p.begin(), pl.p.end());
  return (size_t)svd_qr_lds_doubles(pm) * sizeof(double);
}

hipError_t configure_svd_kernels() {
  hipError_t e = hipFuncSetAttribute((const void*)k_svd_tsqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     kSvdLdsLimit);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_svd_finish, hipFuncAttributeMaxDynamicSharedMemorySize, kSvdLdsLimit);
}

SvdSplit svd_split(const Plan& pl, long long n) {
  SvdSplit s;
  s.W0 = (int)((n + kSvdRowsPerGroup - 1) / kSvdRowsPerGroup);
  s.W1 = (int)((2 * n + kSvdRowsPerGroup - 1) / kSvdRowsPerGroup);
  const long long t0 = (long long)pl.p[0] * (pl.p[0] + 1) / 2;
  s.base1 = (long long)s.W0 * t0;
  s.r_doubles = s.base1 + (long long)s.W1 * (pl.tri_off[pl.k_max + 1] - pl.tri_off[1]);
  s.mean_doubles = (pl.p[0] + 31) / 32 * 32;
  s.total_doubles = s.mean_doubles + s.r_doubles + pl.cov_size;
  return s;
}

hipError_t launch_svd(const Plan& pl, const float* coeffs, long long n, double* evals, double* evecs,
                      double* mean_out, double* ws, hipStream_t st) {
  const SvdSplit s = svd_split(pl, n);
  double* mean = mean_out ? mean_out : ws;
  double* Rws = ws + s.mean_doubles;
  double* Mws = Rws + s.r_doubles;
  pl.prof.begin(ST_SVD, st);
  hipLaunchKernelGGL(k_svd_mean, dim3((unsigned)pl.p[0]), dim3(256), 0, st, coeffs, n, (long long)pl.p_half, mean);
  pl.prof.end(st);
  const long long nblk = (long long)s.W0 + (long long)s.W1 * pl.k_max;
  pl.prof.begin(ST_SVD, st);
  const int nthr = svd_threads(pl);
  hipLaunchKernelGGL(k_svd_tsqr, dim3((unsigned)nblk), dim3(nthr), svd_qr_lds_bytes(pl), st, coeffs, n,
                     (long long)pl.p_half, mean, pl.d_p, pl.d_coef_off, pl.d_tri_off, s.W0, s.W1, s.base1,
                     (long long)kSvdRowsPerGroup, Rws);
  pl.prof.end(st);
  pl.prof.begin(ST_SVD, st);
  const size_t fin_lds = svd_finish_lds_bytes(pl);
  hipLaunchKernelGGL(k_svd_finish, dim3((unsigned)(pl.k_max + 1)), dim3(nthr), fin_lds, st, Rws, n, pl.d_p,
                     pl.d_coef_off, pl.d_cov_off, pl.d_tri_off, s.W0, s.W1, s.base1, Mws, evals, evecs,
                     (long long)(fin_lds / sizeof(double)));
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
