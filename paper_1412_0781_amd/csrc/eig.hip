// Algorithm 2, steps 1 and 4 in FP64 on the device: finalise each covariance
// block C^(k) = G^(k)/n (k = 0: minus d d^T with d = S0/n, the mean of the k = 0
// coefficients in the coordinates they were accumulated in: a_{0,q} - s_q when the
// accumulation used a shift s; the mean itself is s + d) and
// diagonalise it, one workgroup per k.  Where the block fits in LDS, by one-sided
// Jacobi rotations on its columns in LDS; otherwise by cyclic two-sided Jacobi
// rotations in global memory, every round applying p_k/2 disjoint rotations in
// parallel (round-robin pairing), so a sweep of p_k - 1 rounds visits every pair once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "jacobi_dev.h"
#include "kernels.h"

namespace fb {

constexpr int EIG_THREADS = 256;
constexpr int EIG_MAX_SWEEPS = 40;

__device__ double block_sum(double v, double* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];  // fixed order
  return s;
}

// C^(k) entry i = q p_k + r: G/n, minus m_q m_r for k = 0
__device__ __forceinline__ double cov_entry(const double* G, const double* S0, long long base, int k, int pk, int i,
                                            double inv) {
  const int q = i / pk, r = i - q * pk;
  double v = G[base + i] * inv;
  if (k == 0) v -= (S0[q] * inv) * (S0[r] * inv);
  return v;
}

// Two-sided cyclic Jacobi on A (global, p_k x p_k, destroyed) with the rotations
// accumulated into V (global, starts as the identity; ends as the sign-normalised
// eigenvectors in descending eigenvalue order), eigenvalues to evals + off_k.
__device__ void eig_two_sided(double* A, double* V, int pk, int off_k, double* evals) {
  __shared__ double red[EIG_THREADS / 64];
  __shared__ double cs[EIG_MAX_P / 2], sn[EIG_MAX_P / 2];
  __shared__ int pa[EIG_MAX_P / 2], pb[EIG_MAX_P / 2];
  __shared__ int stop;

  const int m = pk + (pk & 1);  // even number of positions; position pk is a dummy when pk is odd
  const int npair = m / 2;
  for (int sweep = 0; sweep < EIG_MAX_SWEEPS && pk > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = threadIdx.x; i < pk * pk; i += blockDim.x) {
      int q = i / pk, r = i - q * pk;
      double a2 = A[i] * A[i];
      tot += a2;
      if (q != r) off += a2;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) stop = (off <= 1e-30 * tot) || (off == 0.0);
    __syncthreads();
    if (stop) break;
    for (int round = 0; round < m - 1; ++round) {
      for (int i = threadIdx.x; i < npair; i += blockDim.x) {
        int t0 = i, t1 = m - 1 - i;
        int a = t0 == 0 ? 0 : 1 + (t0 - 1 + round) % (m - 1);
        int b = t1 == 0 ? 0 : 1 + (t1 - 1 + round) % (m - 1);
        double c = 1.0, s = 0.0;
        if (a < pk && b < pk) {
          double apq = A[(size_t)a * pk + b];
          if (apq != 0.0) {
            double app = A[(size_t)a * pk + a], aqq = A[(size_t)b * pk + b];
            double theta = (aqq - app) / (2.0 * apq);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[i] = c;
        sn[i] = s;
        pa[i] = a;
        pb[i] = b;
      }
      __syncthreads();
      // columns: A <- A J and V <- V J
      for (int i = threadIdx.x; i < npair * pk; i += blockDim.x) {
        int pr = i / pk, r = i - pr * pk;
        int a = pa[pr], b = pb[pr];
        if (a >= pk || b >= pk) continue;
        double c = cs[pr], s = sn[pr];
        double x = A[(size_t)r * pk + a], y = A[(size_t)r * pk + b];
        A[(size_t)r * pk + a] = c * x - s * y;
        A[(size_t)r * pk + b] = s * x + c * y;
        x = V[(size_t)r * pk + a];
        y = V[(size_t)r * pk + b];
        V[(size_t)r * pk + a] = c * x - s * y;
        V[(size_t)r * pk + b] = s * x + c * y;
      }
      __syncthreads();
      // rows: A <- J^T A
      for (int i = threadIdx.x; i < npair * pk; i += blockDim.x) {
        int pr = i / pk, r = i - pr * pk;
        int a = pa[pr], b = pb[pr];
        if (a >= pk || b >= pk) continue;
        double c = cs[pr], s = sn[pr];
        double x = A[(size_t)a * pk + r], y = A[(size_t)b * pk + r];
        A[(size_t)a * pk + r] = c * x - s * y;
        A[(size_t)b * pk + r] = s * x + c * y;
      }
      __syncthreads();
    }
  }
  // eigenvalues = diagonal, ordered descending (ties by index); columns sign-normalised
  // so that the entry of largest magnitude (lowest index on ties) is positive
  __shared__ int rk[EIG_MAX_P];
  for (int col = threadIdx.x; col < pk; col += blockDim.x) {
    double di = A[(size_t)col * pk + col];
    int rank = 0;
    for (int j = 0; j < pk; ++j) {
      double dj = A[(size_t)j * pk + j];
      rank += (dj > di) || (dj == di && j < col);
    }
    rk[col] = rank;
    evals[off_k + rank] = di;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < pk * pk; i += blockDim.x) A[i] = V[i];  // A is scratch from here on
  __syncthreads();
  for (int col = threadIdx.x; col < pk; col += blockDim.x) {
    int imax = 0;
    double vmax = -1.0;
    for (int r = 0; r < pk; ++r) {
      double v = fabs(A[(size_t)r * pk + col]);
      if (v > vmax) {
        vmax = v;
        imax = r;
      }
    }
    double sg = A[(size_t)imax * pk + col] < 0 ? -1.0 : 1.0;
    int rank = rk[col];
    for (int r = 0; r < pk; ++r) V[(size_t)r * pk + rank] = sg * A[(size_t)r * pk + col];
  }
}

// Two-sided form, A and V in global memory (any p_k up to EIG_MAX_P).
__global__ __launch_bounds__(EIG_THREADS) void k_eig(const double* __restrict__ G, const double* __restrict__ S0,
                                                     const float* __restrict__ shift, long long count, double* __restrict__ evals,
                                                     double* __restrict__ evecs, double* __restrict__ C_out,
                                                     double* __restrict__ mean_out, double* __restrict__ work,
                                                     const int* __restrict__ p, const int* __restrict__ coef_off,
                                                     const long long* __restrict__ cov_off) {
  const int k = blockIdx.x, pk = p[k];
  const long long base = cov_off[k];
  double* A = work + base;
  double* V = evecs + base;
  const double inv = 1.0 / (double)count;
  for (int i = threadIdx.x; i < pk * pk; i += blockDim.x) {
    const double v = cov_entry(G, S0, base, k, pk, i, inv);
    A[i] = v;
    if (C_out) C_out[base + i] = v;
    V[i] = (i / pk == i % pk) ? 1.0 : 0.0;
  }
  if (k == 0 && mean_out)
    for (int q = threadIdx.x; q < pk; q += blockDim.x) mean_out[q] = (shift ? (double)shift[q] : 0.0) + S0[q] * inv;
  __syncthreads();
  eig_two_sided(A, V, pk, coef_off[k], evals);
}

// One-sided form with C^(k) in LDS (p_k^2 + p_k doubles must fit): the columns of C are
// orthogonalised by Jacobi rotations, C V = B, with the rotations accumulated into V (in
// the workspace, column-major).  (C V)^T (C V) = V^T C^2 V diagonal makes V^T C V diagonal
// for a positive semidefinite C (the PSD square root of a diagonal matrix is diagonal), so
// the columns of V are the eigenvectors, each accurate to the orthogonality tolerance times
// ||C|| however small its eigenvalue; lambda_l = v_l . b_l (the Rayleigh quotient).
__global__ __launch_bounds__(EIG_THREADS) void k_eig_lds(const double* __restrict__ G, const double* __restrict__ S0,
                                                         const float* __restrict__ shift, long long count, double* __restrict__ evals,
                                                         double* __restrict__ evecs, double* __restrict__ C_out,
                                                         double* __restrict__ mean_out, double* __restrict__ work,
                                                         const int* __restrict__ p, const int* __restrict__ coef_off,
                                                         const long long* __restrict__ cov_off) {
  extern __shared__ double sm[];
  __shared__ int s_rot;
  __shared__ int rk[EIG_MAX_P];
  const int k = blockIdx.x, pk = p[k], tid = threadIdx.x;
  const long long base = cov_off[k];
  double* M = sm;                       // C^(k), column-major (symmetric)
  double* lam = sm + (long long)pk * pk;
  double* V = work + base;              // accumulated rotations, column-major
  const double inv = 1.0 / (double)count;
  for (int i = tid; i < pk * pk; i += blockDim.x) {
    const double v = cov_entry(G, S0, base, k, pk, i, inv);
    M[i] = v;
    V[i] = (i / pk == i % pk) ? 1.0 : 0.0;
    if (C_out) C_out[base + i] = v;
  }
  if (k == 0 && mean_out)
    for (int q = tid; q < pk; q += blockDim.x) mean_out[q] = (shift ? (double)shift[q] : 0.0) + S0[q] * inv;
  __syncthreads();
  one_sided_jacobi<true>(M, pk, &s_rot, V);
  for (int l = tid; l < pk; l += blockDim.x) {
    double a = 0.0;
    for (int e = 0; e < pk; ++e) a = fma(V[(long long)l * pk + e], M[(long long)l * pk + e], a);
    lam[l] = a;
  }
  __syncthreads();
  // eigenvalues descending (ties by index); columns sign-normalised so that the entry of
  // largest magnitude (lowest index on ties) is positive
  const int off_k = coef_off[k];
  for (int l = tid; l < pk; l += blockDim.x) {
    const double d = lam[l];
    int rank = 0;
    for (int j = 0; j < pk; ++j) rank += (lam[j] > d) || (lam[j] == d && j < l);
    rk[l] = rank;
    evals[off_k + rank] = d;
  }
  __syncthreads();
  for (int l = tid; l < pk; l += blockDim.x) {
    const double* col = V + (long long)l * pk;
    int imax = 0;
    double vmax = -1.0;
    for (int r = 0; r < pk; ++r)
      if (fabs(col[r]) > vmax) {
        vmax = fabs(col[r]);
        imax = r;
      }
    const double sg = col[imax] < 0.0 ? -1.0 : 1.0;
    double* out = evecs + base;
    for (int r = 0; r < pk; ++r) out[(long long)r * pk + rk[l]] = sg * col[r];
  }
}

size_t eig_workspace_bytes(const Plan& pl) { return (size_t)pl.cov_size * sizeof(double); }

static_assert((size_t)kEigLdsLimit / sizeof(double) < (size_t)(64 * kJacobiMaxPerLane) * (64 * kJacobiMaxPerLane),
              "the LDS form accumulates rotations for p_k <= 64 kJacobiMaxPerLane only");
static size_t eig_lds_bytes(const Plan& pl) {
  const int pm = *std::max_element(pl.p.begin(), pl.p.end());
  return ((size_t)pm * pm + pm) * sizeof(double);
}

hipError_t configure_eig_kernels() {
  return hipFuncSetAttribute((const void*)k_eig_lds, hipFuncAttributeMaxDynamicSharedMemorySize, kEigLdsLimit);
}

hipError_t launch_eig(const Plan& pl, const double* G, const double* S0, const float* shift, long long count,
                      double* evals, double* evecs, double* C_out, double* mean_out, double* work, hipStream_t st) {
  pl.prof.begin(ST_EIG, st);
  const size_t lds = eig_lds_bytes(pl);
  if (lds <= (size_t)kEigLdsLimit)
    hipLaunchKernelGGL(k_eig_lds, dim3((unsigned)(pl.k_max + 1)), dim3(EIG_THREADS), lds, st, G, S0, shift, count,
                       evals, evecs, C_out, mean_out, work, pl.d_p, pl.d_coef_off, pl.d_cov_off);
  else
    hipLaunchKernelGGL(k_eig, dim3((unsigned)(pl.k_max + 1)), dim3(EIG_THREADS), 0, st, G, S0, shift, count, evals,
                       evecs, C_out, mean_out, work, pl.d_p, pl.d_coef_off, pl.d_cov_off);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
