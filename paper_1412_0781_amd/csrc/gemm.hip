// The two dense contractions of the method on the gfx950 matrix cores:
//   radial quadrature Eq.(a):  A^(k) = B^(k) Fhat^(k)       (B^(k): p_k x n_xi, per angular frequency k)
//   covariance Eqs.(ck),(ck_0): G^(k) += Re(A^(k) A^(k)^*) = Ar Ar^T + Ai Ai^T
// and the transpose of the radial step used by the adjoint.
//
// Tiles are 64 x 64 per 256-thread workgroup (four wavefronts of 32 x 32).
// FP32 form: v_mfma_f32_32x32x2_f32.  BF16x3 form: every operand is split as
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi), and the product is
// hi*hi + hi*lo + lo*hi on v_mfma_f32_32x32x16_bf16, accumulated in FP32.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fb {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16;   // FP32 tiles
constexpr int BKH = 32;                    // BF16 K chunk
constexpr int LDH = BKH + 8;               // padded LDS row (80 bytes)

__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_to_f(hi));
}

__device__ __forceinline__ int acc_row(int i, int lane) { return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3); }

__device__ __forceinline__ void mma_f32(const float (*As)[BM + 4], const float (*Bs)[BN + 4], f32x16& acc, int wm,
                                        int wn, int lane) {
#pragma unroll
  for (int kk = 0; kk < BK; kk += 2) {
    float a = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
    float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
}

__device__ __forceinline__ bf16x8 ld8(const unsigned short* p) { return __builtin_bit_cast(bf16x8, *(const uint4*)p); }

__device__ __forceinline__ void mma_bf16x3(const unsigned short (*Ah)[LDH], const unsigned short (*Al)[LDH],
                                           const unsigned short (*Bh)[LDH], const unsigned short (*Bl)[LDH],
                                           f32x16& acc, int wm, int wn, int lane) {
  const int ra = wm * 32 + (lane & 31), rb = wn * 32 + (lane & 31);
#pragma unroll
  for (int kb = 0; kb < BKH; kb += 16) {
    const int c = kb + 8 * (lane >> 5);
    bf16x8 ah = ld8(&Ah[ra][c]), al = ld8(&Al[ra][c]);
    bf16x8 bh = ld8(&Bh[rb][c]), bl = ld8(&Bl[rb][c]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// radial quadrature.  grid: (column tiles of 64 = 32 images, work items (k, 128-row tile))
// Fh: float [K+1][n_xi][ncol], ncol = 2 * images (re, im interleaved)
// coeffs: float [image][p_half][2]
// A wave owns 32 rows x 64 columns (two 32x32 MFMA tiles).  The next K chunk is
// loaded into registers while the current one is multiplied from LDS; the output
// tile is transposed through LDS so that each image's rows are written as one run.
// ---------------------------------------------------------------------------
constexpr int RBM = 128, RBN = 64, RBK = 32;
constexpr int RLDH = RBK + 8;

template <int PREC>
struct RadialSmem;
template <>
struct RadialSmem<0> {
  float As[RBK][RBM + 4];
  float Bs[RBK][RBN + 4];
};
template <>
struct RadialSmem<1> {
  unsigned short Ah[RBM][RLDH], Al[RBM][RLDH];
  unsigned short Bh[RBN][RLDH], Bl[RBN][RLDH];
};
union RadialOut {
  float Cs[RBN][RBM + 4];
};

template <int PREC>
__global__ __launch_bounds__(256) void k_radial_fwd(const float* __restrict__ radial, const float* __restrict__ Fh,
                                                    float* __restrict__ coeffs, const GemmItem* __restrict__ items,
                                                    const int* __restrict__ coef_off, const int* __restrict__ p,
                                                    int n_xi, int ncol, long long p_half) {
  constexpr size_t SZ = sizeof(RadialSmem<PREC>) > sizeof(RadialOut) ? sizeof(RadialSmem<PREC>) : sizeof(RadialOut);
  __shared__ __attribute__((aligned(16))) unsigned char smem[SZ];
  RadialSmem<PREC>& S = *reinterpret_cast<RadialSmem<PREC>*>(smem);
  RadialOut& O = *reinterpret_cast<RadialOut*>(smem);
  const GemmItem it = items[blockIdx.y];
  const int k = it.k, m0 = it.t0, pk = p[k], off = coef_off[k];
  const int n0 = blockIdx.x * RBN;
  const int tid = threadIdx.x, lane = tid & 63, wm = tid >> 6;
  const float* fk = Fh + (size_t)k * n_xi * ncol;
  const bool vec = ((n_xi & 3) == 0) && ((ncol & 3) == 0);
  float4 ra[4], rb[2];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {  // A: 128 rows x 32 k, four consecutive k per thread
      int idx = tid + u * 256, m = idx >> 3, kq = (idx & 7) * 4;
      int row = m0 + m, kc = k0 + kq;
      const float* src = radial + (size_t)(off + row) * n_xi + kc;
      if (row < pk && vec && kc + 3 < n_xi) {
        ra[u] = *(const float4*)src;
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (row < pk && kc + e < n_xi) ? src[e] : 0.f;
        ra[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {  // B: 32 k x 64 columns, four consecutive columns per thread
      int idx = tid + u * 256, kk = idx >> 4, nq = (idx & 15) * 4;
      int kc = k0 + kk, col = n0 + nq;
      const float* src = fk + (size_t)kc * ncol + col;
      if (kc < n_xi && vec && col + 3 < ncol) {
        rb[u] = *(const float4*)src;
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (kc < n_xi && col + e < ncol) ? src[e] : 0.f;
        rb[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  auto lstore = [&]() {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int idx = tid + u * 256, m = idx >> 3, kq = (idx & 7) * 4;
      float v[4] = {ra[u].x, ra[u].y, ra[u].z, ra[u].w};
      if constexpr (PREC == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) S.As[kq + e][m] = v[e];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          unsigned short h, l;
          split_bf16(v[e], h, l);
          S.Ah[m][kq + e] = h;
          S.Al[m][kq + e] = l;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int idx = tid + u * 256, kk = idx >> 4, nq = (idx & 15) * 4;
      float v[4] = {rb[u].x, rb[u].y, rb[u].z, rb[u].w};
      if constexpr (PREC == 0) {
        *(float4*)&S.Bs[kk][nq] = rb[u];
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          unsigned short h, l;
          split_bf16(v[e], h, l);
          S.Bh[nq + e][kk] = h;
          S.Bl[nq + e][kk] = l;
        }
      }
    }
  };
  f32x16 acc0 = {}, acc1 = {};
  const int nch = (n_xi + RBK - 1) / RBK;
  gload(0);
  lstore();
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    if (c + 1 < nch) gload((c + 1) * RBK);
    if constexpr (PREC == 0) {
#pragma unroll
      for (int kk = 0; kk < RBK; kk += 2) {
        float a = S.As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
        float b0 = S.Bs[kk + (lane >> 5)][lane & 31];
        float b1 = S.Bs[kk + (lane >> 5)][32 + (lane & 31)];
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
      }
    } else {
      const int ra_ = wm * 32 + (lane & 31), rb0 = lane & 31, rb1 = 32 + (lane & 31);
#pragma unroll
      for (int kb = 0; kb < RBK; kb += 16) {
        const int cc = kb + 8 * (lane >> 5);
        bf16x8 ah = ld8(&S.Ah[ra_][cc]), al = ld8(&S.Al[ra_][cc]);
        bf16x8 bh0 = ld8(&S.Bh[rb0][cc]), bl0 = ld8(&S.Bl[rb0][cc]);
        bf16x8 bh1 = ld8(&S.Bh[rb1][cc]), bl1 = ld8(&S.Bl[rb1][cc]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh0, acc0, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl0, acc0, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh1, acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl1, acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh1, acc1, 0, 0, 0);
      }
    }
    __syncthreads();
    if (c + 1 < nch) {
      lstore();
      __syncthreads();
    }
  }
  // transpose the 128 x 64 tile through LDS: Cs[column][row]
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int r = wm * 32 + acc_row(i, lane);
    O.Cs[lane & 31][r] = acc0[i];
    O.Cs[32 + (lane & 31)][r] = acc1[i];
  }
  __syncthreads();
  const int nq = min(RBM, pk - m0);
  const int nimg_t = min(RBN, ncol - n0) / 2;
  for (int i = tid; i < nimg_t * nq; i += 256) {
    int il = i / nq, q = i - il * nq;
    float re = O.Cs[2 * il][q];
    float im = (k == 0) ? 0.f : O.Cs[2 * il + 1][q];
    *(float2*)&coeffs[(size_t)(n0 / 2 + il) * 2 * p_half + 2 * (size_t)(off + m0 + q)] = make_float2(re, im);
  }
}

// ---------------------------------------------------------------------------
// transpose of the radial step: D^(k)[j][col] = w_k sum_q B^(k)[q][j] X^(k)[q][col]
// grid: (column tiles, work items (k, j-tile)); FP32
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_radial_adj_f32(const float* __restrict__ radial,
                                                        const float* __restrict__ coeffs, float* __restrict__ D,
                                                        const GemmItem* __restrict__ items,
                                                        const int* __restrict__ coef_off, const int* __restrict__ p,
                                                        int n_xi, int ncol, long long p_half, int weight_mode) {
  __shared__ float As[BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  const GemmItem it = items[blockIdx.y];
  const int k = it.k, j0 = it.t0, pk = p[k], off = coef_off[k];
  const int n0 = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  f32x16 acc = {};
  for (int k0 = 0; k0 < pk; k0 += BK) {
    for (int i = tid; i < BM * BK; i += 256) {
      int kk = i / BM, m = i - kk * BM;
      int q = k0 + kk, j = j0 + m;
      As[kk][m] = (q < pk && j < n_xi) ? radial[(size_t)(off + q) * n_xi + j] : 0.f;
    }
    for (int i = tid; i < BK * BN; i += 256) {
      int il = i / (2 * BK), rem = i - il * 2 * BK, kk = rem >> 1, ri = rem & 1;
      int n = 2 * il + ri, q = k0 + kk, col = n0 + n;
      bool ok = q < pk && col < ncol && !(k == 0 && ri);
      Bs[kk][n] = ok ? coeffs[(size_t)(col >> 1) * 2 * p_half + 2 * (size_t)(off + q) + ri] : 0.f;
    }
    __syncthreads();
    mma_f32(As, Bs, acc, wm, wn, lane);
    __syncthreads();
  }
  const float wk = (k == 0 || weight_mode == 1) ? 1.f : 2.f;
  float* dk = D + (size_t)k * n_xi * ncol;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int j = j0 + wm * 32 + acc_row(i, lane), c = n0 + wn * 32 + (lane & 31);
    if (j < n_xi && c < ncol) dk[(size_t)j * ncol + c] = wk * acc[i];
  }
}

// ---------------------------------------------------------------------------
// covariance accumulation.  grid: work items (k, q-tile, q'-tile) with q'-tile >= q-tile.
// Each block runs over all n images; FP32 partial sums over 256 images are
// added into FP64 registers, then into G (and its mirror) in a fixed order.
// The k = 0 diagonal tiles also accumulate S0.
// ---------------------------------------------------------------------------
constexpr int COV_FLUSH_COLS = 512;

template <int PREC>
__global__ __launch_bounds__(256) void k_covariance(const float* __restrict__ coeffs, double* __restrict__ G,
                                                    double* __restrict__ S0, const GemmItem* __restrict__ items,
                                                    const int* __restrict__ coef_off, const int* __restrict__ p,
                                                    const long long* __restrict__ cov_off, long long n,
                                                    long long p_half) {
  // FP32 path uses As/Bs; BF16 path uses the hi/lo arrays
  __shared__ float As[PREC ? BKH : BK][BM + 4];
  __shared__ float Bs[BK][BN + 4];
  __shared__ __attribute__((aligned(16))) unsigned short Ah[PREC ? BM : 1][LDH];
  __shared__ __attribute__((aligned(16))) unsigned short Al[PREC ? BM : 1][LDH];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[PREC ? BN : 1][LDH];
  __shared__ __attribute__((aligned(16))) unsigned short Bl[PREC ? BN : 1][LDH];
  const GemmItem it = items[blockIdx.x];
  const int k = it.k, m0 = it.t0, n0 = it.t1, pk = p[k], off = coef_off[k];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  const bool do_sum = (k == 0 && m0 == n0);
  const long long ncol = 2 * n;
  const int bk = PREC ? BKH : BK;
  f32x16 acc = {};
  double dacc[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) dacc[i] = 0.0;
  float ssum = 0.f;
  double dsum = 0.0;
  int since_flush = 0;
  for (long long c0 = 0; c0 < ncol; c0 += bk) {
    // X[q][col] = coeffs[col/2][off + q][col%2]; the k = 0 imaginary parts are masked
    for (int i = tid; i < BM * bk; i += 256) {
      int il = i / (2 * BM), rem = i - il * 2 * BM, m = rem >> 1, ri = rem & 1;
      int kk = 2 * il + ri;
      long long col = c0 + kk;
      bool okc = col < ncol && !(k == 0 && ri);
      size_t base = (size_t)(col >> 1) * 2 * p_half + 2 * (size_t)off + ri;
      float xa = (okc && m0 + m < pk) ? coeffs[base + 2 * (size_t)(m0 + m)] : 0.f;
      float xb = (okc && n0 + m < pk) ? coeffs[base + 2 * (size_t)(n0 + m)] : 0.f;
      if (PREC) {
        unsigned short h, l;
        split_bf16(xa, h, l);
        Ah[m][kk] = h;
        Al[m][kk] = l;
        split_bf16(xb, h, l);
        Bh[m][kk] = h;
        Bl[m][kk] = l;
        if (do_sum) As[kk][m] = xa;  // exact values for the k = 0 sums
      } else {
        As[kk][m] = xa;
        Bs[kk][m] = xb;
      }
    }
    __syncthreads();
    if (PREC)
      mma_bf16x3(Ah, Al, Bh, Bl, acc, wm, wn, lane);
    else
      mma_f32(As, Bs, acc, wm, wn, lane);
    if (do_sum && tid < BM) {
      for (int kk = 0; kk < bk; kk += 2) ssum += As[kk][tid];
    }
    __syncthreads();
    since_flush += bk;
    if (since_flush >= COV_FLUSH_COLS) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        dacc[i] += (double)acc[i];
        acc[i] = 0.f;
      }
      dsum += (double)ssum;
      ssum = 0.f;
      since_flush = 0;
    }
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) dacc[i] += (double)acc[i];
  dsum += (double)ssum;
  double* gk = G + cov_off[k];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int q = m0 + wm * 32 + acc_row(i, lane), q2 = n0 + wn * 32 + (lane & 31);
    if (q < pk && q2 < pk) {
      gk[(size_t)q * pk + q2] += dacc[i];
      if (m0 != n0) gk[(size_t)q2 * pk + q] += dacc[i];
    }
  }
  if (do_sum && tid < BM && m0 + tid < pk) S0[m0 + tid] += dsum;
}

// ---------------------------------------------------------------------------
hipError_t launch_radial_forward(const Plan& pl, const float2* Fh, float* coeffs, int nimg, int precision,
                                 hipStream_t st) {
  const int ncol = 2 * nimg;
  dim3 g((unsigned)((ncol + RBN - 1) / RBN), (unsigned)pl.items_fwd.size());
  pl.prof.begin(ST_RADIAL_FWD, st);
  if (precision == FB_BF16X3)
    hipLaunchKernelGGL(k_radial_fwd<1>, g, dim3(256), 0, st, pl.d_radial, (const float*)Fh, coeffs, pl.d_items_fwd,
                       pl.d_coef_off, pl.d_p, pl.n_xi, ncol, (long long)pl.p_half);
  else
    hipLaunchKernelGGL(k_radial_fwd<0>, g, dim3(256), 0, st, pl.d_radial, (const float*)Fh, coeffs, pl.d_items_fwd,
                       pl.d_coef_off, pl.d_p, pl.n_xi, ncol, (long long)pl.p_half);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_radial_adjoint(const Plan& pl, const float* coeffs, float2* D, int nimg, int weight_mode,
                                 hipStream_t st) {
  const int ncol = 2 * nimg;
  dim3 g((unsigned)((ncol + BN - 1) / BN), (unsigned)pl.items_adj.size());
  pl.prof.begin(ST_RADIAL_ADJ, st);
  hipLaunchKernelGGL(k_radial_adj_f32, g, dim3(256), 0, st, pl.d_radial, coeffs, (float*)D, pl.d_items_adj,
                     pl.d_coef_off, pl.d_p, pl.n_xi, ncol, (long long)pl.p_half, weight_mode);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_covariance(const Plan& pl, const float* coeffs, long long n, double* G, double* S0, int precision,
                             hipStream_t st) {
  dim3 g((unsigned)pl.items_cov.size());
  pl.prof.begin(ST_COVARIANCE, st);
  if (precision == FB_BF16X3)
    hipLaunchKernelGGL(k_covariance<1>, g, dim3(256), 0, st, coeffs, G, S0, pl.d_items_cov, pl.d_coef_off,
                       pl.d_p, pl.d_cov_off, n, (long long)pl.p_half);
  else
    hipLaunchKernelGGL(k_covariance<0>, g, dim3(256), 0, st, coeffs, G, S0, pl.d_items_cov, pl.d_coef_off,
                       pl.d_p, pl.d_cov_off, n, (long long)pl.p_half);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
