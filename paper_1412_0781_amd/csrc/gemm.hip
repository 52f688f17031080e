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

#include <algorithm>

#include "dev_common.h"
#include "kernels.h"

namespace fb {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16;   // FP32 tiles
constexpr int BKH = 32;                    // BF16 K chunk
constexpr int LDH = BKH + 8;               // padded LDS row (80 bytes)

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// The BF16x3 operand split of two values at once, hi = bf16(x), lo = bf16(x - hi), both
// rounded to nearest even by the hardware conversion (v_cvt_pk_bf16_f32; x - hi is exact
// in FP32): hi and lo packed two per word, x0 in the low half.
__device__ __forceinline__ void split_bf16_pair(float x0, float x1, unsigned& hi, unsigned& lo) {
  const f32x2_t xv = {x0, x1};
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(xv, bf16x2_t));
  const f32x2_t rv = {x0 - __uint_as_float(hi << 16), x1 - __uint_as_float(hi & 0xffff0000u)};
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(rv, bf16x2_t));
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
// radial quadrature.  grid: (work items (k, 128-row tile), column tiles of 64 = 32 images)
// Fh: complex [group][n_xi][nk][16] (images in groups of 16, nk = K+1); as a real matrix
// per k, column 2 i + r (r = re, im) of row j sits at float
// ((group * n_xi + j) * nk + k) * 32 + (2 i + r) % 32.
// ncol = 2 * images.
// coeffs: float [image][p_half][2]
// A wave owns 32 rows x 64 columns (two 32x32 MFMA tiles).  The next K chunk is
// loaded into registers while the current one is multiplied from LDS; the output
// tile is transposed through LDS so that each image's rows are written as one run.
// The K loop starts at the chunk holding ring jmin[k]: on the rings before it every table
// entry of block k is below 2^-30 of its row's largest (J_k far below its turning point),
// and the angular step does not write F-hat there.  The workgroup barriers wait for LDS
// operations only, so the F-hat loads issued ahead stay in flight across them.
// ---------------------------------------------------------------------------
constexpr int RBM = 128, RBN = 64, RBK = 32;
constexpr int RLDH = RBK + 8;

// FP32 form, built like the BF16x3 form below.  Each v_mfma_f32_32x32x2f32 takes the pair
// j = (i, 16 + i) of the chunk in its two lane halves, so that a lane's table fragments
// for a chunk are 16 consecutive values of its row, loaded straight from global memory
// (tab: rows zero-padded to kRadialK); F-hat is staged in LDS as [j][column], its loads
// issued two chunks ahead.  Waves whose rows all lie beyond p_k skip loads and products.
__global__ __launch_bounds__(256) void k_radial_fwd_f32(const float* __restrict__ tab, const float* __restrict__ Fh,
                                                        float* __restrict__ coeffs, const GemmItem* __restrict__ items,
                                                        const int* __restrict__ coef_off, const int* __restrict__ p,
                                                        const int* __restrict__ jmin, int n_xi, int nxp, int nk,
                                                        int ncol, long long p_half, int weight_mode) {
  union Smem {
    float Bs[RBK][RBN + 4];      // F-hat chunk, [j][column]
    float Cs[RBN / 2][RBM + 4];  // half of the output tile, [column][row]
  };
  __shared__ __attribute__((aligned(16))) Smem S;
  const GemmItem it = items[blockIdx.x];
  const int k = it.k, m0 = it.t0, pk = p[k], off = coef_off[k], jm = jmin[k];
  const int n0 = blockIdx.y * RBN;
  const int tid = threadIdx.x, lane = tid & 63, wm = tid >> 6, hf = lane >> 5;
  const bool live = m0 + wm * 32 < pk;  // uniform over the wave
  const int row = m0 + wm * 32 + (lane & 31);
  const bool rlive = row < pk;
  const float* ta = tab + (size_t)(off + (rlive ? row : 0)) * nxp + 16 * hf;
  // F-hat staging: thread -> rows j = 2 jp, 2 jp + 1 of the chunk, columns nq .. nq + 3
  const int jp = tid & 15, nq = 4 * (tid >> 4), col = n0 + nq;
  const float* fk = Fh + (size_t)k * (2 * kImgGroup) +
                    (size_t)(col / (2 * kImgGroup)) * n_xi * nk * (2 * kImgGroup) + (col & (2 * kImgGroup - 1));
  float4 a_cu[4];       // this lane's 16 table values of the chunk
  float4 b1[2], b2[2];  // F-hat of the next chunk and of the one after
#pragma unroll
  for (int u = 0; u < 4; ++u) a_cu[u] = make_float4(0.f, 0.f, 0.f, 0.f);
  auto load_a = [&](int k0) {
    if (live && rlive) {
#pragma unroll
      for (int u = 0; u < 4; ++u) a_cu[u] = *(const float4*)(ta + k0 + 4 * u);
    }
  };
  auto load_b = [&](int k0, float4* dst) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kc = k0 + 2 * jp + u;
      const float* src = fk + (size_t)kc * nk * (2 * kImgGroup);
      const bool ring = kc >= jm && kc < n_xi;  // rings before jmin[k] hold no F-hat for this k
      if (ring && col + 3 < ncol) {
        dst[u] = *(const float4*)src;
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (ring && col + e < ncol) ? src[e] : 0.f;
        dst[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  auto lstore = [&]() {
    *(float4*)&S.Bs[2 * jp][nq] = b1[0];
    *(float4*)&S.Bs[2 * jp + 1][nq] = b1[1];
  };
  f32x16 acc0 = {}, acc1 = {};
  const int nch = nxp / RBK;
  const int cb = jm / RBK;  // the chunks before the one holding ring jmin[k] add nothing
  load_b(cb * RBK, b1);
  load_a(cb * RBK);
  lstore();
  if (cb + 1 < nch) load_b((cb + 1) * RBK, b1);
  lds_barrier();
  for (int c = cb; c < nch; ++c) {
    if (c + 2 < nch) load_b((c + 2) * RBK, b2);
    if (live) {
      const float av[16] = {a_cu[0].x, a_cu[0].y, a_cu[0].z, a_cu[0].w, a_cu[1].x, a_cu[1].y, a_cu[1].z, a_cu[1].w,
                            a_cu[2].x, a_cu[2].y, a_cu[2].z, a_cu[2].w, a_cu[3].x, a_cu[3].y, a_cu[3].z, a_cu[3].w};
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float bv0 = S.Bs[16 * hf + i][lane & 31], bv1 = S.Bs[16 * hf + i][32 + (lane & 31)];
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv1, acc1, 0, 0, 0);
      }
    }
    if (c + 1 < nch) load_a((c + 1) * RBK);
    lds_barrier();
    if (c + 1 < nch) {
      lstore();
      b1[0] = b2[0];
      b1[1] = b2[1];
      lds_barrier();
    }
  }
  // the 128 x 64 tile leaves through LDS in two halves of 32 columns: Cs[column][row]
  const int nrow = min(RBM, pk - m0);
  const float wk = (weight_mode == 0 && k > 0) ? 2.f : 1.f;  // +-k fold weight (exact)
  auto emit = [&](const f32x16& acc, int half) {
#pragma unroll
    for (int i = 0; i < 16; ++i) S.Cs[lane & 31][wm * 32 + acc_row(i, lane)] = acc[i];
    lds_barrier();
    const int c0 = n0 + 32 * half;
    const int nimg_t = max(0, min(32, ncol - c0)) / 2;
    for (int i = tid; i < nimg_t * nrow; i += 256) {
      const int il = i / nrow, q = i - il * nrow;
      const float re = S.Cs[2 * il][q];
      const float im = (k == 0) ? 0.f : S.Cs[2 * il + 1][q];
      st_out((float2*)&coeffs[(size_t)(c0 / 2 + il) * 2 * p_half + 2 * (size_t)(off + m0 + q)],
             make_float2(wk * re, wk * im));
    }
  };
  emit(acc0, 0);
  lds_barrier();
  emit(acc1, 1);
}

// BF16x3 form of the radial quadrature.  The table operand is split once, at plan time
// (tab: hi parts, then lo parts, rows padded to kRadialK with zeros), and each lane loads
// its 8-value MFMA fragments straight from global memory: a wave's 32 rows are its own.
// Only the F-hat operand, which the four waves share, is split here and staged in LDS,
// two consecutive j of one column packed into each 32-bit store, its global loads issued
// two chunks ahead.  Waves whose rows all lie
// beyond p_k skip their loads and products.  Same grid and output as k_radial_fwd_f32.
__global__ __launch_bounds__(256) void k_radial_fwd_b3(const unsigned short* __restrict__ tab,
                                                       const float* __restrict__ Fh, float* __restrict__ coeffs,
                                                       const GemmItem* __restrict__ items,
                                                       const int* __restrict__ coef_off, const int* __restrict__ p,
                                                       const int* __restrict__ jmin, int n_xi, int nxp, int nk,
                                                       int ncol, long long p_half, int weight_mode) {
  union Smem {
    struct {
      unsigned int Bh[RBN][RLDH / 2], Bl[RBN][RLDH / 2];  // [column][j / 2], two BF16 per word
    } b;
    float Cs[RBN / 2][RBM + 4];  // half of the output tile, [column][row]
  };
  __shared__ __attribute__((aligned(16))) Smem S;
  const GemmItem it = items[blockIdx.x];
  const int k = it.k, m0 = it.t0, pk = p[k], off = coef_off[k], jm = jmin[k];
  const int n0 = blockIdx.y * RBN;
  const int tid = threadIdx.x, lane = tid & 63, wm = tid >> 6;
  const bool live = m0 + wm * 32 < pk;  // uniform over the wave
  const int row = m0 + wm * 32 + (lane & 31);
  const bool rlive = row < pk;
  const size_t plane = (size_t)p_half * nxp;
  const unsigned short* th = tab + (size_t)(off + (rlive ? row : 0)) * nxp + 8 * (lane >> 5);
  // F-hat staging: thread -> rows j = 2 jp, 2 jp + 1 of the chunk, columns nq .. nq + 3
  const int jp = tid & 15, nq = 4 * (tid >> 4), col = n0 + nq;
  const float* fk = Fh + (size_t)k * (2 * kImgGroup) +
                    (size_t)(col / (2 * kImgGroup)) * n_xi * nk * (2 * kImgGroup) + (col & (2 * kImgGroup - 1));
  uint4 a_cu[4];        // A fragments: hi (j0, j0 + 16), lo (j0, j0 + 16)
  float4 b1[2], b2[2];  // F-hat of the next chunk and of the one after
#pragma unroll
  for (int u = 0; u < 4; ++u) a_cu[u] = make_uint4(0u, 0u, 0u, 0u);
  // the next chunk's fragments are loaded into the same registers once this chunk's
  // products have been issued; their latency overlaps the barrier and the F-hat staging
  auto load_a = [&](int k0) {
    if (live && rlive) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const unsigned short* src = th + (size_t)h * plane + k0;
        a_cu[2 * h] = *(const uint4*)src;
        a_cu[2 * h + 1] = *(const uint4*)(src + 16);
      }
    }
  };
  auto load_b = [&](int k0, float4* dst) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kc = k0 + 2 * jp + u;
      const float* src = fk + (size_t)kc * nk * (2 * kImgGroup);
      const bool ring = kc >= jm && kc < n_xi;  // rings before jmin[k] hold no F-hat for this k
      if (ring && col + 3 < ncol) {
        dst[u] = *(const float4*)src;
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (ring && col + e < ncol) ? src[e] : 0.f;
        dst[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  auto lstore = [&]() {
    const float v0[4] = {b1[0].x, b1[0].y, b1[0].z, b1[0].w};
    const float v1[4] = {b1[1].x, b1[1].y, b1[1].z, b1[1].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      unsigned h, l;
      split_bf16_pair(v0[e], v1[e], h, l);
      S.b.Bh[nq + e][jp] = h;
      S.b.Bl[nq + e][jp] = l;
    }
  };
  f32x16 acc0 = {}, acc1 = {};
  const int nch = nxp / RBK;
  const int cb = jm / RBK;  // the chunks before the one holding ring jmin[k] add nothing
  load_b(cb * RBK, b1);
  load_a(cb * RBK);
  lstore();
  if (cb + 1 < nch) load_b((cb + 1) * RBK, b1);
  lds_barrier();
  const unsigned short* Bh = (const unsigned short*)&S.b.Bh[0][0];
  const unsigned short* Bl = (const unsigned short*)&S.b.Bl[0][0];
  for (int c = cb; c < nch; ++c) {
    if (c + 2 < nch) load_b((c + 2) * RBK, b2);
    if (live) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const int cc = 16 * kb + 8 * (lane >> 5);
        const bf16x8 ah = __builtin_bit_cast(bf16x8, a_cu[kb]), al = __builtin_bit_cast(bf16x8, a_cu[2 + kb]);
        const int r0 = (lane & 31) * RLDH + cc, r1 = (32 + (lane & 31)) * RLDH + cc;
        const bf16x8 bh0 = ld8(Bh + r0), bl0 = ld8(Bl + r0), bh1 = ld8(Bh + r1), bl1 = ld8(Bl + r1);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh0, acc0, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl0, acc0, 0, 0, 0);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh1, acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl1, acc1, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh1, acc1, 0, 0, 0);
      }
    }
    if (c + 1 < nch) load_a((c + 1) * RBK);
    lds_barrier();
    if (c + 1 < nch) {
      lstore();
      b1[0] = b2[0];
      b1[1] = b2[1];
      lds_barrier();
    }
  }
  // the 128 x 64 tile leaves through LDS in two halves of 32 columns: Cs[column][row]
  const int nrow = min(RBM, pk - m0);
  const float wk = (weight_mode == 0 && k > 0) ? 2.f : 1.f;  // +-k fold weight (exact)
  auto emit = [&](const f32x16& acc, int half) {
#pragma unroll
    for (int i = 0; i < 16; ++i) S.Cs[lane & 31][wm * 32 + acc_row(i, lane)] = acc[i];
    lds_barrier();
    const int c0 = n0 + 32 * half;
    const int nimg_t = max(0, min(32, ncol - c0)) / 2;
    for (int i = tid; i < nimg_t * nrow; i += 256) {
      const int il = i / nrow, q = i - il * nrow;
      const float re = S.Cs[2 * il][q];
      const float im = (k == 0) ? 0.f : S.Cs[2 * il + 1][q];
      st_out((float2*)&coeffs[(size_t)(c0 / 2 + il) * 2 * p_half + 2 * (size_t)(off + m0 + q)],
             make_float2(wk * re, wk * im));
    }
  };
  emit(acc0, 0);
  lds_barrier();
  emit(acc1, 1);
}

// ---------------------------------------------------------------------------
// transpose of the radial step: D^(k)[j][col] = w_k sum_q B^(k)[q][j] X^(k)[q][col]
// grid: (runs of kAdjBlocks column tiles of 32 images, work items (k, j-tile)); FP32.
// PANEL: the item's table panel (all p_k rows of its 64 rings) sits in LDS for the whole
// run; otherwise it is read per chunk of 16 rows (blocks above the panel's capacity).  An
// image's block-k coefficients are one contiguous run, read as (re, im) pairs along q with
// the next chunk in flight.
// ---------------------------------------------------------------------------
constexpr int kAdjBlocks = 8;
template <bool PANEL>
__global__ __launch_bounds__(256) void k_radial_adj_f32(const float* __restrict__ radial,
                                                        const float* __restrict__ coeffs, float* __restrict__ D,
                                                        const GemmItem* __restrict__ items,
                                                        const int* __restrict__ coef_off, const int* __restrict__ p,
                                                        int n_xi, int nk, int ncol, long long p_half,
                                                        int weight_mode, const float* __restrict__ ring_filter) {
  extern __shared__ float adj_lds[];
  float(*Bs)[BN + 4] = (float(*)[BN + 4])adj_lds;                   // BK rows: coefficients
  float(*As)[BM + 4] = (float(*)[BM + 4])(adj_lds + BK * (BN + 4));  // table rows
  const GemmItem it = items[blockIdx.y];
  const int k = it.k, j0 = it.t0, pk = p[k], off = coef_off[k];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  auto load_a = [&](int r0, int nr) {  // table rows r0 .. r0 + nr - 1 into As[0 ..] (PANEL: As[r0 ..])
    for (int i = tid; i < BM * nr; i += 256) {
      const int kk = i / BM, m = i - kk * BM;
      const int q = r0 + kk, j = j0 + m;
      As[(PANEL ? r0 : 0) + kk][m] = (q < pk && j < n_xi) ? radial[(size_t)(off + q) * n_xi + j] : 0.f;
    }
  };
  if (PANEL) {
    load_a(0, (pk + BK - 1) / BK * BK);
    __syncthreads();
  }
  const float wk = (k == 0 || weight_mode == 1) ? 1.f : 2.f;
  const int nimg = ncol / 2;
  const int bi = tid >> 3, bq = 2 * (tid & 7);  // coefficient loads: image bi of the block, q = k0 + bq + {0, 1}
  for (int blk = 0; blk < kAdjBlocks; ++blk) {
    const int n0 = (blockIdx.x * kAdjBlocks + blk) * BN;
    if (n0 >= ncol) break;
    const int img = n0 / 2 + bi;
    const float2* brow = (const float2*)(coeffs + (size_t)min(img, nimg - 1) * 2 * p_half) + off;
    float2 pb[2];
    auto fetch = [&](int k0) {  // unconditional (clamped to the block): stays in flight
#pragma unroll
      for (int h = 0; h < 2; ++h) pb[h] = brow[min(k0 + bq + h, pk - 1)];
    };
    fetch(0);
    f32x16 acc = {};
    for (int k0 = 0; k0 < pk; k0 += BK) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = k0 + bq + h;
        float2 v = (img < nimg && q < pk) ? pb[h] : make_float2(0.f, 0.f);
        if (k == 0) v.y = 0.f;  // the k = 0 coefficients are real
        *(float2*)&Bs[bq + h][2 * bi] = v;
      }
      if (!PANEL) load_a(k0, BK);
      __syncthreads();
      if (k0 + BK < pk) fetch(k0 + BK);
      const int a0 = PANEL ? k0 : 0;
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        const float a = As[a0 + kk + (lane >> 5)][wm * 32 + (lane & 31)];
        const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
      __syncthreads();
    }
    // D grouped like the forward spectrum: [image group][ring j][k][16 images] complex, so
    // that a (ring, group) unit of the angular step reads one contiguous run
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int j = j0 + wm * 32 + acc_row(i, lane), c = n0 + wn * 32 + (lane & 31);
      if (j < n_xi && c < ncol) {
        const int im = c >> 1;
        const float h = ring_filter ? ring_filter[j] : 1.f;  // radial filter H(xi_j), if any
        D[((((size_t)(im / kImgGroup) * n_xi + j) * nk + k) * kImgGroup + (im & (kImgGroup - 1))) * 2 + (c & 1)] =
            h * (wk * acc[i]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// covariance accumulation (Eqs.(ck),(ck_0)), split over image slices.
// grid: work items x S image slices; a work item stages up to kCovSegs segments of 32
// coefficients (rows) for every chunk of images and each of its kCovWaves waves forms one
// 32 x 32 tile: the product of two segments of the same block k (eight waves of at most 128
// registers: two workgroups per compute unit; the Hermitian form takes more registers and
// runs one).  The K dimension is
// (image, re/im): X[q][2i + r] = (Re, Im) a^i_{kq}, so Re(A A^*) = X X^T.  A K chunk is
// 16 images = 32 columns; the next chunk is held in registers while the current one is
// multiplied (the workgroup barriers wait for LDS operations only, so those loads stay in
// flight across them).  In the BF16x3 form each thread stores the hi and lo parts of four
// consecutive images of its row as two 16-byte runs, which keeps the stores free of LDS
// bank conflicts.  FP32 tile sums are moved to FP64 registers every COV_FLUSH_COLS
// columns; each wave writes its FP64 tile (and the mirrored tile) into its slice's partial
// copy of G, which k_cov_reduce then adds into G in slice order, so the result does not
// depend on scheduling.
// The k = 0 imaginary parts are masked and the k = 0 rows also sum S0 (in the item that
// owns the segment's sums).  With a shift s (FP32 [p_0]) the k = 0 rows enter as
// a_{0q} - s_q, before the BF16 split, so the sums stay of the order of the spread of the
// data rather than of its mean.
// HERM also forms the imaginary part of A A^* for k > 0 (the Hermitian covariance
// under rotations only): Im(A A^*) = Ai Ar^T - Ar Ai^T = X Y^T with the second operand
// taken as Y[q][2i] = -Im a^i_{kq}, Y[q][2i + 1] = Re a^i_{kq}: one more product per
// chunk from the same staged rows.
// ---------------------------------------------------------------------------
constexpr int COV_FLUSH_COLS = 512;
constexpr int COV_IMG = 16;                 // images per K chunk
constexpr int COV_K = 2 * COV_IMG;          // columns per K chunk
constexpr int COV_ROWS = kCovSegs * kCovSeg;  // staged rows per item
constexpr int COV_THREADS = 64 * kCovWaves;
static_assert(COV_K == BKH, "BF16 tiles hold one K chunk");
static_assert(kCovSeg == 32, "one 32 x 32 MFMA tile per wave");
static_assert(COV_THREADS == 4 * COV_ROWS, "four loader threads (four images each) per staged row");

template <int PREC>
struct CovSmem;
template <>
struct CovSmem<0> {
  float As[COV_K][COV_ROWS + 4];
};
template <>
struct CovSmem<1> {
  unsigned short Ah[COV_ROWS][LDH], Al[COV_ROWS][LDH];
};

// rows ra0.. and rb0.. of the staged chunk (32 each): acc += X_a X_b^T
__device__ __forceinline__ void mma_f32_k32(const float (*As)[COV_ROWS + 4], f32x16& acc, int ra0, int rb0,
                                            int lane) {
#pragma unroll
  for (int kk = 0; kk < COV_K; kk += 2) {
    float a = As[kk + (lane >> 5)][ra0 + (lane & 31)];
    float b = As[kk + (lane >> 5)][rb0 + (lane & 31)];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
}

// X_a Y_b^T with Y[2i] = -X[2i + 1], Y[2i + 1] = X[2i] on the second operand (FP32 form)
__device__ __forceinline__ void mma_f32_k32_im(const float (*As)[COV_ROWS + 4], f32x16& acc, int ra0, int rb0,
                                               int lane) {
  const int h = lane >> 5;
#pragma unroll
  for (int kk = 0; kk < COV_K; kk += 2) {
    float a = As[kk + h][ra0 + (lane & 31)];
    float b = As[kk + 1 - h][rb0 + (lane & 31)];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, h ? b : -b, acc, 0, 0, 0);
  }
}

// (re, im) BF16 pairs of a fragment -> (-im, re): swap the halves of each word, negate the low one
__device__ __forceinline__ bf16x8 swap_neg_pairs(bf16x8 x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x = ((u.x >> 16) | (u.x << 16)) ^ 0x8000u;
  u.y = ((u.y >> 16) | (u.y << 16)) ^ 0x8000u;
  u.z = ((u.z >> 16) | (u.z << 16)) ^ 0x8000u;
  u.w = ((u.w >> 16) | (u.w << 16)) ^ 0x8000u;
  return __builtin_bit_cast(bf16x8, u);
}

// BF16x3 products of the real part (acc) and, when im, of the imaginary part (acc_im)
template <bool IM>
__device__ __forceinline__ void mma_bf16x3_cov(const unsigned short (*Ah)[LDH], const unsigned short (*Al)[LDH],
                                               f32x16& acc, f32x16& acc_im, bool im, int ra0, int rb0, int lane) {
  const int ra = ra0 + (lane & 31), rb = rb0 + (lane & 31);
#pragma unroll
  for (int kb = 0; kb < BKH; kb += 16) {
    const int c = kb + 8 * (lane >> 5);
    bf16x8 ah = ld8(&Ah[ra][c]), al = ld8(&Al[ra][c]);
    bf16x8 bh = ld8(&Ah[rb][c]), bl = ld8(&Al[rb][c]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    if (IM && im) {
      const bf16x8 yh = swap_neg_pairs(bh), yl = swap_neg_pairs(bl);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, yh, acc_im, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, yl, acc_im, 0, 0, 0);
      acc_im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, yh, acc_im, 0, 0, 0);
    }
  }
}

template <int PREC, bool HERM>
__global__ __launch_bounds__(COV_THREADS, HERM ? 1 : 4) void k_covariance(const float* __restrict__ coeffs,
                                                            double* __restrict__ partG, double* __restrict__ partS0,
                                                            double* __restrict__ partGi,
                                                            const float* __restrict__ shift,
                                                            const CovItem* __restrict__ items,
                                                            const int* __restrict__ p,
                                                            const long long* __restrict__ cov_off, long long n,
                                                            long long p_half, int nitems, long long per,
                                                            long long cov_size, int p0) {
  __shared__ __attribute__((aligned(16))) CovSmem<PREC> S;
  __shared__ double dred[4][COV_ROWS];
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int itx = lin % nitems, slice = lin / nitems;  // items of neighbouring k are neighbours on one XCD
  const CovItem& it = items[itx];
  const long long i0 = (long long)slice * per, i1 = min(n, i0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // loader: thread owns staged row `row` (segment sg, row r of it) for the four consecutive
  // images 4 ib + u, u < 4, of each chunk (one 16-byte LDS store per part in the BF16x3 form)
  const int row = tid % COV_ROWS, ib = tid / COV_ROWS, sg = row / kCovSeg, r = row % kCovSeg;
  const int kr = it.k[sg];
  const bool valid = kr >= 0 && it.q0[sg] + r < p[max(kr, 0)];
  const bool k0r = (kr == 0);
  const bool do_sum = k0r && it.sum0[sg] && valid;
  const float2* src = (const float2*)coeffs + it.row[sg] + r;
  // k = 0 rows enter shifted (rows past p_0 and images past the run stay exactly zero)
  const float sh = (k0r && shift && valid) ? shift[it.q0[sg] + r] : 0.f;
  // this wave's tile: segments ta <= tb of block kt
  const int ta = it.ta[wave], tb = it.tb[wave];
  const bool has = ta != 255;
  const int kt = has ? it.k[ta] : 0;
  const bool im = HERM && has && kt != 0;  // the imaginary part of a k = 0 block is zero
  auto gload = [&](long long c0, float2 (&R)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      long long img = c0 + 4 * ib + u;
      bool ok = img < i1 && valid;
      R[u] = ok ? src[img * p_half] : make_float2(0.f, 0.f);
      if (k0r) {
        if (ok) R[u].x -= sh;
        R[u].y = 0.f;
      }
    }
  };
  float ssum = 0.f;
  auto lstore = [&](const float2 (&R)[4]) {
    if constexpr (PREC == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = 2 * (4 * ib + u);
        if (do_sum) ssum += R[u].x;
        S.As[col][row] = R[u].x;
        S.As[col + 1][row] = R[u].y;
      }
    } else {
      // columns 8 ib .. 8 ib + 7 of the row: four (re, im) pairs, hi and lo, 16 bytes each
      uint4 h4, l4;
      unsigned* h = (unsigned*)&h4;
      unsigned* l = (unsigned*)&l4;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (do_sum) ssum += R[u].x;
        split_bf16_pair(R[u].x, R[u].y, h[u], l[u]);
      }
      *(uint4*)&S.Ah[row][8 * ib] = h4;
      *(uint4*)&S.Al[row][8 * ib] = l4;
    }
  };
  f32x16 acc = {}, acc_im = {};
  double dacc[16], dacc_im[HERM ? 16 : 1];
#pragma unroll
  for (int i = 0; i < 16; ++i) dacc[i] = 0.0;
  if constexpr (HERM) {
#pragma unroll
    for (int i = 0; i < 16; ++i) dacc_im[i] = 0.0;
  }
  double dsum = 0.0;
  int since_flush = 0;
  const int ra0 = ta * kCovSeg, rb0 = tb * kCovSeg;
  // chunk c0 is staged from R, then the loads of the next chunk go into R and stay in flight
  // through the products (the barriers wait for LDS operations only)
  auto step = [&](long long c0, float2 (&R)[4]) {
    lstore(R);
    lds_barrier();
    if (c0 + COV_IMG < i1) gload(c0 + COV_IMG, R);
    if (has) {
      if constexpr (PREC == 0) {
        mma_f32_k32(S.As, acc, ra0, rb0, lane);
        if (HERM && im) mma_f32_k32_im(S.As, acc_im, ra0, rb0, lane);
      } else {
        mma_bf16x3_cov<HERM>(S.Ah, S.Al, acc, acc_im, im, ra0, rb0, lane);
      }
    }
    lds_barrier();
    since_flush += COV_K;
    if (since_flush >= COV_FLUSH_COLS) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        dacc[i] += (double)acc[i];
        acc[i] = 0.f;
      }
      if constexpr (HERM) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          dacc_im[i] += (double)acc_im[i];
          acc_im[i] = 0.f;
        }
      }
      dsum += (double)ssum;
      ssum = 0.f;
      since_flush = 0;
    }
  };
  float2 R0[4];
  gload(i0, R0);
  for (long long c0 = i0; c0 < i1; c0 += COV_IMG) step(c0, R0);
#pragma unroll
  for (int i = 0; i < 16; ++i) dacc[i] += (double)acc[i];
  if constexpr (HERM) {
#pragma unroll
    for (int i = 0; i < 16; ++i) dacc_im[i] += (double)acc_im[i];
  }
  dsum += (double)ssum;
  if (has) {
    const int pk = p[kt], ma = it.q0[ta], nb = it.q0[tb];
    const bool diag = (ta == tb);
    double* gk = partG + (size_t)slice * cov_size + cov_off[kt];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int rr = ma + acc_row(i, lane), cc = nb + (lane & 31);
      if (rr < pk && cc < pk) {
        gk[(size_t)rr * pk + cc] = dacc[i];
        if (!diag) gk[(size_t)cc * pk + rr] = dacc[i];
      }
    }
    if constexpr (HERM) {
      // the imaginary part is antisymmetric: every value is written at (r, c) with r < c and
      // negated at (c, r), the diagonal as zero (a diagonal tile keeps its upper triangle)
      double* gi = partGi + (size_t)slice * cov_size + cov_off[kt];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        int rr = ma + acc_row(i, lane), cc = nb + (lane & 31);
        if (rr < pk && cc < pk && rr <= cc) {
          const double v = (rr == cc) ? 0.0 : dacc_im[i];
          gi[(size_t)rr * pk + cc] = v;
          gi[(size_t)cc * pk + rr] = -v;
        }
      }
    }
  }
  // the four loader threads of a k = 0 row hold FP64 sums of disjoint images
  dred[ib][row] = dsum;
  __syncthreads();
  if (tid < COV_ROWS) {
    const int s2 = tid / kCovSeg, r2 = tid % kCovSeg;
    if (it.k[s2] == 0 && it.sum0[s2] && it.q0[s2] + r2 < p0)
      partS0[(size_t)slice * p0 + it.q0[s2] + r2] = ((dred[0][tid] + dred[1][tid]) + dred[2][tid]) + dred[3][tid];
  }
}

// G[i] += sum over slices s = 0..S-1 (in that order) of partG[s][i]; the same for S0
// and, when partGi is given, for Gi.
__global__ void k_cov_reduce(const double* __restrict__ partG, const double* __restrict__ partS0,
                             const double* __restrict__ partGi, int S, long long cov_size, int p0,
                             double* __restrict__ G, double* __restrict__ S0, double* __restrict__ Gi) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cov_size) {
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += partG[(size_t)s * cov_size + i];
    G[i] += t;
    if (partGi) {
      double u = 0.0;
      for (int s = 0; s < S; ++s) u += partGi[(size_t)s * cov_size + i];
      Gi[i] += u;
    }
  } else if (i < cov_size + p0) {
    const int m = (int)(i - cov_size);
    double t = 0.0;
    for (int s = 0; s < S; ++s) t += partS0[(size_t)s * p0 + m];
    S0[m] += t;
  }
}

// shift[q] = mean of a_{0,q} over the first m images (FP64 sum in image order), rounded to FP32
__global__ void k_cov_shift(const float* __restrict__ coeffs, int m, long long p_half, int p0,
                            float* __restrict__ shift) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= p0) return;
  // eight loads in flight, added in image order
  double t = 0.0;
  int i = 0;
  for (; i + 8 <= m; i += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = coeffs[2 * ((size_t)(i + u) * p_half + q)];
#pragma unroll
    for (int u = 0; u < 8; ++u) t += (double)v[u];
  }
  for (; i < m; ++i) t += (double)coeffs[2 * ((size_t)i * p_half + q)];
  shift[q] = (float)(t / m);
}

// ---------------------------------------------------------------------------
hipError_t launch_radial_forward(const Plan& pl, const float2* Fh, float* coeffs, int nimg, int precision,
                                 int weight_mode, hipStream_t st) {
  const int ncol = 2 * nimg;
  dim3 g((unsigned)pl.items_fwd.size(), (unsigned)((ncol + RBN - 1) / RBN));
  const int nk = pl.k_max + 1;
  pl.prof.begin(ST_RADIAL_FWD, st);
  if (precision == FB_BF16X3) {
    hipLaunchKernelGGL(k_radial_fwd_b3, g, dim3(256), 0, st, pl.d_radial_bf, (const float*)Fh, coeffs,
                       pl.d_items_fwd, pl.d_coef_off, pl.d_p, pl.d_jmin, pl.n_xi, pl.n_xi_pad, nk, ncol,
                       (long long)pl.p_half, weight_mode);
  } else {
    hipLaunchKernelGGL(k_radial_fwd_f32, g, dim3(256), 0, st, pl.d_radial_pad, (const float*)Fh, coeffs,
                       pl.d_items_fwd, pl.d_coef_off, pl.d_p, pl.d_jmin, pl.n_xi, pl.n_xi_pad, nk, ncol,
                       (long long)pl.p_half, weight_mode);
  }
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_radial_adjoint(const Plan& pl, const float* coeffs, float2* D, int nimg, int weight_mode,
                                 const float* ring_filter, hipStream_t st) {
  const int ncol = 2 * nimg;
  const int tiles = (ncol + BN - 1) / BN;
  dim3 g((unsigned)((tiles + kAdjBlocks - 1) / kAdjBlocks), (unsigned)pl.items_adj.size());
  int pmax = 0;
  for (int v : pl.p) pmax = std::max(pmax, v);
  const int rows = (pmax + BK - 1) / BK * BK;
  // table panel resident while the kernel's LDS stays within 64 KB (p_k <= 224)
  const bool panel = (size_t)(BK * (BN + 4) + rows * (BM + 4)) * sizeof(float) <= 64u * 1024u;
  const size_t lds = (size_t)(BK * (BN + 4) + (panel ? rows : BK) * (BM + 4)) * sizeof(float);
  pl.prof.begin(ST_RADIAL_ADJ, st);
  if (panel)
    hipLaunchKernelGGL(k_radial_adj_f32<true>, g, dim3(256), lds, st, pl.d_radial, coeffs, (float*)D,
                       pl.d_items_adj, pl.d_coef_off, pl.d_p, pl.n_xi, pl.k_max + 1, ncol, (long long)pl.p_half,
                       weight_mode, ring_filter);
  else
    hipLaunchKernelGGL(k_radial_adj_f32<false>, g, dim3(256), lds, st, pl.d_radial, coeffs, (float*)D,
                       pl.d_items_adj, pl.d_coef_off, pl.d_p, pl.n_xi, pl.k_max + 1, ncol, (long long)pl.p_half,
                       weight_mode, ring_filter);
  pl.prof.end(st);
  return hipGetLastError();
}

CovSplit cov_split(const Plan& pl, long long n, bool hermitian) {
  CovSplit sp{};
  if (n <= 0) return sp;
  long long S = std::min<long long>(kCovMaxSlices, std::max<long long>(1, (n + kCovSliceImages - 1) / kCovSliceImages));
  long long per = (n + S - 1) / S;
  per = (per + COV_IMG - 1) / COV_IMG * COV_IMG;
  sp.per = per;
  sp.slices = (int)((n + per - 1) / per);
  sp.bytes_g = (size_t)sp.slices * pl.cov_size * sizeof(double);
  sp.bytes_gi = hermitian ? sp.bytes_g : 0;
  sp.bytes = sp.bytes_g + sp.bytes_gi + (size_t)sp.slices * pl.p0 * sizeof(double);
  return sp;
}

hipError_t launch_cov_shift(const Plan& pl, const float* coeffs, long long n, float* shift, hipStream_t st) {
  const int m = (int)std::min<long long>(n, kCovShiftImages);
  hipLaunchKernelGGL(k_cov_shift, dim3((unsigned)((pl.p0 + 255) / 256)), dim3(256), 0, st, coeffs, m,
                     (long long)pl.p_half, pl.p0, shift);
  return hipGetLastError();
}

hipError_t launch_covariance(const Plan& pl, const float* coeffs, long long n, double* G, double* S0, double* Gi,
                             const float* shift, int precision, void* ws, hipStream_t st) {
  const bool herm = Gi != nullptr;
  const CovSplit sp = cov_split(pl, n, herm);
  const int nitems = (int)pl.items_cov.size();
  double* partG = (double*)ws;
  double* partGi = herm ? (double*)((char*)ws + sp.bytes_g) : nullptr;
  double* partS0 = (double*)((char*)ws + sp.bytes_g + sp.bytes_gi);
  dim3 g((unsigned)(nitems * sp.slices));
  pl.prof.begin(ST_COVARIANCE, st);
#define FB_COV(P, H)                                                                                              \
  hipLaunchKernelGGL((k_covariance<P, H>), g, dim3(COV_THREADS), 0, st, coeffs, partG, partS0, partGi, shift,     \
                     pl.d_items_cov, pl.d_p, pl.d_cov_off, n, (long long)pl.p_half, nitems, sp.per,                \
                     (long long)pl.cov_size, pl.p0)
  if (precision == FB_BF16X3) {
    if (herm) FB_COV(1, true);
    else FB_COV(1, false);
  } else {
    if (herm) FB_COV(0, true);
    else FB_COV(0, false);
  }
#undef FB_COV
  const long long tot = (long long)pl.cov_size + pl.p0;
  hipLaunchKernelGGL(k_cov_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, partG, partS0, partGi,
                     sp.slices, (long long)pl.cov_size, pl.p0, G, S0, Gi);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
