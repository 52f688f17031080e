// Non-uniform FFT stages of the expansion (Algorithm 1, step 3, Eq.(nufft)),
// the angular FFT (Eq.(1DFFT)) and their transposes, for gfx950.
//
// Forward, per image (s = 1, full L x L grid):
//   rows    : deconvolve by 1/phi_hat(x1/N) 1/phi_hat(x2/N), zero-pad to N, FFT along i2
//             (two real rows packed in one complex FFT), keep m2 = -hw..N/2+hw
//   cols    : FFT along i1 of every kept m2 row  ->  oversampled half-plane grid G(m1, m2)
//   gather  : F(xi_j, theta_l) = sum_taps phi(t1 - m1) phi(t2 - m2) G(m1, m2), l < n_theta/2
//   angular : real FFT of length n_theta of s_l = Re F_l + Im F_l, s_{l+H} = Re F_l - Im F_l,
//             then Fhat(k) = (2 pi/n_theta) S(k) (k even) or i (2 pi/n_theta) S(k) (k odd)
// Adjoint: the transpose of each stage in reverse order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_common.h"
#include "fft_dev.h"
#include "kernels.h"

namespace fb {

// Copy `total` elements with every thread issuing U global loads before it stores
// any of them, so that the loads of one thread are in flight together.
template <int U, class LoadF, class StoreF>
__device__ __forceinline__ void batched_copy(int total, LoadF ld, StoreF stv) {
  for (int base = threadIdx.x; base < total; base += U * blockDim.x) {
    decltype(ld(0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int i = base + u * blockDim.x;
      if (i < total) v[u] = ld(i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int i = base + u * blockDim.x;
      if (i < total) stv(i, v[u]);
    }
  }
}

// Same, over an (outer, inner) index space with inner < INNER <= 64: thread t takes
// inner = t % INNER and outer = t / INNER + multiples of blockDim / INNER (no division).
template <int U, int INNER, class LoadF, class StoreF>
__device__ __forceinline__ void batched_copy2d(int n_outer, int n_inner, LoadF ld, StoreF stv) {
  const int in = threadIdx.x % INNER, os = blockDim.x / INNER;
  if (in >= n_inner) return;
  for (int base = threadIdx.x / INNER; base < n_outer; base += U * os) {
    decltype(ld(0, 0)) v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int o = base + u * os;
      if (o < n_outer) v[u] = ld(o, in);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int o = base + u * os;
      if (o < n_outer) stv(o, in, v[u]);
    }
  }
}

// ---------------------------------------------------------------------------
// forward rows: images [n][L][L] -> G1 [n][M2][L]   (m2 = -hw..N/2+hw)
// block: RP row pairs of one image
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_fwd_rows(const float* __restrict__ img, float2* __restrict__ g1, const float* __restrict__ deconv,
                           FftDesc fd, const float2* __restrict__ tw, int L, int M2, int hw, int RP, FastDiv dL) {
  extern __shared__ float2 sm[];
  const int N = fd.n, S = N + 1;  // odd stride: the unpack reads all transforms at one frequency
  float2* buf = sm;
  float2* tmp = sm + RP * S;
  const int im = blockIdx.y;
  const int pair0 = blockIdx.x * RP;
  const int npairs = (L + 1) / 2;
  const int np = min(RP, npairs - pair0);
  const int x0 = -((L - 1 + 1) / 2);  // -ceil((L-1)/2)
  const float* src = img + (size_t)im * L * L;
  for (int i = threadIdx.x; i < RP * S; i += blockDim.x) buf[i] = make_float2(0.f, 0.f);
  __syncthreads();
  // rows a = 2 pair0 + r, r < 2 np; row r goes to transform r / 2, real (r even) or imaginary part
  batched_copy<8>(
      np * 2 * L,
      [&](int i) -> float {
        int r = dL.div(i), b = i - r * L;
        int a = 2 * pair0 + r;
        return (a < L) ? src[(size_t)a * L + b] * deconv[a] * deconv[b] : 0.f;
      },
      [&](int i, float v) {
        int r = dL.div(i), b = i - r * L;
        int pos = x0 + b;
        pos += (pos < 0) ? N : 0;
        float* slot = (float*)&buf[(r >> 1) * S + pos];
        slot[r & 1] = v;
      });
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, np, S, fd, tw);
  // unpack: row a: (Z(m) + conj Z(-m)) / 2, row a+1: (Z(m) - conj Z(-m)) / (2i); lanes over the rows
  float2* out = g1 + (size_t)im * M2 * L;
  const int r = threadIdx.x & 31;
  const int a = 2 * pair0 + r;
  if (r < 2 * np && a < L) {
    const int p = r >> 1, which = r & 1;
    for (int mi = threadIdx.x >> 5; mi < M2; mi += blockDim.x >> 5) {
      int m2 = mi - hw;
      int mp = m2 < 0 ? m2 + N : m2;      // |m2| < N
      int mn = m2 > 0 ? N - m2 : -m2;
      float2 z1 = res[p * S + mp], z2 = cconj(res[p * S + mn]);
      float2 v;
      if (which == 0) v = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y));
      else {
        float2 u = csub(z1, z2);
        v = make_float2(0.5f * u.y, -0.5f * u.x);
      }
      out[(size_t)mi * L + a] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// forward cols: G1 [n][M2][L] -> G [M2][group][N][kImgGroup]   (images innermost, grouped)
// block: one stored row m2 for CI (<= kImgGroup) consecutive image slots; LDS
// transforms padded to N+1.  Slots past nimg are written as zeros.
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_fwd_cols(const float2* __restrict__ g1, float2* __restrict__ g, FftDesc fd,
                           const float2* __restrict__ tw, int L, int M2, int nimg, int ngrp, int CI, FastDiv dL) {
  extern __shared__ float2 sm[];
  const int N = fd.n, S = N + 1;
  float2* buf = sm;
  float2* tmp = sm + CI * S;
  const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int m2 = lin / gridDim.x;             // image groups vary fastest: neighbours share lines
  const int i0 = (lin - m2 * gridDim.x) * CI;
  const int ni = max(0, min(CI, nimg - i0));           // images with data
  const int nw = min(CI, ngrp * kImgGroup - i0);       // slots written
  const int x0 = -((L - 1 + 1) / 2);
  for (int i = threadIdx.x; i < CI * S; i += blockDim.x) buf[i] = make_float2(0.f, 0.f);
  __syncthreads();
  batched_copy<8>(
      ni * L,
      [&](int i) -> float2 {
        int c = dL.div(i), a = i - c * L;
        return g1[((size_t)(i0 + c) * M2 + m2) * L + a];
      },
      [&](int i, float2 v) {
        int c = dL.div(i), a = i - c * L;
        int pos = x0 + a;
        pos += (pos < 0) ? N : 0;
        buf[c * S + pos] = v;
      });
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, ni, S, fd, tw);
  const int c = threadIdx.x & (kImgGroup - 1);  // CI <= kImgGroup slots in the workgroup
  if (c < nw) {
    const int i = i0 + c;
    float2* dst = g + ((size_t)m2 * ngrp + (i / kImgGroup)) * N * kImgGroup + (i & (kImgGroup - 1));
    const bool live = c < ni;
    for (int m1 = threadIdx.x / kImgGroup; m1 < N; m1 += blockDim.x / kImgGroup)
      dst[(size_t)m1 * kImgGroup] = live ? res[c * S + m1] : make_float2(0.f, 0.f);
  }
}

// ---------------------------------------------------------------------------
// Streaming forms of the two grid passes (in-place FFT with radices 8/4, N <= 512,
// 1024 threads, 16 transforms per unit).  Same results as k_fwd_rows / k_fwd_cols.
// A workgroup runs U consecutive units; the next unit's inputs are loaded into
// registers before the current unit is transformed and written, the FFT reads its
// twiddles from LDS and meets at LDS-only barriers, so those loads stay in flight.
// ---------------------------------------------------------------------------
constexpr int kGridStreamN = 512;   // largest power-of-two grid side of the streaming forms
constexpr int kStreamMixedN = 720;  // the compile-time mixed-radix length (L = 360 grid, R = 180 rings)
// LDS and prefetch registers of a streaming kernel are sized for the larger of its own
// compile-time length and the largest power-of-two one; a kernel longer than 512 holds one
// workgroup per compute unit (its LDS), so it may take twice the registers.
constexpr int stream_cap(int nc, int base) { return nc > base ? nc : base; }
constexpr int stream_waves(int nc) { return nc > kGridStreamN ? 4 : 8; }

// rows: unit = (image, 16 row pairs); rows a = 2 p0 .. 2 p0 + 31 of the image.  Thread t
// stages row t / 32 of the unit at the pixel quads t % 32 + 32 q, and zero-pads transform
// t / 64 at the columns t % 64 + 64 q, so its LDS positions are the same for every unit.
template <int NC>
__global__ __launch_bounds__(1024, stream_waves(NC)) void k_fwd_rows_stream(const float* __restrict__ img, float2* __restrict__ g1,
                                                             const float* __restrict__ deconv, FftDesc fd,
                                                             const float2* __restrict__ tw, int L, int M2, int hw,
                                                             int nimg, int U) {
  constexpr bool SW = grid_swizzle(NC);  // LDS layout of the transforms
  constexpr int RP = 16, NM = stream_cap(NC, kGridStreamN);
  __shared__ __attribute__((aligned(16))) float2 s_buf[RP * lds_span<NC, SW>(NM)];
  __shared__ float2 s_tw[NM];
  __shared__ float s_dec[NM / 2];
  const int N = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(N);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nrb = ((L + 1) / 2 + RP - 1) / RP;  // row blocks per image
  const int total = nimg * nrb;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int x0 = -((L - 1 + 1) / 2);  // -ceil((L-1)/2)
  for (int i = tid; i < N; i += nthr) s_tw[i] = tw[fd.tw_off + i];
  for (int i = tid; i < L; i += nthr) s_dec[i] = deconv[i];
  __syncthreads();
  // one item = four consecutive pixels of a row (L % 4 == 0, L <= N / 2); rows past L read as zero
  static_assert(2 * RP * 32 == 1024, "32 threads per row of the unit");
  constexpr int PF = (NM / 2 / 4 + 31) / 32;
  const int L4 = L / 4;
  const int r = tid >> 5, bq = tid & 31;  // this thread's row of the unit, first pixel quad
  float2* zrow = s_buf + (tid >> 6) * S;  // the transform this thread zero-pads
  float4 pre[PF];
  auto load = [&](int u) {
    const int im = u / nrb, a = 2 * RP * (u - im * nrb) + r;
    const float4* src = (const float4*)(img + ((size_t)im * L + min(a, L - 1)) * L) + bq;
#pragma unroll
    for (int q = 0; q < PF; ++q)
      pre[q] = (a < L && bq + 32 * q < L4) ? src[32 * q] : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    const int im = u / nrb, a0 = 2 * RP * (u - im * nrb);
    // row a0 + r goes to transform r / 2, real part (r even) or imaginary part (r odd),
    // deconvolved and centred; the N - L padded columns of every transform are zero
    {
      const int a = a0 + r;
      const float da = (a < L) ? s_dec[a] : 0.f;
      float* row = (float*)(s_buf + (r >> 1) * S) + (r & 1);
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int b0 = 4 * (bq + 32 * q);
        if (b0 < L) {
          const float vv[4] = {pre[q].x, pre[q].y, pre[q].z, pre[q].w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int pos = x0 + b0 + i;
            pos += (pos < 0) ? N : 0;
            row[2 * lds_pos<NC, SW>(pos)] = vv[i] * da * s_dec[b0 + i];
          }
        }
      }
    }
    for (int z = tid & 63; z < N - L; z += 64) {  // columns past the image, wrapped
      int pos = x0 + L + z;
      pos -= (pos >= N) ? N : 0;
      zrow[lds_pos<NC, SW>(pos)] = make_float2(0.f, 0.f);
    }
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);
    fft_stream<NC, RP, SW>(s_buf, S, fd, s_tw);
    // unpack: row a: (Z(m) + conj Z(-m)) / 2, row a+1: (Z(m) - conj Z(-m)) / (2i); lanes over the rows
    float2* out = g1 + (size_t)im * M2 * L;
    const int ru = tid & 31, au = a0 + ru;  // the unpacking lanes run over the unit's rows
    if (au < L) {
      const int pp = ru >> 1, which = ru & 1;
      for (int mi = tid >> 5; mi < M2; mi += nthr >> 5) {
        int m2 = mi - hw;
        int mp = m2 < 0 ? m2 + N : m2;
        int mn = m2 > 0 ? N - m2 : -m2;
        float2 z1 = s_buf[pp * S + lds_pos<NC, SW>(mp)], z2 = cconj(s_buf[pp * S + lds_pos<NC, SW>(mn)]);
        float2 v;
        if (which == 0) {
          v = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y + z2.y));
        } else {
          float2 dd = csub(z1, z2);
          v = make_float2(0.5f * dd.y, -0.5f * dd.x);
        }
        out[(size_t)mi * L + au] = v;
      }
    }
    stage_barrier<true>();
  }
}

// columns: unit = (stored row m2, image group); output G [M2][group][N][16], of each row
// only the centred m1 range gcols[m2] that the gather's boxes read.  Thread t stages image
// slot t / 64 of the group at the columns t % 64 + 64 q, so its positions in LDS (and in the
// zero padding) are the same for every unit and its loads are one run per image.
// blocks of 64 columns in which the columns form reads an image row of at most n / 2 values
constexpr int cols_stream_blocks(int n) { return (n / 2 + 63) / 64; }

template <int NC>
__global__ __launch_bounds__(1024, stream_waves(NC)) void k_fwd_cols_stream(const float2* __restrict__ g1, float2* __restrict__ g,
                                                             FftDesc fd, const float2* __restrict__ tw,
                                                             const int2* __restrict__ gcols, int L, int M2,
                                                             int nimg, int ngrp, int U) {
  constexpr bool SW = grid_swizzle(NC);  // LDS layout of the transforms
  constexpr int G = kImgGroup, NM = stream_cap(NC, kGridStreamN);
  static_assert(G * 64 == 1024, "64 threads per image slot");
  __shared__ __attribute__((aligned(16))) float2 s_buf[G * lds_span<NC, SW>(NM)];
  __shared__ float2 s_tw[NM];
  const int N = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(N);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = M2 * ngrp;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int x0 = -((L - 1 + 1) / 2);
  for (int i = tid; i < N; i += nthr) s_tw[i] = tw[fd.tw_off + i];
  __syncthreads();
  // column blocks per row: L <= N / 2; for a compiled length L > 64 (PF - 1) (checked at launch)
  constexpr int PF = cols_stream_blocks(NC > 0 ? NC : NM);
  const int ci = tid >> 6, ai = tid & 63;
  float2* row = s_buf + ci * S;
  float2 pre[PF];
  // unit u = (m2, group): groups vary fastest, so consecutive units write consecutive runs of G
  // the loads are unconditional (a conditional load is waited for where it is issued, which
  // would undo the prefetch): a slot past the last image reads the last image and a column
  // past L reads column L - 1, and the LDS stores put zeros in their place
  auto load = [&](int u) {
    const int m2 = u / ngrp, i0 = (u - m2 * ngrp) * G;
    const float2* src = g1 + ((size_t)min(i0 + ci, nimg - 1) * M2 + m2) * L;
#pragma unroll
    for (int q = 0; q < PF; ++q)  // (the run-time-length form sizes PF for its largest N: clamps all)
      pre[q] = src[q + 1 < PF && NC > 0 ? ai + 64 * q : min(ai + 64 * q, L - 1)];
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    const int m2 = u / ngrp, grp = u - m2 * ngrp;
    const bool live = grp * G + ci < nimg;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int a = ai + 64 * q;
      if (a < L) {
        int pos = x0 + a;
        pos += (pos < 0) ? N : 0;
        row[lds_pos<NC, SW>(pos)] = live ? pre[q] : make_float2(0.f, 0.f);
      }
    }
    for (int z = ai; z < N - L; z += 64) {  // the columns past the image, wrapped
      int pos = x0 + L + z;
      pos -= (pos >= N) ? N : 0;
      row[lds_pos<NC, SW>(pos)] = make_float2(0.f, 0.f);
    }
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);
    fft_stream<NC, G, SW>(s_buf, S, fd, s_tw);
    const int c = tid & (G - 1);
    float2* dst = g + ((size_t)m2 * ngrp + grp) * N * G + c;
    const int2 rg = gcols[m2];
    for (int ic = rg.x + tid / G; ic <= rg.y; ic += nthr / G) {
      const int m1 = ic < 0 ? ic + N : ic;
      st_out(&dst[(size_t)m1 * G], s_buf[c * S + lds_pos<NC, SW>(m1)]);
    }
    stage_barrier<true>();
  }
}

// ---------------------------------------------------------------------------
// forward gather: G [M2][group][N][16] -> P [n_xi][group][H][16]
// block = (work item: one grid cell and up to kGatherChunk of its nodes, group of IG images).
// The cell's (CS + W - 1)^2 box of grid points is staged in LDS for the IG images (each
// point's IG values are one contiguous 8*IG-byte run in G), then every (node, image pair)
// lane interpolates its W x W taps from LDS with the node's precomputed weights.  Items
// hold up to kGatherChunk nodes, so the box fill is paid once for many nodes.
// ---------------------------------------------------------------------------
template <int W, int CS, int IG, int NT>
__global__ __launch_bounds__(NT) void k_fwd_gather(const float2* __restrict__ g, float2* __restrict__ P,
                                                    const GatherItem* __restrict__ items,
                                                    const GatherNode* __restrict__ gn, int nitems, int N,
                                                    int M2, int H, int ngrp) {
  static_assert(IG == kImgGroup, "a gather workgroup takes one image group");
  constexpr int BW = CS + W - 1;
  constexpr int NPT = BW * BW;            // grid points in the box
  extern __shared__ float4 lds4[];
  float2* box = (float2*)lds4;                               // [NPT][IG]
  const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  // cells vary fastest inside one image group: an XCD then walks neighbouring cells,
  // whose boxes overlap by the halo, while those rows are still in its L2
  const int itx = lin % nitems;
  const int grp = lin / nitems;
  const GatherItem it = items[itx];
  const int nn = it.s1 - it.s0;
  {
    // every group is whole (padded): issue every load of this thread before the LDS stores;
    // a box row of one group is one contiguous run of BW * IG values in G.  Thread t < BR * RW
    // takes box rows t / RW + BR u and, in each, column and image pair t % RW, so successive
    // loads step by BR rows in G and by a constant in LDS.
    constexpr int RW = BW * (IG / 2);  // float4 per box row
    constexpr int BR = NT / RW;        // box rows per pass of the threads
    constexpr int PR = (BW + BR - 1) / BR;
    static_assert(BR >= 1 && PR * BR >= BW, "the passes cover the box rows");
    const int t = threadIdx.x, rr = t / RW, w = t - rr * RW;
    const int cc = w / (IG / 2), h = w - cc * (IG / 2);
    int col = it.c1 + cc;
    col = col >= N ? col - N : col;
    const size_t row_stride = (size_t)ngrp * N * IG;
    const float4* src = (const float4*)(g + (size_t)grp * N * IG + (size_t)(it.c2 + (rr < BR ? rr : 0)) * row_stride +
                                        (size_t)col * IG + 2 * h);
    float4 v[PR];
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int r = rr + BR * u;
      v[u] = (rr < BR && r < BW && it.c2 + r < M2) ? src[(size_t)(BR * u) * (row_stride / 2)]
                                                   : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int r = rr + BR * u;
      if (rr < BR && r < BW) lds4[r * RW + w] = v[u];
    }
  }
  __syncthreads();
  // each lane interpolates one node for two consecutive images (16-byte LDS reads)
  constexpr int IP = IG / 2;
  const int ip = threadIdx.x % IP;
  const int slot = threadIdx.x / IP;
  constexpr int SLOTS = NT / IP;
  const float4* box4 = (const float4*)box;
  // node records come straight from global memory (the eight lanes of one node share
  // each 64-byte line); the next record is in flight while the current node is summed
  union NodeRegs {
    float4 v[4];
    GatherNode g;
  };
  static_assert(sizeof(GatherNode) == 4 * sizeof(float4), "node record is four 16-byte words");
  const float4* gn4 = (const float4*)(gn + it.s0);
  NodeRegs nxt_nd;
  if (slot < nn) {
#pragma unroll
    for (int q = 0; q < 4; ++q) nxt_nd.v[q] = gn4[slot * 4 + q];
  }
  for (int s = slot; s < nn; s += SLOTS) {
    NodeRegs cur_nd = nxt_nd;
    if (s + SLOTS < nn) {
#pragma unroll
      for (int q = 0; q < 4; ++q) nxt_nd.v[q] = gn4[(s + SLOTS) * 4 + q];
    }
    const GatherNode& nd = cur_nd.g;
    const float4* b = box4 + (size_t)nd.off * IP + ip;
    float ax0 = 0.f, ay0 = 0.f, ax1 = 0.f, ay1 = 0.f;
    // rows of W taps: the next row's loads are issued before this row's products
    float4 cur[W], nxt[W];
#pragma unroll
    for (int a = 0; a < W; ++a) cur[a] = b[a * IP];
#pragma unroll
    for (int bb = 0; bb < W; ++bb) {
      if (bb + 1 < W) {
#pragma unroll
        for (int a = 0; a < W; ++a) nxt[a] = b[((bb + 1) * BW + a) * IP];
      }
      float rx0 = 0.f, ry0 = 0.f, rx1 = 0.f, ry1 = 0.f;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        rx0 = fmaf(nd.w1[a], cur[a].x, rx0);
        ry0 = fmaf(nd.w1[a], cur[a].y, ry0);
        rx1 = fmaf(nd.w1[a], cur[a].z, rx1);
        ry1 = fmaf(nd.w1[a], cur[a].w, ry1);
      }
      ax0 = fmaf(nd.w2[bb], rx0, ax0);
      ay0 = fmaf(nd.w2[bb], ry0, ay0);
      ax1 = fmaf(nd.w2[bb], rx1, ax1);
      ay1 = fmaf(nd.w2[bb], ry1, ay1);
      if (bb + 1 < W) {
#pragma unroll
        for (int a = 0; a < W; ++a) cur[a] = nxt[a];
      }
    }
    float2* dst = P + (((size_t)nd.j * ngrp + grp) * H + nd.l) * IG + 2 * ip;
    st_out((float4*)dst, make_float4(ax0, ay0, ax1, ay1));
  }
}

constexpr int kGatherImages = kImgGroup;  // one image group per gather workgroup
constexpr int kGatherThreads = 512;
size_t gather_lds_bytes() {
  constexpr int BW = kGatherCell + kGatherW - 1;
  return (size_t)BW * BW * kGatherImages * sizeof(float2);
}

// ---------------------------------------------------------------------------
// forward angular: P [n_xi][group][H][16] -> Fh [group][n_xi][K+1][16] (complex); a
// workgroup's output for all k is one contiguous run
// block: ring j for AG (<= kImgGroup) consecutive image slots; LDS transforms padded to H+1
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_fwd_angular(const float2* __restrict__ P, float2* __restrict__ Fh, FftDesc fd,
                              const float2* __restrict__ tw, const float2* __restrict__ angtw, int n_xi, int K,
                              int ngrp, int AG, float scale) {
  extern __shared__ float2 sm[];
  const int H = fd.n, S = H + 1;
  float2* buf = sm;
  float2* tmp = sm + AG * S;
  const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int j = lin / gridDim.x;              // image groups vary fastest: neighbours share lines
  const int g0 = (lin - j * gridDim.x) * AG;
  const int ng = min(AG, ngrp * kImgGroup - g0);
  // image slot g0 + gg of ring j: group (g0 + gg) / 16, lane (g0 + gg) % 16
  auto slot_base = [&](int outer, int inner, int gg) -> size_t {
    const int i = g0 + gg;
    return (((size_t)outer * ngrp + i / kImgGroup) * inner) * kImgGroup + (i & (kImgGroup - 1));
  };
  // packed z_m = s_{2m} + i s_{2m+1}, with s_t = u_t + v_t (t < H), u_{t-H} - v_{t-H} (t >= H)
  batched_copy2d<8, 16>(
      H, ng,
      [&](int m, int gg) -> float4 {
        int t0 = 2 * m, t1 = 2 * m + 1;
        const float2* ring = P + slot_base(j, H, gg);
        float2 f0 = ring[(size_t)(t0 < H ? t0 : t0 - H) * kImgGroup];
        float2 f1 = ring[(size_t)(t1 < H ? t1 : t1 - H) * kImgGroup];
        return make_float4(f0.x, f0.y, f1.x, f1.y);
      },
      [&](int m, int gg, float4 f) {
        float s0 = (2 * m < H) ? (f.x + f.y) : (f.x - f.y);
        float s1 = (2 * m + 1 < H) ? (f.z + f.w) : (f.z - f.w);
        buf[gg * S + m] = make_float2(s0, s1);
      });
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, ng, S, fd, tw);
  const int gg = threadIdx.x & 15;  // AG <= 16 images in the workgroup
  if (gg < ng)
  for (int k = threadIdx.x >> 4; k <= K; k += blockDim.x >> 4) {
    float2 zk = res[gg * S + k];
    float2 zc = cconj(res[gg * S + (k == 0 ? 0 : H - k)]);
    // S(k) = (Z(k) + conj Z(H-k))/2 + e^{-2 pi i k / n_theta} (Z(k) - conj Z(H-k)) / (2i)
    float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
    float2 d = csub(zk, zc);
    float2 o = make_float2(0.5f * d.y, -0.5f * d.x);
    float2 Sk = cadd(e, cmul(angtw[k], o));
    float2 F = (k & 1) ? make_float2(-Sk.y * scale, Sk.x * scale) : make_float2(Sk.x * scale, Sk.y * scale);
    const int i = g0 + gg;
    Fh[((((size_t)(i / kImgGroup) * n_xi + j) * (K + 1)) + k) * kImgGroup + (i & (kImgGroup - 1))] = F;
  }
}

// ---------------------------------------------------------------------------
// forward angular, streaming form (in-place FFT with radices 8/4, H % 8 == 0, H <= 512,
// one group of 16 images per unit).  Same result as k_fwd_angular.  Each workgroup runs
// U consecutive (ring, group) units; the polar samples of the next unit are loaded into
// registers before the current unit is transformed and written, and the FFT reads its
// twiddles from LDS and meets at LDS-only barriers, so those loads stay in flight
// through the transform and HBM traffic overlaps the FFT.
// ---------------------------------------------------------------------------
constexpr int kAngStreamH = 512;  // largest angular half length of the streaming form

template <int NC>
__global__ __launch_bounds__(1024, stream_waves(NC)) void k_fwd_angular_stream(const float2* __restrict__ P, float2* __restrict__ Fh,
                                                             FftDesc fd, const float2* __restrict__ tw,
                                                             const float2* __restrict__ angtw,
                                                             const int* __restrict__ kring, int n_xi, int K,
                                                             int ngrp, int U, float scale) {
  constexpr bool SW = angular_swizzle(NC);  // LDS layout of the transforms
  constexpr int G = kImgGroup, HM = stream_cap(NC, kAngStreamH);
  constexpr int PF = (HM * G / 2 + 1023) / 1024;  // (m, gg) items per thread at the largest H
  __shared__ __attribute__((aligned(16))) float2 s_buf[G * lds_span<NC, SW>(HM)];  // packed transforms, padded
  __shared__ float2 s_tw[HM];
  __shared__ float2 s_angtw[HM];
  const int H = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(H), Hh = H / 2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = n_xi * ngrp;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int nitem = G * Hh;
  for (int i = tid; i < H; i += nthr) s_tw[i] = tw[fd.tw_off + i];
  for (int i = tid; i <= K; i += nthr) s_angtw[i] = angtw[i];
  __syncthreads();
  // unit u = (ring j, group): groups vary fastest, so consecutive units are consecutive in P.
  // Item e = (gg, m) of a unit holds lane gg's samples t = 2m and 2m + 1.
  float4 pre[PF];
  auto load = [&](int u) {
    const float2* src = P + (size_t)u * H * G;
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int e = tid + p * nthr;
      if (e < nitem) {
        const int gg = e & (G - 1), m = e / G;
        const float2 f0 = src[(2 * m) * G + gg], f1 = src[(2 * m + 1) * G + gg];
        pre[p] = make_float4(f0.x, f0.y, f1.x, f1.y);
      }
    }
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    // packed z_m = s_{2m} + i s_{2m+1}, s_t = Re P_t + Im P_t and s_{t+H} = Re P_t - Im P_t (t < H)
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int e = tid + p * nthr;
      if (e < nitem) {
        const int gg = e & (G - 1), m = e / G;
        const float4 f = pre[p];
        s_buf[gg * S + lds_pos<NC, SW>(m)] = make_float2(f.x + f.y, f.z + f.w);
        s_buf[gg * S + lds_pos<NC, SW>(m + Hh)] = make_float2(f.x - f.y, f.z - f.w);
      }
    }
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);  // in flight through the transform and the writes below
    fft_stream<NC, G, SW>(s_buf, S, fd, s_tw);
    const int j = u / ngrp, grp = u - j * ngrp;
    const int gg = tid & (G - 1);
    float2* dst = Fh + (((size_t)grp * n_xi + j) * (K + 1)) * G + gg;
    // only the k whose radial sums read ring j (the table of every larger k is negligible there)
    const int Kj = kring[j];
    for (int k = tid / G; k <= Kj; k += nthr / G) {
      float2 zk = s_buf[gg * S + lds_pos<NC, SW>(k)];
      float2 zc = cconj(s_buf[gg * S + lds_pos<NC, SW>(k == 0 ? 0 : H - k)]);
      // S(k) = (Z(k) + conj Z(H-k))/2 + e^{-2 pi i k / n_theta} (Z(k) - conj Z(H-k)) / (2i)
      float2 e = make_float2(0.5f * (zk.x + zc.x), 0.5f * (zk.y + zc.y));
      float2 d = csub(zk, zc);
      float2 o = make_float2(0.5f * d.y, -0.5f * d.x);
      float2 Sk = cadd(e, cmul(s_angtw[k], o));
      st_out(&dst[(size_t)k * G],
             (k & 1) ? make_float2(-Sk.y * scale, Sk.x * scale) : make_float2(Sk.x * scale, Sk.y * scale));
    }
    stage_barrier<true>();  // s_buf is rewritten by the next unit
  }
}

// ---------------------------------------------------------------------------
// adjoint angular: D [group][n_xi][K+1][16] -> Q [n_xi][group][H][16] (grouped like P)
// Q_l = (s'_l + s'_{l+H}) + i (s'_l - s'_{l+H}),  s'_t = Re sum_{k<=K} E_k e^{2 pi i k t / n_theta},
// E_k = c D_k (k even), -i c D_k (k odd).  Images vary fastest in both loops (whole
// 128-byte lines of D and Q); transforms padded to H+1.
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_adj_angular(const float2* __restrict__ D, float2* __restrict__ Q, FftDesc fd,
                              const float2* __restrict__ tw, const float2* __restrict__ angtw, int n_xi, int K,
                              int nimg, int ngrp, int AG, float scale) {
  extern __shared__ float2 sm[];
  const int H = fd.n, S = H + 1;
  float2* buf = sm;
  float2* tmp = sm + AG * S;
  const int j = blockIdx.x;
  const int g0 = blockIdx.y * AG;
  const int ng = min(AG, ngrp * kImgGroup - g0);  // slots past nimg read zeros
  auto Ek = [&](int k, int gg) -> float2 {
    if (g0 + gg >= nimg) return make_float2(0.f, 0.f);
    const int img = g0 + gg;
    float2 d = D[(((size_t)(img / kImgGroup) * n_xi + j) * (K + 1) + k) * kImgGroup + (img & (kImgGroup - 1))];
    return (k & 1) ? make_float2(d.y * scale, -d.x * scale) : make_float2(d.x * scale, d.y * scale);
  };
  // Zin(k') = (Y_k' + Y_{k'+H}) + i e^{+i pi k'/H} (Y_k' - Y_{k'+H}); stored conjugated for the forward FFT
  for (int i = threadIdx.x; i < ng * H; i += blockDim.x) {
    int kp = i / ng, gg = i - kp * ng;
    float2 y0 = make_float2(0.f, 0.f), y1 = make_float2(0.f, 0.f);
    if (kp == 0) {
      y0 = make_float2(Ek(0, gg).x, 0.f);
    } else if (kp <= K) {
      float2 e = Ek(kp, gg);
      y0 = make_float2(0.5f * e.x, 0.5f * e.y);
    }
    int km = H - kp;  // Y_{k'+H} = conj(E_{H-k'}) / 2
    if (km >= 1 && km <= K) {
      float2 e = Ek(km, gg);
      y1 = make_float2(0.5f * e.x, -0.5f * e.y);
    }
    float2 ze = cadd(y0, y1);
    float2 zo = cmul(cconj(angtw[kp]), csub(y0, y1));
    float2 zin = make_float2(ze.x - zo.y, ze.y + zo.x);
    buf[gg * S + kp] = cconj(zin);
  }
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, ng, S, fd, tw);
  // z_m = conj(res_m) = s'_{2m} + i s'_{2m+1}
  for (int i = threadIdx.x; i < ng * H; i += blockDim.x) {
    int l = i / ng, gg = i - l * ng;
    auto sp = [&](int t) -> float {
      float2 z = res[gg * S + (t >> 1)];
      return (t & 1) ? -z.y : z.x;
    };
    float a = sp(l), b = sp(l + H);
    const int sl = g0 + gg;
    Q[(((size_t)j * ngrp + sl / kImgGroup) * H + l) * kImgGroup + (sl & (kImgGroup - 1))] = make_float2(a + b, a - b);
  }
}

// ---------------------------------------------------------------------------
// adjoint angular, streaming form (conditions as for the forward streaming form).  Same
// result as k_adj_angular.  Each workgroup runs U consecutive (ring, group) units; the
// next unit's spectrum (K+1 values of 16 images, one contiguous run of D) is loaded into
// registers before the current unit is transformed and written.  Per unit the values are
// placed in LDS at their k (zeros above K), the Hermitian completion is formed in place
// for the pairs (k', H - k'), and the in-place FFT meets at LDS-only barriers so that the
// loads stay in flight.
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(1024, stream_waves(NC)) void k_adj_angular_stream(const float2* __restrict__ D, float2* __restrict__ Q,
                                                             FftDesc fd, const float2* __restrict__ tw,
                                                             const float2* __restrict__ angtw, int n_xi, int K,
                                                             int nimg, int ngrp, int U, float scale) {
  constexpr bool SW = angular_swizzle(NC);  // LDS layout of the transforms
  constexpr int G = kImgGroup, HM = stream_cap(NC, kAngStreamH);
  constexpr int PF = (HM * G / 2 + 1023) / 1024;  // pairs of spectrum values per thread (K + 1 <= H)
  __shared__ __attribute__((aligned(16))) float2 s_buf[G * lds_span<NC, SW>(HM)];
  __shared__ float2 s_tw[HM];
  __shared__ float2 s_angtw[HM];
  const int H = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(H), Hh = H / 2;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = n_xi * ngrp;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int nval = (K + 1) * G;
  for (int i = tid; i < H; i += nthr) {
    s_tw[i] = tw[fd.tw_off + i];
    s_angtw[i] = angtw[i];
  }
  __syncthreads();
  // unit u = (ring j, group): groups vary fastest, so consecutive units write consecutive Q
  // item e holds the values 2e and 2e + 1 of the unit's run: k = 2e / 16, images gg, gg + 1
  float4 pre[PF];
  auto load = [&](int u) {
    const int j = u / ngrp, grp = u - j * ngrp;
    const float4* src = (const float4*)(D + ((size_t)grp * n_xi + j) * (K + 1) * G);
    const int live = nimg - grp * G;  // image slots of this group that hold data
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int e = tid + p * nthr;
      if (2 * e < nval) {
        float4 v = src[e];
        const int gg = (2 * e) & (G - 1);
        if (gg >= live) v.x = v.y = 0.f;
        if (gg + 1 >= live) v.z = v.w = 0.f;
        pre[p] = v;
      }
    }
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    // E_k = c D_k (k even), -i c D_k (k odd), at its k; zeros for K < k < H
#pragma unroll
    for (int p = 0; p < PF; ++p) {
      const int e = tid + p * nthr;
      if (2 * e < nval) {
        const int k = (2 * e) / G, gg = (2 * e) & (G - 1);
        const float4 d = pre[p];
        const float sr = (k & 1) ? -scale : scale;  // odd k: -i c D_k
        s_buf[gg * S + lds_pos<NC, SW>(k)] = (k & 1) ? make_float2(d.y * scale, d.x * sr) : make_float2(d.x * scale, d.y * scale);
        s_buf[(gg + 1) * S + lds_pos<NC, SW>(k)] =
            (k & 1) ? make_float2(d.w * scale, d.z * sr) : make_float2(d.z * scale, d.w * scale);
      }
    }
    for (int e = nval + tid; e < H * G; e += nthr) s_buf[(e & (G - 1)) * S + lds_pos<NC, SW>(e / G)] = make_float2(0.f, 0.f);
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);  // in flight through the transform and the writes below
    // Zin(k') = (Y_k' + Y_{k'+H}) + i e^{+i pi k'/H} (Y_k' - Y_{k'+H}), Y_k' = E_k'/2 (Re E_0 at 0),
    // Y_{k'+H} = conj(E_{H-k'})/2; pairs (k', H - k') share their two inputs; stored conjugated
    for (int e = tid; e < (Hh + 1) * G; e += nthr) {
      const int kp = e / G, gg = e & (G - 1), km = H - kp;
      float2* row = s_buf + gg * S;
      const float2 a = row[lds_pos<NC, SW>(kp)];
      const float2 b = kp == 0 ? make_float2(0.f, 0.f) : row[lds_pos<NC, SW>(km)];
      auto zin = [&](int k, float2 ek, float2 eo) {  // ek = E_k, eo = E_{H-k}
        const float2 y0 = k == 0 ? make_float2(ek.x, 0.f) : make_float2(0.5f * ek.x, 0.5f * ek.y);
        const float2 y1 = k == 0 ? make_float2(0.f, 0.f) : make_float2(0.5f * eo.x, -0.5f * eo.y);
        const float2 ze = cadd(y0, y1);
        const float2 zo = cmul(cconj(s_angtw[k]), csub(y0, y1));
        return cconj(make_float2(ze.x - zo.y, ze.y + zo.x));
      };
      row[lds_pos<NC, SW>(kp)] = zin(kp, a, b);
      if (kp != 0 && kp != Hh) row[lds_pos<NC, SW>(km)] = zin(km, b, a);
    }
    stage_barrier<true>();
    fft_stream<NC, G, SW>(s_buf, S, fd, s_tw);
    // z_m = conj(res_m) = s'_{2m} + i s'_{2m+1};  Q_l = (s'_l + s'_{l+H}) + i (s'_l - s'_{l+H})
    float2* dst = Q + (size_t)u * H * G;
    for (int e = tid; e < H * G; e += nthr) {
      const int l = e / G, gg = e & (G - 1);
      const float2* row = s_buf + gg * S;
      auto sp = [&](int t) -> float {
        const float2 z = row[lds_pos<NC, SW>(t >> 1)];
        return (t & 1) ? -z.y : z.x;
      };
      const float a = sp(l), b = sp(l + H);
      dst[e] = make_float2(a + b, a - b);
    }
    stage_barrier<true>();  // s_buf is rewritten by the next unit
  }
}

// ---------------------------------------------------------------------------
// adjoint spread (gather form, tiled): Q [n_xi][group][H][16] -> Y [N/2+1][group][N][16]
// workgroup = (tile: pairs of a cell of kSpreadRows x kSpreadCols output points, one of its
// nsub workgroups, slice of kSpreadSlice image groups); it walks its (chunk, image group)
// steps, chunks outer, with the next step's node values (one 128-byte line per node: 16
// images) and, when the chunk changes, entries on their way into registers.  A tile of
// several chunks keeps the partial sums of its (at most kSpreadHeavyGroups) image groups in
// registers, added in chunk order.  Per step the values and entries sit in LDS and lane
// (slot, image pair) sums the slot's entries in their fixed order, one 16-byte LDS read of
// node values for eight FMAs; the slots of a pair then add their sums in a fixed pattern,
// so the result is the same on every run.  Entries come in aligned batches of
// kSpreadBatch; spreading weights are non-negative, so each weight carries its point's
// conjugate flag as its sign.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT, 4) void k_adj_spread(const float2* __restrict__ Q, float2* __restrict__ Y,
                                                      const SpreadTile* __restrict__ tiles,
                                                      const SpreadBlock* __restrict__ blocks,
                                                      const SpreadChunk* __restrict__ chunks,
                                                      const int* __restrict__ snodes, const int* __restrict__ sseg,
                                                      const uint16_t* __restrict__ sslot,
                                                      const SpreadLocal* __restrict__ sent, int N, int Nh, int H,
                                                      int ngrp, int nsl) {
  constexpr int G = kImgGroup, IP = G / 2, NP = kSpreadPairs, CC = kSpreadCols;
  constexpr int EV = kSpreadEntries * 3 / 4;  // 16-byte vectors of a chunk's entries
  constexpr int KQ = kSpreadNodes * IP / NT, KE = EV / NT;
  static_assert(NT == NP * IP, "one lane per (point pair, image pair)");
  static_assert(KQ * NT == kSpreadNodes * IP && KE * NT == EV, "staging slots per lane");
  static_assert(sizeof(SpreadLocal) == 12 && kSpreadBatch == 4, "a batch is three 16-byte vectors");
  static_assert(kSpreadHeavyGroups == 2, "two partial-sum sets");
  // staging in native vector types, so that the register copies below stay in registers
  __shared__ __attribute__((aligned(16))) fb_f4v s_q[kSpreadNodes * IP];
  __shared__ __attribute__((aligned(16))) fb_u4v s_e[EV];
  const int tid = threadIdx.x, ip = tid & (IP - 1), pp = tid / IP;
  const int slice = (int)(blockIdx.x % (unsigned)nsl);
  const SpreadBlock bk = blocks[blockIdx.x / (unsigned)nsl];
  const SpreadTile t = tiles[bk.tile];
  const int nch = t.c1 - t.c0;
  const int gb = slice * kSpreadSlice + bk.sub, ge = min(ngrp, (slice + 1) * kSpreadSlice);
  // slot pp sums part of the entries of pair pr; the first of the pair's 2^lg2s slots (an
  // aligned run of lane groups in this wavefront) writes the pair's two points
  const unsigned sl = sslot[t.slots + pp];
  const int pr = sl & 63, lg2s = (sl >> 8) & 3;
  const bool lead = !(sl & kSpreadIdleSlot) && (pp & ((1 << lg2s) - 1)) == 0;
  const int m2 = t.m2 + 2 * (pr / CC), m1 = t.m1 + pr % CC;
  const bool outA = lead && m2 < Nh && m1 < N, outB = lead && m2 + 1 < Nh && m1 < N;
  float4* Y4 = (float4*)Y;
  auto yidx = [&](int r, int g) { return (((size_t)r * ngrp + g) * N + m1) * IP + ip; };
  auto put = [&](int g, float4 a, float4 b) {
    if (outA) Y4[yidx(m2, g)] = a;
    if (outB) Y4[yidx(m2 + 1, g)] = b;
  };
  // the slots of one pair add their sums, slots 1, 2, 4 apart in turn (every lane of the
  // wavefront takes part; x + y = y + x, so all slots of a pair end with the same bits)
  auto gather_slots = [&](float4& a, float4& b) {
    for (int k = 1; k < t.maxs; k <<= 1) {
      const int lanes = k * IP;
      const float4 oa = make_float4(__shfl_xor(a.x, lanes), __shfl_xor(a.y, lanes), __shfl_xor(a.z, lanes),
                                    __shfl_xor(a.w, lanes));
      const float4 ob = make_float4(__shfl_xor(b.x, lanes), __shfl_xor(b.y, lanes), __shfl_xor(b.z, lanes),
                                    __shfl_xor(b.w, lanes));
      if (k < (1 << lg2s)) {
        a = make_float4(a.x + oa.x, a.y + oa.y, a.z + oa.z, a.w + oa.w);
        b = make_float4(b.x + ob.x, b.y + ob.y, b.z + ob.z, b.w + ob.w);
      }
    }
  };
  if (nch == 0) {  // no node reaches this cell
    for (int g = gb; g < ge; g += t.nsub) put(g, make_float4(0.f, 0.f, 0.f, 0.f), make_float4(0.f, 0.f, 0.f, 0.f));
    return;
  }
  // image groups of this workgroup; a tile of several chunks has nsub >= 8, so ng <= 2
  const int ng = gb < ge ? (ge - gb + t.nsub - 1) / t.nsub : 0;
  const int nsteps = ng * nch;
  const fb_f4v* Q4 = (const fb_f4v*)Q;
  const fb_u4v* E4 = (const fb_u4v*)sent;
  const size_t gstride = (size_t)H * IP;  // float4s between image groups of one node
  // next step's chunk data, held in registers
  int nl_n = 0, ne_n = 0, e0_n = 0, e1_n = 0;
  unsigned qoff[KQ];  // node value offsets inside one image group's view (fit 32 bits: spread_max_images)
  fb_u4v er[KE];
  fb_f4v qr[KQ];
  auto load_meta_rec = [&](const SpreadChunk ch) {
    nl_n = ch.n1 - ch.n0;
    const int base = sseg[ch.seg];
    ne_n = (sseg[ch.seg + NP] - base) / 4 * 3;  // 16-byte vectors
    e0_n = (sseg[ch.seg + pp] - base) / 4 * 3;
    e1_n = (sseg[ch.seg + pp + 1] - base) / 4 * 3;
    // every chunk has at least one node and one batch of entries; slots past them load the
    // last ones again (and are not stored), so that no load is conditional: a conditional
    // load into a register that lives on is waited for where it is issued
#pragma unroll
    for (int k = 0; k < KE; ++k) er[k] = E4[base / 4 * 3 + min(tid + k * NT, ne_n - 1)];
#pragma unroll
    for (int k = 0; k < KQ; ++k) {
      const int i = min(tid + k * NT, nl_n * IP - 1);
      const int jl = snodes[ch.n0 + i / IP];
      qoff[k] = ((unsigned)(jl >> 16) * ngrp * H + (jl & 0xffff)) * IP + (i & (IP - 1));
    }
  };
  auto load_q_into = [&](fb_f4v (&dst)[KQ], int g) {
    const fb_f4v* Qg = Q4 + (size_t)g * gstride;
#pragma unroll
    for (int k = 0; k < KQ; ++k) dst[k] = Qg[qoff[k]];
  };
  auto load_q = [&](int g) { load_q_into(qr, g); };
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;
  // entry: byte offset of the node row in s_q, the two points' weights signed by their conjugate flags
  const char* s_lane = (const char*)s_q + ip * sizeof(fb_f4v);
  auto acc = [&](unsigned off, unsigned wa_bits, unsigned wb_bits) {
    const fb_f4v q = *(const fb_f4v*)(s_lane + off);
    const float wsa = __uint_as_float(wa_bits), wa = fabsf(wsa);
    const float wsb = __uint_as_float(wb_bits), wb = fabsf(wsb);
    a0 = fmaf(wa, q.x, a0);
    a1 = fmaf(wsa, q.y, a1);
    a2 = fmaf(wa, q.z, a2);
    a3 = fmaf(wsa, q.w, a3);
    b0 = fmaf(wb, q.x, b0);
    b1 = fmaf(wsb, q.y, b1);
    b2 = fmaf(wb, q.z, b2);
    b3 = fmaf(wsb, q.w, b3);
  };
  auto sum_entries = [&](int e0, int e1) {
    a0 = a1 = a2 = a3 = b0 = b1 = b2 = b3 = 0.f;
    for (int e = e0; e < e1; e += 3) {
      const fb_u4v v0 = s_e[e], v1 = s_e[e + 1], v2 = s_e[e + 2];
      acc(v0.x, v0.y, v0.z);
      acc(v0.w, v1.x, v1.y);
      acc(v1.z, v1.w, v2.x);
      acc(v2.y, v2.z, v2.w);
    }
  };
  if (nch == 1) {
    // one chunk: its entries go to LDS once; the image groups' values are prefetched two
    // groups ahead in two register sets
    if (ng == 0) return;
    load_meta_rec(chunks[t.c0]);
    fb_f4v qb[KQ];
    load_q_into(qr, gb);
    if (ng > 1) load_q_into(qb, gb + t.nsub);
    const int e0 = e0_n, e1 = e1_n;
    auto step = [&](fb_f4v (&cur)[KQ], int gi) {
      __syncthreads();  // the previous step's readers are done with LDS
#pragma unroll
      for (int k = 0; k < KQ; ++k)
        if (tid + k * NT < nl_n * IP) s_q[tid + k * NT] = cur[k];
      if (gi == 0) {
#pragma unroll
        for (int k = 0; k < KE; ++k)
          if (tid + k * NT < ne_n) s_e[tid + k * NT] = er[k];
      }
      __syncthreads();
      if (gi + 2 < ng) load_q_into(cur, gb + (gi + 2) * t.nsub);
      sum_entries(e0, e1);
      float4 ra = make_float4(a0, a1, a2, a3), rb = make_float4(b0, b1, b2, b3);
      gather_slots(ra, rb);
      put(gb + gi * t.nsub, ra, rb);
    };
    for (int gi = 0; gi < ng; gi += 2) {
      step(qr, gi);
      if (gi + 1 < ng) step(qb, gi + 1);
    }
    return;
  }
  // the chunk record the next load_meta_rec takes, read one chunk ahead so that the
  // entry and node loads of a chunk change do not wait for it
  SpreadChunk rec_next = chunks[t.c0];
  if (nsteps > 0) {
    load_meta_rec(rec_next);
    if (nch > 1) rec_next = chunks[t.c0 + 1];
    load_q(gb);
  }
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  float4 PA0 = z4, PB0 = z4, PA1 = z4, PB1 = z4;
  for (int s = 0; s < nsteps; ++s) {
    const int ci = s / ng, gi = s - ci * ng;
    const int g = gb + gi * t.nsub;
    __syncthreads();  // the previous step's readers are done with LDS
#pragma unroll
    for (int k = 0; k < KQ; ++k)
      if (tid + k * NT < nl_n * IP) s_q[tid + k * NT] = qr[k];
    if (gi == 0) {
#pragma unroll
      for (int k = 0; k < KE; ++k)
        if (tid + k * NT < ne_n) s_e[tid + k * NT] = er[k];
    }
    const int e0 = e0_n, e1 = e1_n;
    __syncthreads();
    const bool same_chunk = gi + 1 < ng;
    if (same_chunk) {
      load_q(g + t.nsub);
    } else if (ci + 1 < nch) {
      load_meta_rec(rec_next);
      if (ci + 2 < nch) rec_next = chunks[t.c0 + ci + 2];
    }
    sum_entries(e0, e1);
    if (!same_chunk && ci + 1 < nch) load_q(gb);
    float4 ra = make_float4(a0, a1, a2, a3), rb = make_float4(b0, b1, b2, b3);
    if (nch > 1) {
      auto upd = [&](float4& PA, float4& PB) {
        if (ci > 0) {
          ra = make_float4(PA.x + ra.x, PA.y + ra.y, PA.z + ra.z, PA.w + ra.w);
          rb = make_float4(PB.x + rb.x, PB.y + rb.y, PB.z + rb.z, PB.w + rb.w);
        }
        PA = ra;
        PB = rb;
      };
      if (gi == 0) upd(PA0, PB0);
      else upd(PA1, PB1);
    }
    if (ci == nch - 1) {
      gather_slots(ra, rb);
      put(g, ra, rb);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint cols, streaming form (conditions as for the forward streaming forms).  Same
// result as k_adj_cols.  Unit = (row m2, group of 16 image slots), groups fastest; its
// input is one contiguous run Y[m2][group][0..N)[16], loaded into registers while the
// previous unit is transformed; 16 in-place inverse FFTs (conjugate, forward FFT,
// conjugate) with LDS twiddles and LDS-only barriers; the columns x1 of the pixel range go
// to Zc [n][N/2+1][L].
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(1024, 4) void k_adj_cols_stream(const float2* __restrict__ Y, float2* __restrict__ Zc,
                                                            FftDesc fd, const float2* __restrict__ tw, int L,
                                                            int nimg, int ngrp, int U) {
  constexpr bool SW = grid_swizzle(NC);  // LDS layout of the transforms
  constexpr int G = kImgGroup, NM = stream_cap(NC, kGridStreamN);
  constexpr int PF = ((NC > 0 ? NC : NM) * G / 2 + 1023) / 1024;  // pairs of values per thread
  __shared__ __attribute__((aligned(16))) float2 s_buf[G * lds_span<NC, SW>(NM)];
  __shared__ float2 s_tw[NM];
  const int N = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(N), Nh = N / 2 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int total = Nh * ngrp;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int x0 = -((L - 1 + 1) / 2);
  const int nval = N * G / 2;
  for (int i = tid; i < N; i += nthr) s_tw[i] = tw[fd.tw_off + i];
  __syncthreads();
  // item e: the values of slots 2e % 16 and 2e % 16 + 1 at m1 = 2e / 16
  float4 pre[PF];
  auto load = [&](int u) {
    const float4* src = (const float4*)(Y + (size_t)u * N * G);
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * nthr;
      pre[q] = src[min(e, nval - 1)];  // unconditional: stays in flight (items past nval unused)
    }
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    const int m2 = u / ngrp, grp = u - m2 * ngrp;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * nthr;
      if (e < nval) {
        const int m1 = (2 * e) / G, c = (2 * e) & (G - 1);
        const float4 v = pre[q];
        s_buf[c * S + lds_pos<NC, SW>(m1)] = make_float2(v.x, -v.y);
        s_buf[(c + 1) * S + lds_pos<NC, SW>(m1)] = make_float2(v.z, -v.w);
      }
    }
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);
    fft_stream<NC, G, SW>(s_buf, S, fd, s_tw);
    {
      const int c = tid >> 6, i = grp * G + c;  // thread t writes image slot t / 64 at x1 = t % 64 + 64 q
      if (i < nimg) {
        float2* dst = Zc + ((size_t)i * Nh + m2) * L;
        for (int a = tid & 63; a < L; a += 64) {
          int pos = x0 + a;
          pos += (pos < 0) ? N : 0;
          dst[a] = cconj(s_buf[c * S + lds_pos<NC, SW>(pos)]);
        }
      }
    }
    stage_barrier<true>();
  }
}

// ---------------------------------------------------------------------------
// adjoint rows, streaming form (L even).  Same result as k_adj_rows.  Unit = (image, 16
// row pairs): rows a0 .. a0 + 31 of Zc for every m2 (runs of 32 values), loaded into
// registers while the previous unit is transformed.  Row pair (a, a + 1) forms one complex
// sequence z(m) = conj(h_a(m) + i h_b(m)) with the Hermitian completions
// h(m) = r(m) (m <= N/2), conj r(N - m) (above), placed at m and N - m directly.
// ---------------------------------------------------------------------------
template <int NC>
__global__ __launch_bounds__(1024, 4) void k_adj_rows_stream(const float2* __restrict__ Zc, float* __restrict__ img,
                                                            const float* __restrict__ deconv, FftDesc fd,
                                                            const float2* __restrict__ tw, int L, int nimg, int U) {
  constexpr bool SW = grid_swizzle(NC);  // LDS layout of the transforms
  constexpr int RP = 16, NM = stream_cap(NC, kGridStreamN);
  constexpr int PF = ((NM / 2 + 1) * RP + 1023) / 1024;  // row-pair values per thread
  __shared__ __attribute__((aligned(16))) float2 s_buf[RP * lds_span<NC, SW>(NM)];
  __shared__ float2 s_tw[NM];
  __shared__ float s_dec[NM / 2];
  const int N = NC > 0 ? NC : fd.n, S = lds_span<NC, SW>(N), Nh = N / 2 + 1;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nrb = ((L + 1) / 2 + RP - 1) / RP;
  const int total = nimg * nrb;
  const int u0 = xcd_remap(blockIdx.x, gridDim.x) * U;
  const int u1 = min(total, u0 + U);
  const int x0 = -((L - 1 + 1) / 2);
  const int nval = Nh * RP;
  for (int i = tid; i < N; i += nthr) s_tw[i] = tw[fd.tw_off + i];
  for (int i = tid; i < L; i += nthr) s_dec[i] = deconv[i];
  __syncthreads();
  // item e: rows a0 + 2 (e % 16) and the next one at m2 = e / 16 (one 16-byte pair; L even)
  float4 pre[PF];
  auto load = [&](int u) {
    const int im = u / nrb, a0 = 2 * RP * (u - im * nrb);
    const float2* src = Zc + (size_t)im * Nh * L;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * nthr;
      const int ms = e / RP, a = a0 + 2 * (e & (RP - 1));
      if (e < nval) pre[q] = a < L ? *(const float4*)(src + (size_t)ms * L + a) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  if (u0 < u1) load(u0);
  for (int u = u0; u < u1; ++u) {
    const int im = u / nrb, a0 = 2 * RP * (u - im * nrb);
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = tid + q * nthr;
      if (e < nval) {
        const int ms = e / RP, p = e & (RP - 1);
        float4 v = pre[q];  // (r_a(ms), r_{a+1}(ms))
        if (ms == 0 || 2 * ms == N) v.y = v.w = 0.f;
        float2* row = s_buf + p * S;
        row[lds_pos<NC, SW>(ms)] = make_float2(v.x - v.w, -(v.y + v.z));
        if (ms > 0 && 2 * ms < N) row[lds_pos<NC, SW>(N - ms)] = make_float2(v.x + v.w, v.y - v.z);
      }
    }
    stage_barrier<true>();
    if (u + 1 < u1) load(u + 1);
    fft_stream<NC, RP, SW>(s_buf, S, fd, s_tw);
    {
      const int r = tid >> 5, a = a0 + r;  // thread t writes row t / 32 at x2 = t % 32 + 32 q
      if (a < L) {
        float* dst = img + ((size_t)im * L + a) * L;
        const float2* row = s_buf + (r >> 1) * S;
        const float da = s_dec[a];
        for (int b = tid & 31; b < L; b += 32) {
          int pos = x0 + b;
          pos += (pos < 0) ? N : 0;
          const float2 z = row[lds_pos<NC, SW>(pos)];  // conj of the inverse transform
          dst[b] = ((r & 1) ? -z.y : z.x) * da * s_dec[b];
        }
      }
    }
    stage_barrier<true>();
  }
}

// ---------------------------------------------------------------------------
// adjoint cols: Y [N/2+1][group][N][16] -> Zc [n][N/2+1][L]: inverse FFT along m1, keep x1 in
// the pixel range.  workgroup = (row m2, CP consecutive image slots); transforms padded to N+1
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_adj_cols(const float2* __restrict__ Y, float2* __restrict__ Zc, FftDesc fd,
                           const float2* __restrict__ tw, int L, int nimg, int ngrp, int CP) {
  extern __shared__ float2 sm[];
  const int N = fd.n, Nh = N / 2 + 1, S = N + 1;
  float2* buf = sm;
  float2* tmp = sm + CP * S;
  const int m2 = blockIdx.y;
  const int i0 = blockIdx.x * CP;
  const int nc = min(CP, nimg - i0);
  // slot i0 + c of row m2: group (i0 + c) / 16, lane (i0 + c) % 16; slots vary fastest
  for (int i = threadIdx.x; i < nc * N; i += blockDim.x) {
    const int m1 = i / nc, c = i - m1 * nc, sl = i0 + c;
    buf[c * S + m1] = cconj(Y[(((size_t)m2 * ngrp + sl / kImgGroup) * N + m1) * kImgGroup + (sl & (kImgGroup - 1))]);
  }
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, nc, S, fd, tw);
  const int x0 = -((L - 1 + 1) / 2);
  for (int i = threadIdx.x; i < nc * L; i += blockDim.x) {
    int cidx = i / L, a = i - cidx * L;
    int pos = x0 + a;
    pos += (pos < 0) ? N : 0;
    Zc[((size_t)(i0 + cidx) * Nh + m2) * L + a] = cconj(res[cidx * S + pos]);
  }
}

// ---------------------------------------------------------------------------
// adjoint rows: Zc [n][N/2+1][L] -> images [n][L][L]
// two real rows per complex inverse FFT of the Hermitian-completed sequences
// ---------------------------------------------------------------------------
template <int FORM>
__global__ void k_adj_rows(const float2* __restrict__ Zc, float* __restrict__ img, const float* __restrict__ deconv,
                           FftDesc fd, const float2* __restrict__ tw, int L, int RP) {
  extern __shared__ float2 sm[];
  const int N = fd.n, Nh = N / 2 + 1;
  float2* buf = sm;
  float2* tmp = sm + RP * N;
  const int im = blockIdx.y;
  const int pair0 = blockIdx.x * RP;
  const int npairs = (L + 1) / 2;
  const int np = min(RP, npairs - pair0);
  const float2* src = Zc + (size_t)im * Nh * L;
  // h(m) = r(m) for m <= N/2, conj r(N-m) above; h(0), h(N/2) real.  z = conj(h_a + i h_b)
  for (int i = threadIdx.x; i < np * N; i += blockDim.x) {
    int p = i / N, m = i - p * N;
    int a = 2 * (pair0 + p);
    int ms = m <= N / 2 ? m : N - m;
    bool cj = m > N / 2;
    float2 ra = src[(size_t)ms * L + a];
    float2 rb = (a + 1 < L) ? src[(size_t)ms * L + a + 1] : make_float2(0.f, 0.f);
    if (ms == 0 || 2 * ms == N) {
      ra.y = 0.f;
      rb.y = 0.f;
    }
    if (cj) {
      ra.y = -ra.y;
      rb.y = -rb.y;
    }
    float2 h = make_float2(ra.x - rb.y, ra.y + rb.x);
    buf[p * N + m] = cconj(h);
  }
  __syncthreads();
  float2* res = run_fft<FORM>(buf, tmp, np, N, fd, tw);
  const int x0 = -((L - 1 + 1) / 2);
  float* dst = img + (size_t)im * L * L;
  for (int i = threadIdx.x; i < np * 2 * L; i += blockDim.x) {
    int p = i / (2 * L), rem = i - p * 2 * L, which = rem / L, b = rem - which * L;
    int a = 2 * (pair0 + p) + which;
    if (a >= L) continue;
    int pos = x0 + b;
    pos += (pos < 0) ? N : 0;
    float2 z = res[p * N + pos];  // conj of the inverse transform
    float v = which == 0 ? z.x : -z.y;
    dst[(size_t)a * L + b] = v * deconv[a] * deconv[b];
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Transforms per workgroup and FFT form.  The in-place form needs one LDS buffer
// (count * S complex values), the ping-pong forms two; either stays within
// kLdsBudget bytes so that two workgroups share one CU's 160 KiB of LDS.
constexpr int kLdsBudget = 72 * 1024;
constexpr int kFftThreads = 1024;
constexpr int kMaxTransforms = 16;
constexpr int kAngularUnits = 16;                  // (ring, group) units per streaming angular workgroup
constexpr int kGridUnits = 16;                     // units per streaming row / column workgroup
static_assert(kMaxTransforms <= kImgGroup, "an FFT workgroup's image slots map to lanes of one group");
// Units per workgroup of a streaming column launch: enough that the workgroups fill the
// device's resident slots (per_cu per compute unit) once, so no partly filled last round is
// left, and at least `floor` (the prefetch pipeline needs a few units to pay off).  (The
// row and angular launches keep a fixed count: measured, their several rounds balance
// better.)
static int stream_units(const Plan& pl, long long units, int per_cu, int floor) {
  const long long slots = (long long)pl.num_cus * per_cu;
  const long long u = (units + slots - 1) / slots;
  // a pass too small to give every resident slot `floor` units takes one round of
  // workgroups instead of a few long ones
  return (int)(units >= slots * floor ? u : std::max<long long>(1, u));
}
// Units per workgroup of the row and angular launches: `cap` when the pass fills the
// device several times over, fewer when it would leave resident slots idle.
static int fixed_units(const Plan& pl, long long units, int per_cu, int cap) {
  const long long slots = (long long)pl.num_cus * per_cu;
  return (int)std::max<long long>(1, std::min<long long>(cap, (units + slots - 1) / slots));
}
struct FftLaunch {
  int count;
  int form;
  size_t lds;
};
static FftLaunch fft_launch(const FftDesc& d, int S) {
  int cap = fft_inplace_capacity(d, kFftThreads);
  if (cap > 0) {
    int c = std::min(kMaxTransforms, std::min(cap / d.n, kLdsBudget / (8 * S)));
    if (c >= 1) return FftLaunch{c, FFT_INPLACE, (size_t)c * S * sizeof(float2)};
  }
  bool special = true;
  for (int s = 0; s < d.nstage; ++s) {
    int R = d.radix[s];
    special = special && (R == 2 || R == 3 || R == 4 || R == 5 || R == 8);
  }
  int c = std::max(1, std::min(kMaxTransforms, kLdsBudget / (16 * S)));
  return FftLaunch{c, special ? FFT_PINGPONG : FFT_GENERIC, 2 * (size_t)c * S * sizeof(float2)};
}

#define FB_LAUNCH_FFT(KERNEL, form, grid, block, lds, st, ...)                                  \
  do {                                                                                          \
    if ((form) == FFT_INPLACE)                                                                  \
      hipLaunchKernelGGL(KERNEL<FFT_INPLACE>, grid, block, lds, st, __VA_ARGS__);               \
    else if ((form) == FFT_PINGPONG)                                                            \
      hipLaunchKernelGGL(KERNEL<FFT_PINGPONG>, grid, block, lds, st, __VA_ARGS__);              \
    else                                                                                        \
      hipLaunchKernelGGL(KERNEL<FFT_GENERIC>, grid, block, lds, st, __VA_ARGS__);               \
  } while (0)

size_t gather_lds_bytes();

hipError_t configure_kernels() {
  hipError_t e0 = hipFuncSetAttribute((const void*)k_fwd_gather<kGatherW, kGatherCell, kGatherImages, kGatherThreads>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)gather_lds_bytes());
  if (e0 != hipSuccess) return e0;
#define FB_FORMS(K) (const void*)K<FFT_INPLACE>, (const void*)K<FFT_PINGPONG>, (const void*)K<FFT_GENERIC>
  const void* fns[] = {FB_FORMS(k_fwd_rows),    FB_FORMS(k_fwd_cols), FB_FORMS(k_fwd_angular),
                       FB_FORMS(k_adj_angular), FB_FORMS(k_adj_cols), FB_FORMS(k_adj_rows)};
#undef FB_FORMS
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBudget);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Transform lengths the streaming kernels take: powers of two up to nmax whose radices are
// 8 and 4 (compiled for 64 to 512, run-time form below 64), and the mixed-radix 720.
static bool stream_length(const FftDesc& d, int nmax) {
  return d.n == kStreamMixedN || (d.n <= nmax && fft_inplace_capacity(d, kFftThreads) >= kImgGroup * d.n);
}
// Resident workgroups per compute unit of a streaming kernel of length n (its LDS).
static int stream_per_cu(int n) { return n > kGridStreamN ? 1 : 2; }

// Launch a streaming kernel compiled for its transform length n (720, or a power of two
// from 64 to 512), or its run-time-length form for any other n.
#define FB_LAUNCH_STREAM(K, n, grid, st, ...)                                               \
  do {                                                                                      \
    switch (n) {                                                                            \
      case kStreamMixedN:                                                                   \
        hipLaunchKernelGGL(K<kStreamMixedN>, grid, dim3(1024), 0, st, __VA_ARGS__);         \
        break;                                                                              \
      case 512: hipLaunchKernelGGL(K<512>, grid, dim3(1024), 0, st, __VA_ARGS__); break;    \
      case 256: hipLaunchKernelGGL(K<256>, grid, dim3(1024), 0, st, __VA_ARGS__); break;    \
      case 128: hipLaunchKernelGGL(K<128>, grid, dim3(1024), 0, st, __VA_ARGS__); break;    \
      case 64: hipLaunchKernelGGL(K<64>, grid, dim3(1024), 0, st, __VA_ARGS__); break;      \
      default: hipLaunchKernelGGL(K<0>, grid, dim3(1024), 0, st, __VA_ARGS__); break;       \
    }                                                                                       \
  } while (0)

hipError_t launch_forward_nufft(const Plan& pl, const float* images, int nimg, float2* bufA, float2* bufB,
                                hipStream_t st) {
  const int N = pl.N, L = pl.L;
  const int ngrp = (nimg + kImgGroup - 1) / kImgGroup;
  // streaming forms: 16 transforms in place with 1024 threads; the inputs of one unit (32
  // rows or 16 columns of L <= N / 2 values) are held in registers, the rows as float4
  // (the columns form reads each image row in blocks of 64 and clamps only the last block,
  // so L must reach into that block: true whenever N is the smallest 2,3,5-smooth even number
  // >= 2L, as the plan takes it)
  const bool stream_ok =
      stream_length(pl.fft_grid, kGridStreamN) && L % 4 == 0 && L > 64 * (cols_stream_blocks(N) - 1);
  if (stream_ok) {
    const int nrb = ((L + 1) / 2 + 15) / 16;
    const long long ur = (long long)nimg * nrb;
    const int Ur = fixed_units(pl, ur, stream_per_cu(N), kGridUnits);
    pl.prof.begin(ST_FWD_ROWS, st);
    FB_LAUNCH_STREAM(k_fwd_rows_stream, N, dim3((unsigned)((ur + Ur - 1) / Ur)), st,
                       images, bufA, pl.d_deconv, pl.fft_grid, pl.d_tw, L, pl.M2, pl.hw, nimg, Ur);
    pl.prof.end(st);
    const long long uc = (long long)pl.M2 * ngrp;
    pl.prof.begin(ST_FWD_COLS, st);
    const int Uc = stream_units(pl, uc, stream_per_cu(N), kGridUnits);
    FB_LAUNCH_STREAM(k_fwd_cols_stream, N, dim3((unsigned)((uc + Uc - 1) / Uc)), st,
                       bufA, bufB, pl.fft_grid, pl.d_tw, (const int2*)pl.d_gcols, L, pl.M2, nimg, ngrp, Uc);
    pl.prof.end(st);
  } else {
    FftLaunch fr = fft_launch(pl.fft_grid, N + 1);
    dim3 g1((unsigned)(((L + 1) / 2 + fr.count - 1) / fr.count), (unsigned)nimg);
    pl.prof.begin(ST_FWD_ROWS, st);
    FB_LAUNCH_FFT(k_fwd_rows, fr.form, g1, dim3(kFftThreads), fr.lds, st, images, bufA, pl.d_deconv, pl.fft_grid,
                  pl.d_tw, L, pl.M2, pl.hw, fr.count, make_fastdiv(L));
    pl.prof.end(st);
    FftLaunch fc = fft_launch(pl.fft_grid, N + 1);
    dim3 g2((unsigned)((ngrp * kImgGroup + fc.count - 1) / fc.count), (unsigned)pl.M2);
    pl.prof.begin(ST_FWD_COLS, st);
    FB_LAUNCH_FFT(k_fwd_cols, fc.form, g2, dim3(kFftThreads), fc.lds, st, bufA, bufB, pl.fft_grid, pl.d_tw, L,
                  pl.M2, nimg, ngrp, fc.count, make_fastdiv(L));
    pl.prof.end(st);
  }
  constexpr int IG = kGatherImages;
  const int nitems = (int)pl.gitems.size();
  dim3 g3((unsigned)nitems, (unsigned)ngrp);
  pl.prof.begin(ST_FWD_GATHER, st);
  hipLaunchKernelGGL((k_fwd_gather<kGatherW, kGatherCell, IG, kGatherThreads>), g3, dim3(kGatherThreads),
                     gather_lds_bytes(), st, bufB, bufA,
                     pl.d_gitems, pl.d_gnodes, nitems, N, pl.M2, pl.H, ngrp);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_forward_angular(const Plan& pl, const float2* P, float2* Fh, int nimg, hipStream_t st) {
  const int ngrp = (nimg + kImgGroup - 1) / kImgGroup;
  const float scale = (float)(2.0 * 3.14159265358979323846 / pl.n_theta);
  const bool stream_ok = pl.H % 8 == 0 && stream_length(pl.fft_ang, kAngStreamH) && pl.k_max < pl.H;
  if (stream_ok) {
    const int units = pl.n_xi * ngrp;
    const int U = fixed_units(pl, units, stream_per_cu(pl.H), kAngularUnits);
    pl.prof.begin(ST_FWD_ANGULAR, st);
    FB_LAUNCH_STREAM(k_fwd_angular_stream, pl.H, dim3((unsigned)((units + U - 1) / U)), st, P,
                       Fh, pl.fft_ang, pl.d_tw, pl.d_angtw, pl.d_kring, pl.n_xi, pl.k_max, ngrp, U, scale);
    pl.prof.end(st);
    return hipGetLastError();
  }
  FftLaunch fa = fft_launch(pl.fft_ang, pl.H + 1);
  dim3 g((unsigned)((ngrp * kImgGroup + fa.count - 1) / fa.count), (unsigned)pl.n_xi);
  pl.prof.begin(ST_FWD_ANGULAR, st);
  FB_LAUNCH_FFT(k_fwd_angular, fa.form, g, dim3(kFftThreads), fa.lds, st, P, Fh, pl.fft_ang, pl.d_tw, pl.d_angtw,
                pl.n_xi, pl.k_max, ngrp, fa.count, scale);
  pl.prof.end(st);
  return hipGetLastError();
}

hipError_t launch_adjoint_angular(const Plan& pl, const float2* D, float2* Q, int nimg, hipStream_t st) {
  const int ngrp = (nimg + kImgGroup - 1) / kImgGroup;
  const bool stream_ok = pl.H % 8 == 0 && stream_length(pl.fft_ang, kAngStreamH) && pl.k_max < pl.H;
  if (stream_ok) {
    const long long units = (long long)pl.n_xi * ngrp;
    const int U = fixed_units(pl, units, stream_per_cu(pl.H), kAngularUnits);
    const float sc = (float)(2.0 * 3.14159265358979323846 / pl.n_theta);
    pl.prof.begin(ST_ADJ_ANGULAR, st);
    FB_LAUNCH_STREAM(k_adj_angular_stream, pl.H, dim3((unsigned)((units + U - 1) / U)), st, D, Q,
                       pl.fft_ang, pl.d_tw, pl.d_angtw, pl.n_xi, pl.k_max, nimg, ngrp, U, sc);
    pl.prof.end(st);
    return hipGetLastError();
  }
  FftLaunch fa = fft_launch(pl.fft_ang, pl.H + 1);
  dim3 g((unsigned)pl.n_xi, (unsigned)((ngrp * kImgGroup + fa.count - 1) / fa.count));
  const float scale = (float)(2.0 * 3.14159265358979323846 / pl.n_theta);
  pl.prof.begin(ST_ADJ_ANGULAR, st);
  FB_LAUNCH_FFT(k_adj_angular, fa.form, g, dim3(kFftThreads), fa.lds, st, D, Q, pl.fft_ang, pl.d_tw, pl.d_angtw,
                pl.n_xi, pl.k_max, nimg, ngrp, fa.count, scale);
  pl.prof.end(st);
  return hipGetLastError();
}

int64_t spread_max_images(const Plan& pl) {
  // the spread addresses one pass's polar values (n_xi x groups x H x 8 16-byte vectors)
  // with 32-bit offsets
  const int64_t per_group = (int64_t)pl.n_xi * pl.H * (kImgGroup / 2);
  return (int64_t)(0xffffffffull / (uint64_t)per_group) * kImgGroup;
}

hipError_t launch_adjoint_nufft(const Plan& pl, const float2* Q, int nimg, float2* bufA, float2* bufB,
                                float* images, hipStream_t st) {
  const int N = pl.N, L = pl.L, Nh = N / 2 + 1;
  const int ngrp = (nimg + kImgGroup - 1) / kImgGroup;
  constexpr int NT = kSpreadPairs * kImgGroup / 2;
  const int nsl = (ngrp + kSpreadSlice - 1) / kSpreadSlice;
  const size_t nblk = pl.sblocks.size() * (size_t)nsl;
  if (nblk > 0x7fffffffu || nimg > spread_max_images(pl)) return hipErrorInvalidValue;
  pl.prof.begin(ST_ADJ_SPREAD, st);
  hipLaunchKernelGGL((k_adj_spread<NT>), dim3((unsigned)nblk), dim3(NT), 0, st, Q, bufB, pl.d_stiles,
                     pl.d_sblocks, pl.d_schunks, pl.d_snodes, pl.d_sseg, pl.d_sslot, pl.d_sent, N, Nh, pl.H, ngrp,
                     nsl);
  pl.prof.end(st);
  const bool stream_ok = stream_length(pl.fft_grid, kGridStreamN) && L % 2 == 0;
  if (stream_ok) {
    const long long uc = (long long)Nh * ngrp;
    pl.prof.begin(ST_ADJ_COLS, st);
    const int Uc = stream_units(pl, uc, 1, kGridUnits);
    FB_LAUNCH_STREAM(k_adj_cols_stream, N, dim3((unsigned)((uc + Uc - 1) / Uc)), st,
                       bufB, bufA, pl.fft_grid, pl.d_tw, L, nimg, ngrp, Uc);
    pl.prof.end(st);
    const long long ur = (long long)nimg * (((L + 1) / 2 + 15) / 16);
    pl.prof.begin(ST_ADJ_ROWS, st);
    const int Ur = stream_units(pl, ur, 1, kGridUnits);
    FB_LAUNCH_STREAM(k_adj_rows_stream, N, dim3((unsigned)((ur + Ur - 1) / Ur)), st,
                       bufA, images, pl.d_deconv, pl.fft_grid, pl.d_tw, L, nimg, Ur);
    pl.prof.end(st);
    return hipGetLastError();
  }
  FftLaunch fc = fft_launch(pl.fft_grid, N + 1);
  dim3 g2((unsigned)((nimg + fc.count - 1) / fc.count), (unsigned)Nh);
  pl.prof.begin(ST_ADJ_COLS, st);
  FB_LAUNCH_FFT(k_adj_cols, fc.form, g2, dim3(kFftThreads), fc.lds, st, bufB, bufA, pl.fft_grid, pl.d_tw, L, nimg,
                ngrp, fc.count);
  pl.prof.end(st);
  FftLaunch fr = fft_launch(pl.fft_grid, N);
  dim3 g3((unsigned)(((L + 1) / 2 + fr.count - 1) / fr.count), (unsigned)nimg);
  pl.prof.begin(ST_ADJ_ROWS, st);
  FB_LAUNCH_FFT(k_adj_rows, fr.form, g3, dim3(kFftThreads), fr.lds, st, bufA, images, pl.d_deconv, pl.fft_grid,
                pl.d_tw, L, fr.count);
  pl.prof.end(st);
  return hipGetLastError();
}

}  // namespace fb
