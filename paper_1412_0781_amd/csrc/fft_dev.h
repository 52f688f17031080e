// Mixed-radix Stockham FFT on LDS for gfx950 workgroups.
//
// `count` independent transforms of length d.n sit at buf + t * stride (t <
// count) in LDS.  Each stage reads one buffer and writes the other (autosort,
// natural order out); the caller passes both and receives the one holding the
// result.  Forward transform: X_m = sum_x x_x exp(-2 pi i m x / n).  The
// inverse (exp(+...), unnormalised) is obtained as conj(FFT(conj(x))).
#pragma once
#include <hip/hip_runtime.h>

#include "plan.h"

namespace fb {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// In-register DFT of length R with the forward sign.
template <int R>
struct Dft;

template <>
struct Dft<2> {
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <>
struct Dft<4> {
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    float2 b0 = cadd(v[1], v[3]), b1 = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd(a1, b1);
    v[3] = csub(a1, b1);
  }
};

template <>
struct Dft<8> {
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    const float r = 0.70710678118654752440f;
    // radix-2 over pairs (0,4),(1,5),(2,6),(3,7)
    float2 a[4], b[4];
    for (int i = 0; i < 4; ++i) {
      a[i] = cadd(v[i], v[i + 4]);
      b[i] = csub(v[i], v[i + 4]);
    }
    // twiddles w8^i on b
    b[1] = make_float2(r * (b[1].x + b[1].y), r * (b[1].y - b[1].x));
    b[2] = cmul_mi(b[2]);
    b[3] = make_float2(r * (b[3].y - b[3].x), -r * (b[3].x + b[3].y));
    // two radix-4 DFTs
    Dft<4>::run(a, nullptr, 0, 0);
    Dft<4>::run(b, nullptr, 0, 0);
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = a[i];
      v[2 * i + 1] = b[i];
    }
  }
};

template <>
struct Dft<3> {
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    const float c1 = -0.5f, s1 = -0.86602540378443864676f;  // exp(-2 pi i / 3)
    float2 t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    float2 m = make_float2(v[0].x + c1 * t1.x, v[0].y + c1 * t1.y);
    float2 n = make_float2(-s1 * t2.y, s1 * t2.x);  // i s1 t2
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, n);
    v[2] = csub(m, n);
  }
};

template <>
struct Dft<5> {
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    const float s1 = -0.95105651629515357212f, s2 = -0.58778525229247312917f;  // forward sign
    float2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    float2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    float2 x0 = v[0];
    float2 m1 = make_float2(x0.x + c1 * t1.x + c2 * t2.x, x0.y + c1 * t1.y + c2 * t2.y);
    float2 m2 = make_float2(x0.x + c2 * t1.x + c1 * t2.x, x0.y + c2 * t1.y + c1 * t2.y);
    // i*(s1 t3 + s2 t4) and i*(s2 t3 - s1 t4)
    float2 u1 = make_float2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    float2 u2 = make_float2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    float2 iu1 = make_float2(-u1.y, u1.x), iu2 = make_float2(-u2.y, u2.x);
    v[0] = make_float2(x0.x + t1.x + t2.x, x0.y + t1.y + t2.y);
    v[1] = cadd(m1, iu1);
    v[4] = csub(m1, iu1);
    v[2] = cadd(m2, iu2);
    v[3] = csub(m2, iu2);
  }
};

// Prime-factor (Good-Thomas) DFT of length N1 * N2 with coprime factors: no twiddles between
// the two passes.  The input x at (N2 n1 + N1 n2) mod N forms N2 DFTs of length N1 over n1;
// their outputs at k1 form N1 DFTs of length N2 over n2; output (k1, k2) is X at
// (N2 u k1 + N1 v k2) mod N, with u N2 = 1 mod N1 and v N1 = 1 mod N2 (Chinese remainders).
constexpr int mod_inverse(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}
template <int N1, int N2>
struct DftPfa {
  static constexpr int N = N1 * N2, U = mod_inverse(N2 % N1, N1), V = mod_inverse(N1 % N2, N2);
  __device__ __forceinline__ static void run(float2* v, const float2*, int, int) {
    float2 a[N2][N1];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2)
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) a[n2][n1] = v[(N2 * n1 + N1 * n2) % N];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) Dft<N1>::run(a[n2], nullptr, 0, 0);
    float2 b[N1][N2];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) b[k1][n2] = a[n2][k1];
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) Dft<N2>::run(b[k1], nullptr, 0, 0);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) v[(N2 * U * k1 + N1 * V * k2) % N] = b[k1][k2];
  }
};
template <>
struct Dft<12> : DftPfa<4, 3> {};

// Generic odd prime R <= 31: direct O(R^2) DFT with roots taken from the twiddle table of length n.
template <int RMAX>
__device__ __forceinline__ void dft_generic(float2* v, int R, const float2* tw, int n) {
  float2 out[RMAX];
  int step = n / R;
  for (int m = 0; m < R; ++m) {
    float2 s = make_float2(0.f, 0.f);
    for (int x = 0; x < R; ++x) s = cadd(s, cmul(v[x], tw[((m * x) % R) * step]));
    out[m] = s;
  }
  for (int m = 0; m < R; ++m) v[m] = out[m];
}

// One Stockham stage of radix R for `count` transforms (stride `stride`) of length n.
template <int R>
__device__ __forceinline__ void fft_stage_r(const float2* __restrict__ in, float2* __restrict__ out, int n, int Ns,
                                            int count, int stride, const float2* __restrict__ tw, int tid,
                                            int nthr, FastDiv dnb, FastDiv dns) {
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  for (int idx = tid; idx < count * nb; idx += nthr) {
    int t = dnb.div(idx), j = idx - t * nb;
    const float2* src = in + t * stride;
    float2* dst = out + t * stride;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    int k = j - dns.div(j) * Ns;
    if (k) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * twstep]);
    }
    Dft<R>::run(v, tw, n, R);
    int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

__device__ __forceinline__ void fft_stage_generic(const float2* __restrict__ in, float2* __restrict__ out, int n,
                                                  int R, int Ns, int count, int stride,
                                                  const float2* __restrict__ tw, int tid, int nthr, FastDiv dnb,
                                                  FastDiv dns) {
  const int nb = n / R;
  const int twstep = n / (Ns * R);
  for (int idx = tid; idx < count * nb; idx += nthr) {
    int t = dnb.div(idx), j = idx - t * nb;
    const float2* src = in + t * stride;
    float2* dst = out + t * stride;
    float2 v[31];
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    int k = j - dns.div(j) * Ns;
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(k * r * twstep) % n]);
    dft_generic<31>(v, R, tw, n);
    int base = (j - k) * R + k;
    for (int r = 0; r < R; ++r) dst[base + r * Ns] = v[r];
  }
}

// Full forward FFT; buf holds the input and must be followed by scratch of the
// same size at `tmp`.  Returns the pointer holding the result.  All threads of
// the block must call it; it synchronises the block between stages.
template <bool GENERIC>
__device__ inline float2* fft_lds(float2* buf, float2* tmp, int count, int stride, const FftDesc& d,
                                  const float2* __restrict__ tw_all) {
  const float2* tw = tw_all + d.tw_off;
  const int tid = threadIdx.x, nthr = blockDim.x;
  float2* in = buf;
  float2* out = tmp;
  int Ns = 1;
  for (int s = 0; s < d.nstage; ++s) {
    int R = d.radix[s];
    switch (R) {
      case 8: fft_stage_r<8>(in, out, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]); break;
      case 4: fft_stage_r<4>(in, out, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]); break;
      case 2: fft_stage_r<2>(in, out, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]); break;
      case 3: fft_stage_r<3>(in, out, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]); break;
      case 5: fft_stage_r<5>(in, out, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]); break;
      default:
        if constexpr (GENERIC) fft_stage_generic(in, out, d.n, R, Ns, count, stride, tw, tid, nthr, d.dnb[s], d.dns[s]);
        break;
    }
    __syncthreads();
    float2* t = in;
    in = out;
    out = t;
    Ns *= R;
  }
  return in;
}

// In-place variant: a stage first reads every butterfly input of the calling
// thread into registers, then (after a barrier) writes its outputs over the
// same buffer, so one LDS buffer suffices.  A thread holds at most VMAX values;
// the caller guarantees count * n <= fft_inplace_capacity(d, nthreads) and that
// every radix of d is 4 or 8 (each supported radix adds its register arrays to
// the kernel, so the in-place form is kept to the two that cover 2^k lengths).
// Barrier between FFT stages.  The plain form is __syncthreads().  The LDS-only form
// waits for this wave's LDS operations and meets the other waves, without waiting
// for its outstanding global memory operations (used while a copy from HBM into
// another LDS buffer is in flight; the caller's twiddles must then be in LDS too).
template <bool LDS_ONLY>
__device__ __forceinline__ void stage_barrier() {
  if constexpr (LDS_ONLY)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  else
    __syncthreads();
}

// Padded LDS layout of one transform: element i sits at fpad(i), one spare slot after every
// 32 and every 64 elements.  The radix-8 stages read with a stride of n/8 elements and
// write with strides of 8 and 64; in the plain layout those writes put 16 and 8 lanes on
// one bank, in the padded one at most 3 (the least for 64 lanes of 8 bytes is 2).
__host__ __device__ constexpr int fpad(int i) { return i + (i >> 5) + (i >> 6); }
template <bool PAD>
__device__ __forceinline__ int fidx(int i) {
  if constexpr (PAD)
    return fpad(i);
  else
    return i;
}

template <int R, int VMAX, bool LDS_ONLY = false, bool PAD = false>
__device__ __forceinline__ void fft_stage_inplace(float2* buf, int n, int Ns, int count, int stride,
                                                  const float2* __restrict__ tw, int tid, int nthr, FastDiv dnb,
                                                  FastDiv dns) {
  constexpr int BM = VMAX / R;
  const int nb = n / R;
  const int total = count * nb;
  const int twstep = n / (Ns * R);
  // Global twiddle tables are loaded before the barrier, so their latency overlaps the
  // wait for the other waves; LDS tables (LDS_ONLY) are read after it, saving registers.
  constexpr int WR = LDS_ONLY ? 1 : R;
  float2 v[BM][R], w[BM][WR];
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    int idx = tid + b * nthr;
    if (idx < total) {
      int t = dnb.div(idx), j = idx - t * nb;
      const float2* src = buf + t * stride;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[fidx<PAD>(j + r * nb)];
      if constexpr (!LDS_ONLY) {
        int k = j - dns.div(j) * Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) w[b][r] = tw[k * r * twstep];
      }
    }
  }
  stage_barrier<LDS_ONLY>();
#pragma unroll
  for (int b = 0; b < BM; ++b) {
    int idx = tid + b * nthr;
    if (idx < total) {
      int t = dnb.div(idx), j = idx - t * nb;
      int k = j - dns.div(j) * Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], LDS_ONLY ? tw[k * r * twstep] : w[b][r % WR]);  // tw[0] = 1
      Dft<R>::run(v[b], tw, n, R);
      float2* dst = buf + t * stride;
      int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[fidx<PAD>(base + r * Ns)] = v[b][r];
    }
  }
  stage_barrier<LDS_ONLY>();
}

constexpr int kFftVmax = 8;  // values per thread: one radix-8 butterfly or two radix-4

// Largest count * n the in-place FFT can take with nthr threads (0 if a radix is unsupported).
inline int fft_inplace_capacity(const FftDesc& d, int nthr) {
  int cap = 1 << 30;
  for (int s = 0; s < d.nstage; ++s) {
    int R = d.radix[s];
    if (R != 4 && R != 8) return 0;
    cap = cap < (kFftVmax / R) * R * nthr ? cap : (kFftVmax / R) * R * nthr;
  }
  return cap;
}

// tw: the twiddle table of this transform length (tw_all + d.tw_off).
template <bool LDS_ONLY = false, bool PAD = false>
__device__ inline void fft_lds_inplace_tw(float2* buf, int count, int stride, const FftDesc& d,
                                          const float2* __restrict__ tw) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  int Ns = 1;
  for (int s = 0; s < d.nstage; ++s) {
    int R = d.radix[s];
    switch (R) {
      case 8:
        fft_stage_inplace<8, kFftVmax, LDS_ONLY, PAD>(buf, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s],
                                                      d.dns[s]);
        break;
      default:
        fft_stage_inplace<4, kFftVmax, LDS_ONLY, PAD>(buf, d.n, Ns, count, stride, tw, tid, nthr, d.dnb[s],
                                                      d.dns[s]);
        break;
    }
    Ns *= R;
  }
}

// The same in-place padded FFT for a power-of-two length N known at compile time, with
// COUNT transforms at stride STRIDE and NT threads: stage radices follow the plan's rule
// (radix 8 while the remaining length is a multiple of 8 other than 16, then 4), and
// every index and twiddle position is a shift or mask, most LDS offsets immediates.
// Same operations in the same order as the run-time form (the first stage's unit
// twiddles are skipped: multiplying by exactly 1 changes nothing).
constexpr int pow2_stage_radix(int rem) { return (rem % 8 == 0 && rem != 16) ? 8 : 4; }

// LDS layout of one transform in the compile-time streaming forms: element i of a length-N
// transform sits at lds_pos<N, SW>(i), and transforms follow each other every
// lds_span<N, SW>(N) elements.  SW = false: the padded layout fpad.  SW = true: powers of two
// swizzle each aligned run of 16 elements by i / 16, 720 swizzles runs of 32 by i / 64; both
// stay inside their runs (no padding), and a span of N + 2 puts the same element of 16
// side-by-side transforms on distinct banks.  Measured, the swizzle pays at 720 in every
// streaming kernel and at 512 in the four grid kernels, where the stride-8 and stride-64
// butterfly writes meet fewer bank conflicts; elsewhere the padded layout is as fast or
// faster (the swizzled addresses take more registers).  The run-time-length form (N = 0)
// is always padded.
constexpr bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
template <int N, bool SW>
__host__ __device__ constexpr int lds_pos(int i) {
  if constexpr (N == 0 || !SW)
    return fpad(i);
  else if constexpr (is_pow2(N))
    return i ^ ((i >> 4) & 15);
  else
    return i ^ ((i >> 6) & 31);
}
template <int N, bool SW>
__host__ __device__ constexpr int lds_span(int n) {
  if constexpr (N == 0 || !SW)
    return fpad(n - 1) + 2;
  else
    return n + 2;
}
// the layouts chosen per kernel family: grid (rows, columns and their transposes), angular
constexpr bool grid_swizzle(int nc) { return nc == 720 || nc == 512; }
constexpr bool angular_swizzle(int nc) { return nc == 720; }
// the layout of length N maps [0, N) one to one into [0, lds_span - 1)
template <int N, bool SW>
constexpr bool lds_layout_ok() {
  bool seen[lds_span<N, SW>(N)] = {};
  for (int i = 0; i < N; ++i) {
    const int p = lds_pos<N, SW>(i);
    if (p < 0 || p > lds_span<N, SW>(N) - 2 || seen[p]) return false;
    seen[p] = true;
  }
  return true;
}
static_assert(lds_layout_ok<64, true>() && lds_layout_ok<256, true>() && lds_layout_ok<512, true>() &&
                  lds_layout_ok<720, true>() && lds_layout_ok<512, false>() && lds_layout_ok<720, false>(),
              "each streaming layout is one to one within its span");

template <int N, int R, int NS, int COUNT, int STRIDE, int NT, bool SW>
__device__ __forceinline__ void fft_stage_pow2(float2* buf, const float2* __restrict__ tw, unsigned tid) {
  constexpr unsigned NB = N / R, TWS = N / (NS * R), BM = kFftVmax / R, TOTAL = COUNT * NB;
  static_assert((N & (N - 1)) == 0 && TOTAL <= BM * NT, "one pass of the threads covers every butterfly");
  float2 v[BM][R];
#pragma unroll
  for (unsigned b = 0; b < BM; ++b) {
    const unsigned idx = tid + b * NT;
    if (idx < TOTAL) {
      const unsigned t = idx / NB, j = idx % NB;
      const float2* src = buf + t * STRIDE;
#pragma unroll
      for (unsigned r = 0; r < R; ++r) v[b][r] = src[lds_pos<N, SW>(j + r * NB)];
    }
  }
  stage_barrier<true>();
#pragma unroll
  for (unsigned b = 0; b < BM; ++b) {
    const unsigned idx = tid + b * NT;
    if (idx < TOTAL) {
      const unsigned t = idx / NB, j = idx % NB, k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (unsigned r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[k * r * TWS]);
      }
      Dft<R>::run(v[b], tw, N, R);
      float2* dst = buf + t * STRIDE;
      const unsigned base = (j - k) * R + k;
#pragma unroll
      for (unsigned r = 0; r < R; ++r) dst[lds_pos<N, SW>(base + r * NS)] = v[b][r];
    }
  }
  stage_barrier<true>();
}

template <int N, int COUNT, int STRIDE, int NT, bool SW, int NS = 1>
__device__ __forceinline__ void fft_pow2_inplace(float2* buf, const float2* __restrict__ tw, unsigned tid) {
  if constexpr (NS < N) {
    constexpr int R = pow2_stage_radix(N / NS);
    fft_stage_pow2<N, R, NS, COUNT, STRIDE, NT, SW>(buf, tw, tid);
    fft_pow2_inplace<N, COUNT, STRIDE, NT, SW, NS * R>(buf, tw, tid);
  }
}

// The same in-place padded stage for a compile-time length that is not a power of two
// (2, 3, 5-smooth, e.g. 720 = 12 * 12 * 5): radix 12 (a prime-factor 4 x 3 butterfly)
// while the remaining length allows it, then 8, 4, 5, 3, 2, so that 720 takes three
// stages instead of the five of its prime-power split.  A thread takes
// ceil(COUNT * N / R / NT) butterflies per stage.
constexpr int mixed_stage_radix(int rem) {
  return rem % 12 == 0 ? 12 : rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 5 == 0 ? 5 : rem % 3 == 0 ? 3 : 2;
}
constexpr bool mixed_supported(int n) {
  while (n > 1) {
    const int r = mixed_stage_radix(n);
    if (n % r != 0) return false;
    n /= r;
  }
  return n == 1;
}

template <int N, int R, int NS, int COUNT, int STRIDE, int NT, bool SW>
__device__ __forceinline__ void fft_stage_mixed(float2* buf, const float2* __restrict__ tw, unsigned tid) {
  constexpr unsigned NB = N / R, TWS = N / (NS * R), TOTAL = COUNT * NB, BM = (TOTAL + NT - 1) / NT;
  static_assert(N % R == 0, "the radix divides the remaining length");
  float2 v[BM][R];
#pragma unroll
  for (unsigned b = 0; b < BM; ++b) {
    const unsigned idx = tid + b * NT;
    if (idx < TOTAL) {
      const unsigned t = idx / NB, j = idx % NB;
      const float2* src = buf + t * STRIDE;
#pragma unroll
      for (unsigned r = 0; r < R; ++r) v[b][r] = src[lds_pos<N, SW>(j + r * NB)];
    }
  }
  stage_barrier<true>();
#pragma unroll
  for (unsigned b = 0; b < BM; ++b) {
    const unsigned idx = tid + b * NT;
    if (idx < TOTAL) {
      const unsigned t = idx / NB, j = idx % NB, k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (unsigned r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], tw[k * r * TWS]);
      }
      Dft<R>::run(v[b], tw, N, R);
      float2* dst = buf + t * STRIDE;
      const unsigned base = (j - k) * R + k;
#pragma unroll
      for (unsigned r = 0; r < R; ++r) dst[lds_pos<N, SW>(base + r * NS)] = v[b][r];
    }
  }
  stage_barrier<true>();
}

template <int N, int COUNT, int STRIDE, int NT, bool SW, int NS = 1>
__device__ __forceinline__ void fft_mixed_inplace(float2* buf, const float2* __restrict__ tw, unsigned tid) {
  if constexpr (NS < N) {
    constexpr int R = mixed_stage_radix(N / NS);
    fft_stage_mixed<N, R, NS, COUNT, STRIDE, NT, SW>(buf, tw, tid);
    fft_mixed_inplace<N, COUNT, STRIDE, NT, SW, NS * R>(buf, tw, tid);
  }
}

// The FFT of the streaming kernels (1024 threads, in-place layout lds_pos, LDS twiddles):
// the compile-time forms for NC > 0 (NC = d.n; powers of two and the mixed-radix lengths
// above), the run-time form for NC = 0.  In the compile-time forms the thread index
// passes through an empty asm statement, so that the stages' addresses are formed here
// rather than held in registers across the caller's loop (they depend on nothing else
// that changes).
template <int NC, int COUNT, bool SW>
__device__ __forceinline__ void fft_stream(float2* buf, int stride, const FftDesc& d, const float2* __restrict__ tw) {
  if constexpr (NC > 0) {
    unsigned tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if constexpr (is_pow2(NC)) {
      fft_pow2_inplace<NC, COUNT, lds_span<NC, SW>(NC), 1024, SW>(buf, tw, tid);
    } else {
      static_assert(mixed_supported(NC), "a length of radices 12, 8, 4, 5, 3, 2");
      fft_mixed_inplace<NC, COUNT, lds_span<NC, SW>(NC), 1024, SW>(buf, tw, tid);
    }
  } else {
    fft_lds_inplace_tw<true, true>(buf, COUNT, stride, d, tw);
  }
}

__device__ inline void fft_lds_inplace(float2* buf, int count, int stride, const FftDesc& d,
                                       const float2* __restrict__ tw_all) {
  fft_lds_inplace_tw<false>(buf, count, stride, d, tw_all + d.tw_off);
}

// FFT forms, chosen per plan on the host and compiled as separate kernels so that
// each kernel carries only its own code (and register budget):
//   FFT_INPLACE  one LDS buffer, radices 4 and 8
//   FFT_PINGPONG two LDS buffers, radices 2, 3, 4, 5, 8
//   FFT_GENERIC  two LDS buffers, also odd primes up to 31
enum FftForm { FFT_INPLACE = 0, FFT_PINGPONG = 1, FFT_GENERIC = 2 };

template <int FORM>
__device__ __forceinline__ float2* run_fft(float2* buf, float2* tmp, int count, int stride, const FftDesc& d,
                                           const float2* __restrict__ tw_all) {
  if constexpr (FORM == FFT_INPLACE) {
    fft_lds_inplace(buf, count, stride, d, tw_all);
    return buf;
  } else {
    return fft_lds<FORM == FFT_GENERIC>(buf, tmp, count, stride, d, tw_all);
  }
}

}  // namespace fb
