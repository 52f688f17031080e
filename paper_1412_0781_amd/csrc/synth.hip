// Seeded synthetic inputs on the device (not part of the method): Philox-4x32-10
// (Salmon, Moraes, Dror, Shaw, SC'11) with counter (block, index_lo, index_hi,
// stream) and key (seed_lo, seed_hi); Box-Muller normals on consecutive word
// pairs: u1 = (w0 + 1) 2^-32, u2 = w1 2^-32, z = sqrt(-2 ln u1) (cos, sin)(2 pi u2).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fb {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k.x += W0;
      k.y += W1;
    }
    unsigned hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    unsigned hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__global__ void k_synth_words(unsigned long long seed, unsigned stream, long long first, long long n,
                              long long n_per, unsigned* __restrict__ out) {
  const long long nblk = (n_per + 3) / 4;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nblk) return;
  long long i = t / nblk, b = t - i * nblk;
  unsigned long long idx = (unsigned long long)(first + i);
  uint4 w = philox4x32_10(make_uint4((unsigned)b, (unsigned)idx, (unsigned)(idx >> 32), stream),
                          make_uint2((unsigned)seed, (unsigned)(seed >> 32)));
  unsigned ww[4] = {w.x, w.y, w.z, w.w};
  for (int e = 0; e < 4; ++e) {
    long long col = 4 * b + e;
    if (col < n_per) out[i * n_per + col] = ww[e];
  }
}

__global__ void k_synth_normals(unsigned long long seed, unsigned stream, long long first, long long n,
                                long long n_per, float scale, float* __restrict__ out) {
  const long long npair = (n_per + 1) / 2;
  const long long nblk = (2 * npair + 3) / 4;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nblk) return;
  long long i = t / nblk, b = t - i * nblk;
  unsigned long long idx = (unsigned long long)(first + i);
  uint4 w = philox4x32_10(make_uint4((unsigned)b, (unsigned)idx, (unsigned)(idx >> 32), stream),
                          make_uint2((unsigned)seed, (unsigned)(seed >> 32)));
  unsigned ww[4] = {w.x, w.y, w.z, w.w};
  const double two32 = 2.3283064365386962890625e-10;  // 2^-32
  for (int pr = 0; pr < 2; ++pr) {
    double u1 = ((double)ww[2 * pr] + 1.0) * two32;
    double u2 = (double)ww[2 * pr + 1] * two32;
    double rad = sqrt(-2.0 * log(u1));
    double sv, cv;
    sincospi(2.0 * u2, &sv, &cv);
    long long col = 4 * b + 2 * pr;
    if (col < n_per) out[i * n_per + col] = (float)(scale * rad * cv);
    if (col + 1 < n_per) out[i * n_per + col + 1] = (float)(scale * rad * sv);
  }
}

hipError_t launch_synth_words(unsigned long long seed, unsigned rng_stream, long long first, long long n,
                              long long n_per, unsigned* out, hipStream_t st) {
  long long total = n * ((n_per + 3) / 4);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_synth_words, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, seed, rng_stream,
                     first, n, n_per, out);
  return hipGetLastError();
}

hipError_t launch_synth_normals(unsigned long long seed, unsigned rng_stream, long long first, long long n,
                                long long n_per, float scale, float* out, hipStream_t st) {
  long long total = n * ((2 * ((n_per + 1) / 2) + 3) / 4);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_synth_normals, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, seed, rng_stream,
                     first, n, n_per, scale, out);
  return hipGetLastError();
}

}  // namespace fb
