// One-sided (Hestenes) Jacobi orthogonalisation of the columns of a p x p FP64 matrix held
// in LDS, shared by the SVD route and the eigendecomposition.
#pragma once
#include <hip/hip_runtime.h>

namespace fb {

constexpr int kJacobiMaxSweeps = 60;
constexpr double kJacobiTol = 1e-15;  // rotate while |x.y| > tol ||x|| ||y||
constexpr int kJacobiMaxPerLane = 3;  // accumulated rotations: p <= 192 (three entries per lane)

// M: column-major p x p (column l at M + l p) in LDS; the whole workgroup calls it and
// waves take disjoint column pairs.  Cyclic sweeps in round-robin order (circle method: the
// P/2 disjoint pairs of a round, P = p rounded up to even, one pair per wave at a time)
// rotate each pair (x, y) with t = sign(z) / (|z| + sqrt(1 + z^2)), z = (|y|^2 - |x|^2) /
// (2 x.y), x' = c x - s y, y' = s x + c y, until a sweep rotates nothing.  The columns
// then are mutually orthogonal: M_out = M_in V with V orthogonal.  s_rot: an int in LDS.
// kAccum: the same rotations are applied to the columns of V (column-major p x p, any
// address space, holding the identity on entry), which then holds that orthogonal V.
template <bool kAccum = false>
__device__ inline void one_sided_jacobi(double* M, int pk, int* s_rot, double* V = nullptr) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = (int)(blockDim.x >> 6);
  const int P = pk + (pk & 1);
  for (int sweep = 0; sweep < kJacobiMaxSweeps && P > 1; ++sweep) {
    if (tid == 0) *s_rot = 0;
    __syncthreads();
    for (int rd = 0; rd < P - 1; ++rd) {
      for (int s = wave; s < P / 2; s += nw) {
        const int i = s == 0 ? 0 : (s - 1 + rd) % (P - 1) + 1;
        const int j = (P - 2 - s + rd) % (P - 1) + 1;
        if (i >= pk || j >= pk) continue;
        double* ci = M + (long long)i * pk;
        double* cj = M + (long long)j * pk;
        double vx[kJacobiMaxPerLane], vy[kJacobiMaxPerLane];
        if constexpr (kAccum) {  // issued before the dot products so that their latency overlaps
#pragma unroll
          for (int u = 0; u < kJacobiMaxPerLane; ++u) {
            const int e = lane + 64 * u;
            vx[u] = e < pk ? V[(long long)i * pk + e] : 0.0;
            vy[u] = e < pk ? V[(long long)j * pk + e] : 0.0;
          }
        }
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int e = lane; e < pk; e += 64) {
          const double x = ci[e], y = cj[e];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        for (int m = 32; m > 0; m >>= 1) {
          al += __shfl_xor(al, m);
          be += __shfl_xor(be, m);
          ga += __shfl_xor(ga, m);
        }
        if (ga != 0.0 && fabs(ga) > kJacobiTol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          for (int e = lane; e < pk; e += 64) {
            const double x = ci[e], y = cj[e];
            ci[e] = cs * x - sn * y;
            cj[e] = sn * x + cs * y;
          }
          if constexpr (kAccum) {
#pragma unroll
            for (int u = 0; u < kJacobiMaxPerLane; ++u) {
              const int e = lane + 64 * u;
              if (e < pk) {
                V[(long long)i * pk + e] = cs * vx[u] - sn * vy[u];
                V[(long long)j * pk + e] = sn * vx[u] + cs * vy[u];
              }
            }
          }
          if (lane == 0) *s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = *s_rot;
    __syncthreads();
    if (!rot) break;
  }
}

}  // namespace fb
