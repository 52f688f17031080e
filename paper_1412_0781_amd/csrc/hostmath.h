// FP64 host numerics used to build a plan: Bessel functions of integer order,
// their positive zeros, Gauss-Legendre rules and the spreading kernel with its
// Fourier transform.  Pure C++ (no HIP), so it runs and is tested on any host.
#pragma once
#include <cstdint>
#include <vector>

namespace fb {

// J_0(x) .. J_nmax(x) for x >= 0 by Miller's backward recurrence, normalised
// with J_0 + 2 sum_{m>=1} J_{2m} = 1 (Abramowitz & Stegun 9.1.46, 9.12).
void bessel_j_all(double x, int nmax, double* out);

// J_k(x) alone (same recurrence).
double bessel_j(int k, double x);

// Positive zeros of J_k that are <= bound, ascending, for every k = 0..kmax
// where at least one exists.  Bracketed on a uniform scan (zeros of J_k are
// more than pi apart), refined by safeguarded Newton steps with
// J_k' = (J_{k-1} - J_{k+1}) / 2.
std::vector<std::vector<double>> bessel_zeros_upto(double bound);

// n-point Gauss-Legendre nodes (ascending) and weights on [-1, 1], by Newton's
// method on the three-term Legendre recurrence.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Modified Bessel function I_0(x), x >= 0, by its power series.
double bessel_i0(double x);

// Spreading kernel: the Kaiser-Bessel window phi(z) = I_0(beta sqrt(1 - z^2)) / I_0(beta) on
// |z| <= 1, 0 outside (Jackson, Meyer, Nishimura, Macovski, IEEE Trans. Med. Imaging 10 (1991);
// shape beta of Beatty, Nishimura, Pauly, IEEE Trans. Med. Imaging 24 (2005)).  In grid units u
// the kernel is phi(2u / w).
double kb_kernel(double z, double beta);

// Its Fourier transform in grid units, in closed form:
//   phi_hat(t) = int_{-w/2}^{w/2} phi(2u/w) exp(-2 pi i u t) du
//              = (w/2) int_{-1}^{1} phi(z) cos(pi w z t) dz
//              = w sinh(sqrt(beta^2 - (pi w t)^2)) / (sqrt(beta^2 - (pi w t)^2) I_0(beta)).
double kb_kernel_ft(double t, int w, double beta);

// Smallest n >= m that factors into 2, 3 and 5 only.
int next_smooth_235(int m);

// Factor n into FFT radices (8 first, then 4, 2, 3, 5, 7 and primes <= 31).
// Returns false if a prime factor above 31 remains.
bool fft_radices(int n, std::vector<int>& radices);

}  // namespace fb
