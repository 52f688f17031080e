#include "hostmath.h"

#include <algorithm>
#include <cmath>

namespace fb {

void bessel_j_all(double x, int nmax, double* out) {
  if (nmax < 0) return;
  if (x == 0.0) {
    out[0] = 1.0;
    for (int k = 1; k <= nmax; ++k) out[k] = 0.0;
    return;
  }
  // Start order: comfortably beyond both nmax and x so that the ratio
  // J_{m+1}/J_m at the start is negligible (A&S 9.12 start-index rule).
  double top = std::max((double)nmax, x);
  int m = 2 * ((int)(top + 20.0 + std::sqrt(60.0 * top)) / 2) + 2;
  double jp1 = 0.0, j = 1e-300, sum = 0.0;
  const double big = 1e250, small = 1e-250;
  for (int k = m; k >= 1; --k) {
    // J_{k-1} = (2k/x) J_k - J_{k+1}
    double jm1 = (2.0 * k / x) * j - jp1;
    jp1 = j;
    j = jm1;
    if (k - 1 <= nmax) out[k - 1] = j;
    if (((k - 1) % 2) == 0 && k - 1 > 0) sum += 2.0 * j;
    if (std::fabs(j) > big) {  // rescale everything carried so far
      j *= small;
      jp1 *= small;
      sum *= small;
      for (int t = k - 1; t <= nmax; ++t) out[t] *= small;
    }
  }
  sum += j;  // J_0 term
  double inv = 1.0 / sum;
  for (int k = 0; k <= nmax; ++k) out[k] *= inv;
}

double bessel_j(int k, double x) {
  std::vector<double> buf(k + 2);
  bessel_j_all(x, k + 1, buf.data());
  return buf[k];
}

static void jk_and_deriv(int k, double x, double& f, double& df) {
  std::vector<double> buf(k + 3);
  bessel_j_all(x, k + 1, buf.data());
  f = buf[k];
  if (k == 0)
    df = -buf[1];
  else
    df = 0.5 * (buf[k - 1] - buf[k + 1]);
}

std::vector<std::vector<double>> bessel_zeros_upto(double bound) {
  std::vector<std::vector<double>> zeros;
  if (!(bound > 0)) return zeros;
  // No zero of J_k lies below k, so only k < bound can have one.
  int kmax = (int)std::floor(bound) + 1;
  const double h = 0.25;
  std::vector<double> xs;
  for (int i = 1; i * h < bound; ++i) xs.push_back(i * h);  // start away from x = 0
  xs.push_back(bound);
  int np = (int)xs.size();
  std::vector<double> tab((size_t)np * (kmax + 1));
  for (int i = 0; i < np; ++i) bessel_j_all(xs[i], kmax, &tab[(size_t)i * (kmax + 1)]);
  for (int k = 0; k <= kmax; ++k) {
    std::vector<double> zk;
    for (int i = 0; i + 1 < np; ++i) {
      double fa = tab[(size_t)i * (kmax + 1) + k], fb = tab[(size_t)(i + 1) * (kmax + 1) + k];
      if (fa == 0.0) {  // exactly on a grid point (measure zero in practice)
        if (xs[i] > k) zk.push_back(xs[i]);
        continue;
      }
      if ((fa < 0) == (fb < 0) || fb == 0.0) continue;
      double a = xs[i], b = xs[i + 1], x = 0.5 * (a + b);
      // safeguarded Newton
      for (int it = 0; it < 100; ++it) {
        double f, df;
        jk_and_deriv(k, x, f, df);
        if ((f < 0) == (fa < 0)) a = x; else b = x;
        double xn = x - f / df;
        if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
        double dx = std::fabs(xn - x);
        x = xn;
        if (dx <= 1e-15 * x) break;
      }
      zk.push_back(x);
    }
    // a root exactly at the last scan point (bound itself)
    double flast = tab[(size_t)(np - 1) * (kmax + 1) + k];
    if (flast == 0.0) zk.push_back(xs[np - 1]);
    if (zk.empty()) break;
    zeros.push_back(zk);
  }
  return zeros;
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    // P_n(z) and P_n'(z) = n (z P_n - P_{n-1}) / (z^2 - 1) from the recurrence
    auto legendre = [n](double zz, double& pn, double& dpn) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * zz * p2 - (j - 1.0) * p3) / j;
      }
      pn = p1;
      dpn = n * (zz * p1 - p2) / (zz * zz - 1.0);
    };
    for (int it = 0; it < 100; ++it) {
      double pn;
      legendre(z, pn, pp);
      double z1 = z;
      z = z1 - pn / pp;
      if (std::fabs(z - z1) <= 4e-16) break;
    }
    {
      double pn;
      legendre(z, pn, pp);
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

double bessel_i0(double x) {
  // sum_{m >= 0} ((x/2)^m / m!)^2: every term positive, so the sum loses nothing to cancellation
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int m = 1; m < 1000; ++m) {
    term *= q / ((double)m * (double)m);
    sum += term;
    if (term <= 1e-17 * sum) break;
  }
  return sum;
}

double kb_kernel(double z, double beta) {
  if (std::fabs(z) > 1.0) return 0.0;
  return bessel_i0(beta * std::sqrt(1.0 - z * z)) / bessel_i0(beta);
}

double kb_kernel_ft(double t, int w, double beta) {
  // int_{-1}^{1} I_0(beta sqrt(1 - z^2)) cos(a z) dz = 2 sinh(s) / s, s = sqrt(beta^2 - a^2)
  // (2 sin(s) / s with s = sqrt(a^2 - beta^2) once a > beta), here a = pi w t
  const double pi = 3.14159265358979323846;
  const double a = pi * w * t;
  const double d = beta * beta - a * a;
  double f;
  if (std::fabs(d) < 1e-12)
    f = 2.0;
  else if (d > 0.0)
    f = 2.0 * std::sinh(std::sqrt(d)) / std::sqrt(d);
  else
    f = 2.0 * std::sin(std::sqrt(-d)) / std::sqrt(-d);
  return 0.5 * w * f / bessel_i0(beta);
}

int next_smooth_235(int m) {
  for (int n = std::max(m, 1);; ++n) {
    int r = n;
    for (int p : {2, 3, 5})
      while (r % p == 0) r /= p;
    if (r == 1) return n;
  }
}

bool fft_radices(int n, std::vector<int>& radices) {
  radices.clear();
  int r = n;
  while (r % 8 == 0 && r != 16) { radices.push_back(8); r /= 8; }  // 16 = 4 * 4 rather than 8 * 2
  while (r % 4 == 0) { radices.push_back(4); r /= 4; }
  while (r % 2 == 0) { radices.push_back(2); r /= 2; }
  for (int p = 3; p <= 31; p += 2) {
    while (r % p == 0) { radices.push_back(p); r /= p; }
  }
  return r == 1;
}

}  // namespace fb
