// Host-side plan construction under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Built by tests/test_host_sanitizers.py with g++ -fsanitize=address,undefined from the
// library's plan.cpp and hostmath.cpp (host code only; no HIP call is made): builds the
// plans of several shapes and rejects the invalid ones, and checks the FP64 host numerics
// against values they must reproduce.  Any memory error or undefined behaviour aborts the
// run; a wrong value makes it exit non-zero.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <vector>

#include "hostmath.h"
#include "plan.h"

namespace fb {
// upload_plan references these kernel set-up calls; no device work is done here
hipError_t configure_kernels() { return hipSuccess; }
hipError_t configure_eig_kernels() { return hipSuccess; }
hipError_t configure_svd_kernels() { return hipSuccess; }
}  // namespace fb

static int failures = 0;
static void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++failures;
  }
}

int main() {
  struct Shape {
    int L;
    double c, R;
    int want;
  };
  const Shape shapes[] = {
      {8, 0.5, 4, FB_OK},      {16, 0.5, 8, FB_OK},      {31, 0.5, 15.5, FB_OK},   {24, 0.375, 12, FB_OK},
      {64, 0.3, 32, FB_OK},    {128, 0.5, 64, FB_OK},    {256, 0.5, 128, FB_OK},   {1024, 0.5, 32, FB_OK},
      {1, 0.5, 0.5, FB_ERR_INVALID_ARG}, {32, 0.6, 16, FB_ERR_INVALID_ARG}, {32, 0.5, 17, FB_ERR_INVALID_ARG},
      {4, 0.5, 0.5, FB_ERR_INVALID_ARG},
  };
  for (const Shape& s : shapes) {
    fb::Plan pl;
    const int rc = fb::build_host_plan(s.L, s.c, s.R, pl);
    std::printf("plan L=%d c=%g R=%g: rc %d", s.L, s.c, s.R, rc);
    if (rc == FB_OK) {
      std::printf(" n_xi %d n_theta %d k_max %d p_half %lld grid %d\n", pl.n_xi, pl.n_theta, pl.k_max,
                  (long long)pl.p_half, pl.N);
      check(pl.coef_off.back() == pl.p_half, "coefficient offsets end at p_half");
      check((int)pl.jmin.size() == pl.k_max + 1 && (int)pl.kring.size() == pl.n_xi, "ring tables sized");
      bool ok = true;
      for (int k = 0; k <= pl.k_max; ++k) ok = ok && pl.jmin[k] >= 0 && pl.jmin[k] < pl.n_xi;
      check(ok, "every block reads at least one ring");
      // the column pass's stored ranges: one centred interval per grid row, inside the row
      ok = pl.gcols.size() == 2 * (size_t)pl.M2;
      long long stored = 0;
      for (int r = 0; ok && r < pl.M2; ++r) {
        const int lo = pl.gcols[2 * r], hi = pl.gcols[2 * r + 1];
        if (lo <= hi) {
          ok = lo >= -pl.N / 2 && hi < pl.N - pl.N / 2;
          stored += hi - lo + 1;
        }
      }
      check(ok, "grid column ranges");
      // covariance items: every 32 x 32 tile of the upper triangle of every block once, from
      // two segments of that block; every k = 0 segment's S0 sums once
      {
        std::vector<std::vector<int>> cover(pl.k_max + 1);
        for (int k = 0; k <= pl.k_max; ++k) {
          const int nb = (pl.p[k] + fb::kCovSeg - 1) / fb::kCovSeg;
          cover[k].assign(nb * nb, 0);
        }
        std::vector<int> s0((pl.p[0] + fb::kCovSeg - 1) / fb::kCovSeg, 0);
        bool cov_ok = true;
        for (const fb::CovItem& it : pl.items_cov) {
          for (int s = 0; s < fb::kCovSegs; ++s) {
            if (it.k[s] < 0) continue;
            const int k = it.k[s];
            cov_ok = cov_ok && k <= pl.k_max && it.q0[s] % fb::kCovSeg == 0 && it.q0[s] < pl.p[k] &&
                     it.row[s] == pl.coef_off[k] + it.q0[s];
            if (k == 0 && it.sum0[s]) s0[it.q0[s] / fb::kCovSeg]++;
            cov_ok = cov_ok && (k == 0 || !it.sum0[s]);
          }
          for (int w = 0; w < fb::kCovWaves; ++w) {
            if (it.ta[w] == 255) continue;
            const int a = it.ta[w], b = it.tb[w];
            cov_ok = cov_ok && a < fb::kCovSegs && b < fb::kCovSegs && it.k[a] >= 0 && it.k[a] == it.k[b] &&
                     it.q0[a] <= it.q0[b];
            if (!cov_ok) break;
            const int k = it.k[a], nb = (pl.p[k] + fb::kCovSeg - 1) / fb::kCovSeg;
            cover[k][(it.q0[a] / fb::kCovSeg) * nb + it.q0[b] / fb::kCovSeg]++;
          }
        }
        for (int k = 0; cov_ok && k <= pl.k_max; ++k) {
          const int nb = (pl.p[k] + fb::kCovSeg - 1) / fb::kCovSeg;
          for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) cov_ok = cov_ok && cover[k][i * nb + j] == (i <= j ? 1 : 0);
        }
        for (int v : s0) cov_ok = cov_ok && v == 1;
        check(cov_ok, "covariance items cover every tile once");
        std::printf("  covariance: %zu items\n", pl.items_cov.size());
      }
      // spread chunks: the kernel's unconditional staging loads rely on every chunk holding
      // 1..kSpreadNodes nodes and at least one batch of entries, at most kSpreadEntries, each
      // pointing at one of its chunk's nodes
      {
        bool sp_ok = !pl.stiles.empty();
        long long nsent = 0;
        for (const fb::SpreadTile& t : pl.stiles) {
          sp_ok = sp_ok && t.c0 <= t.c1 && t.c1 <= (int)pl.schunks.size() && t.nsub >= 1 && t.nsub <= fb::kSpreadSlice;
          sp_ok = sp_ok && (t.c1 - t.c0 <= 1 || t.nsub * fb::kSpreadHeavyGroups >= fb::kSpreadSlice);
        }
        for (size_t c = 0; sp_ok && c < pl.schunks.size(); ++c) {
          const fb::SpreadChunk& ch = pl.schunks[c];
          const int nl = ch.n1 - ch.n0;
          sp_ok = nl >= 1 && nl <= fb::kSpreadNodes && ch.n1 <= (int)pl.snodes.size() &&
                  ch.seg + fb::kSpreadPairs < (int)pl.sseg.size();
          if (!sp_ok) break;
          const int e0 = pl.sseg[ch.seg], e1 = pl.sseg[ch.seg + fb::kSpreadPairs];
          sp_ok = e1 > e0 && e1 - e0 <= fb::kSpreadEntries && e1 <= (int)pl.sent.size();
          for (int p = 0; sp_ok && p < fb::kSpreadPairs; ++p)
            sp_ok = pl.sseg[ch.seg + p] <= pl.sseg[ch.seg + p + 1] && pl.sseg[ch.seg + p] % fb::kSpreadBatch == 0;
          for (int e = e0; sp_ok && e < e1; ++e)
            sp_ok = pl.sent[e].off % (fb::kImgGroup * 8u) == 0 && pl.sent[e].off / (fb::kImgGroup * 8u) < (unsigned)nl;
          nsent += e1 - e0;
        }
        check(sp_ok, "spread chunks within their limits");
        // slot tables: each pair of each cell has exactly one leading slot over the cell's
        // tiles; a pair's slots are an aligned run of 1, 2, 4 or 8 inside one wavefront of 8
        bool sl_ok = pl.sslot.size() == pl.stiles.size() * (size_t)fb::kSpreadPairs;
        std::map<std::pair<int, int>, std::vector<int>> leads;
        for (size_t ti = 0; sl_ok && ti < pl.stiles.size(); ++ti) {
          const fb::SpreadTile& t = pl.stiles[ti];
          auto& cov = leads[{t.m2, t.m1}];
          cov.resize(fb::kSpreadPairs, 0);
          sl_ok = t.slots == (int)ti * fb::kSpreadPairs && t.maxs >= 1 && t.maxs <= 8;
          for (int sl = 0; sl_ok && sl < fb::kSpreadPairs; ++sl) {
            const unsigned v = pl.sslot[t.slots + sl];
            if (v & fb::kSpreadIdleSlot) continue;
            const int pr = v & 63, sp = 1 << ((v >> 8) & 3), lead = sl & ~(sp - 1);
            sl_ok = sp <= t.maxs && lead / 8 == (lead + sp - 1) / 8;
            for (int j = lead; sl_ok && j < lead + sp; ++j) sl_ok = pl.sslot[t.slots + j] == v;
            if (sl == lead) cov[pr]++;
          }
        }
        for (auto& kv : leads)
          for (int v : kv.second) sl_ok = sl_ok && v == 1;
        check(sl_ok, "spread slot tables cover every pair once");
        // balance: a step lasts as long as its fullest slot, so the mean slot load over the
        // fullest one, summed over chunks, is the share of lane time that does work
        double mean_sum = 0.0, max_sum = 0.0;
        for (const fb::SpreadChunk& ch : pl.schunks) {
          int mx = 0, tot = 0;
          for (int sl = 0; sl < fb::kSpreadPairs; ++sl) {
            const int c = pl.sseg[ch.seg + sl + 1] - pl.sseg[ch.seg + sl];
            mx = std::max(mx, c);
            tot += c;
          }
          mean_sum += (double)tot / fb::kSpreadPairs;
          max_sum += mx;
        }
        const double balance = max_sum > 0 ? mean_sum / max_sum : 1.0;
        std::printf("  spread slot balance %.3f\n", balance);
        if (s.L >= 128 && s.R == s.L / 2.0) check(balance >= 0.7, "spread slots balanced");
        std::printf("  spread: %zu cells, %zu chunks, %lld entries\n", pl.stiles.size(), pl.schunks.size(), nsent);
      }
      std::printf("  grid points stored by the column pass: %.3f of %d x %d\n", (double)stored / ((double)pl.M2 * pl.N),
                  pl.M2, pl.N);
    } else {
      std::printf("\n");
    }
    check(rc == s.want, "plan return code");
  }

  // I_0 at tabulated points (Abramowitz and Stegun, Table 9.8)
  check(std::fabs(fb::bessel_i0(1.0) - 1.266065877752008) < 1e-14, "I_0(1)");
  check(std::fabs(fb::bessel_i0(10.0) / 2815.716628466254 - 1.0) < 1e-13, "I_0(10)");
  // the closed-form kernel transform against a Gauss-Legendre quadrature of the kernel
  std::vector<double> x, w;
  fb::gauss_legendre(200, x, w);
  double wsum = 0.0;
  for (double v : w) wsum += v;
  check(std::fabs(wsum - 2.0) < 1e-13, "Gauss-Legendre weights sum to 2");
  const double beta = 16.25, pi = 3.14159265358979323846;
  for (double t : {0.0, 0.1, 0.25, 0.5, 1.0}) {
    double q = 0.0;
    for (size_t i = 0; i < x.size(); ++i) q += w[i] * fb::kb_kernel(x[i], beta) * std::cos(pi * 7 * x[i] * t);
    q *= 3.5;
    const double f = fb::kb_kernel_ft(t, 7, beta);
    check(std::fabs(q - f) <= 1e-9 * std::fabs(fb::kb_kernel_ft(0.0, 7, beta)), "kernel transform");
  }
  // the zeros of J_0 below 8 (2.4048, 5.5201; the next is 8.6537) and the first of J_1
  const auto z = fb::bessel_zeros_upto(8.0);
  check(z.size() >= 2 && z[0].size() == 2 && std::fabs(z[0][0] - 2.404825557695773) < 1e-12, "zeros of J_0");
  check(z.size() >= 2 && std::fabs(z[1][0] - 3.831705970207512) < 1e-12, "first zero of J_1");
  std::printf("%d failure(s)\n", failures);
  return failures ? 1 : 0;
}
