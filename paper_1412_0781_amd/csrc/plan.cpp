// Plan construction (Algorithm 1, steps 1-2) in FP64 on the host, and its upload.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "hostmath.h"
#include "kernels.h"

namespace fb {

static const double kPi = 3.14159265358979323846;

static void add_fft(FftDesc& d, int n, std::vector<float>& tw) {
  d.n = n;
  std::vector<int> rad;
  fft_radices(n, rad);
  d.nstage = (int)rad.size();
  int ns = 1;
  for (int i = 0; i < d.nstage; ++i) {
    d.radix[i] = rad[i];
    d.dnb[i] = make_fastdiv(n / rad[i]);
    d.dns[i] = make_fastdiv(ns);
    ns *= rad[i];
  }
  d.tw_off = (int)(tw.size() / 2);
  for (int t = 0; t < n; ++t) {
    double a = -2.0 * kPi * (double)t / (double)n;
    tw.push_back((float)std::cos(a));
    tw.push_back((float)std::sin(a));
  }
}

int build_host_plan(int L, double c, double R, Plan& pl) {
  if (L < 2) return FB_ERR_INVALID_ARG;
  if (L > 2048) return FB_ERR_UNSUPPORTED;  // FFT rows of the 2L grid must fit the 64 KiB LDS budget
  if (!(c > 0.0 && c <= 0.5)) return FB_ERR_INVALID_ARG;
  if (!(R > 0.0 && R <= L / 2.0)) return FB_ERR_INVALID_ARG;
  pl.L = L;
  pl.c = c;
  pl.R = R;
  pl.n_xi = (int)std::ceil(4 * c * R);
  pl.n_theta = (int)std::ceil(16 * c * R);
  const double bound = 2 * kPi * c * R;

  // (k, q) selection, Eq.(criterion1): q admissible iff R_{k,q+1} <= 2 pi c R
  std::vector<std::vector<double>> z = bessel_zeros_upto(bound);
  pl.p.clear();
  for (size_t k = 0; k < z.size(); ++k) {
    int pk = (int)z[k].size() - 1;
    if (pk < 1) break;
    pl.p.push_back(pk);
  }
  if (pl.p.empty()) return FB_ERR_INVALID_ARG;
  pl.k_max = (int)pl.p.size() - 1;
  pl.p0 = pl.p[0];
  if (pl.p0 > 256) return FB_ERR_UNSUPPORTED;  // the device eigensolver handles blocks up to 256
  if (pl.n_theta % 2 != 0) return FB_ERR_UNSUPPORTED;  // half-ring symmetry needs even n_theta
  if (pl.k_max >= pl.n_theta / 2) return FB_ERR_UNSUPPORTED;

  pl.coef_off.assign(pl.k_max + 2, 0);
  pl.cov_off.assign(pl.k_max + 2, 0);
  for (int k = 0; k <= pl.k_max; ++k) {
    pl.coef_off[k + 1] = pl.coef_off[k] + pl.p[k];
    pl.cov_off[k + 1] = pl.cov_off[k] + (int64_t)pl.p[k] * pl.p[k];
  }
  pl.p_half = pl.coef_off[pl.k_max + 1];
  pl.cov_size = pl.cov_off[pl.k_max + 1];
  pl.tri_off.assign(pl.k_max + 2, 0);  // packed upper triangles p_k (p_k + 1) / 2, by k
  for (int k = 0; k <= pl.k_max; ++k) pl.tri_off[k + 1] = pl.tri_off[k] + (long long)pl.p[k] * (pl.p[k] + 1) / 2;
  pl.p_total = pl.p0 + 2 * (pl.p_half - pl.p0);
  pl.kq_k.resize(pl.p_half);
  pl.kq_q.resize(pl.p_half);
  pl.roots.resize(pl.p_half);
  pl.norms.resize(pl.p_half);
  for (int k = 0; k <= pl.k_max; ++k)
    for (int q = 0; q < pl.p[k]; ++q) {
      int64_t i = pl.coef_off[k] + q;
      pl.kq_k[i] = k;
      pl.kq_q[i] = q + 1;
      pl.roots[i] = z[k][q];
      // N_{k,q} = 1 / (c sqrt(pi) |J_{k+1}(R_{k,q})|)   (Eq.(FB))
      pl.norms[i] = 1.0 / (c * std::sqrt(kPi) * std::fabs(bessel_j(k + 1, z[k][q])));
    }

  // Gauss-Legendre nodes and weights on [0, c] (Eq.(a))
  std::vector<double> gx, gw;
  gauss_legendre(pl.n_xi, gx, gw);
  pl.xi.resize(pl.n_xi);
  pl.wq.resize(pl.n_xi);
  for (int j = 0; j < pl.n_xi; ++j) {
    pl.xi[j] = c * (gx[j] + 1.0) / 2.0;
    pl.wq[j] = (c / 2.0) * gw[j];
  }

  // radial table B_{(k,q), j} = N_{k,q} J_k(R_{k,q} xi_j / c) xi_j w_j  (Eq.(a)); rows split over threads
  pl.radial.assign((size_t)pl.p_half * pl.n_xi, 0.0);
  {
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t)
      th.emplace_back([&, t]() {
        std::vector<double> buf(pl.k_max + 2);
        for (int64_t i = t; i < pl.p_half; i += nth) {
          int k = pl.kq_k[i];
          for (int j = 0; j < pl.n_xi; ++j) {
            bessel_j_all(pl.roots[i] * pl.xi[j] / c, k, buf.data());
            pl.radial[(size_t)i * pl.n_xi + j] = pl.norms[i] * buf[k] * pl.xi[j] * pl.wq[j];
          }
        }
      });
    for (auto& x : th) x.join();
  }

  // rings each block's radial sum needs (the rest of each row is below kRadialNegligible of
  // the row's largest entry), and per ring the largest k that reads it
  pl.jmin.assign(pl.k_max + 1, pl.n_xi);
  for (int k = 0; k <= pl.k_max; ++k)
    for (int q = 0; q < pl.p[k]; ++q) {
      const double* r = &pl.radial[(size_t)(pl.coef_off[k] + q) * pl.n_xi];
      double m = 0.0;
      for (int j = 0; j < pl.n_xi; ++j) m = std::max(m, std::fabs(r[j]));
      int j = 0;
      while (j < pl.n_xi && !(std::fabs(r[j]) >= kRadialNegligible * m)) ++j;
      pl.jmin[k] = std::min(pl.jmin[k], j);
    }
  pl.kring.assign(pl.n_xi, -1);
  for (int k = 0; k <= pl.k_max; ++k)
    for (int j = pl.jmin[k]; j < pl.n_xi; ++j) pl.kring[j] = std::max(pl.kring[j], k);

  // Non-uniform FFT: oversampled grid N >= 2L (2,3,5-smooth), Kaiser-Bessel kernel of width 7
  // with the shape beta = pi sqrt((w / sigma)^2 (sigma - 1/2)^2 - 0.8) for oversampling sigma = N / L.
  pl.N = next_smooth_235(2 * L);
  if (pl.N % 2) pl.N = next_smooth_235(pl.N + 1);
  pl.w = 7;
  double sigma = (double)pl.N / L;
  pl.beta = kPi * std::sqrt((pl.w / sigma) * (pl.w / sigma) * (sigma - 0.5) * (sigma - 0.5) - 0.8);
  pl.hw = pl.w / 2 + 1;
  pl.M2 = pl.N / 2 + 2 * pl.hw + 1;
  pl.H = pl.n_theta / 2;

  int x0 = -(int)std::ceil((L - 1) / 2.0);
  pl.deconv.resize(L);
  for (int a = 0; a < L; ++a) pl.deconv[a] = 1.0 / kb_kernel_ft((double)(x0 + a) / pl.N, pl.w, pl.beta);

  // polar half-ring nodes theta_l = 2 pi l / n_theta, l < n_theta / 2
  if (pl.n_xi > 65535 || pl.H > 65535) return FB_ERR_UNSUPPORTED;  // node records hold 16-bit j, l
  pl.nodes.resize((size_t)pl.n_xi * pl.H);
  for (int j = 0; j < pl.n_xi; ++j)
    for (int l = 0; l < pl.H; ++l) {
      double th = 2.0 * kPi * l / pl.n_theta;
      double t1 = pl.N * pl.xi[j] * std::cos(th);
      double t2 = pl.N * pl.xi[j] * std::sin(th);
      double b1 = std::ceil(t1 - pl.w / 2.0), b2 = std::ceil(t2 - pl.w / 2.0);
      NodeTap nt;
      int ib1 = (int)b1, ib2 = (int)b2;
      nt.b1 = ((ib1 % pl.N) + pl.N) % pl.N;
      nt.b2 = ib2 + pl.hw;
      nt.f1 = (float)(t1 - b1);
      nt.f2 = (float)(t2 - b2);
      if (nt.b2 < 0 || nt.b2 + pl.w > pl.M2) return FB_ERR_UNSUPPORTED;  // cannot happen for c <= 1/2
      pl.nodes[(size_t)j * pl.H + l] = nt;
    }

  // LDS-tiled gather: nodes grouped by the cell of their tap origin (b1, b2); cells in
  // row-major order so that consecutive work items are neighbouring cells.  Weights in FP64.
  {
    if (pl.w != kGatherW) return FB_ERR_UNSUPPORTED;
    const int CS = kGatherCell;
    const int ncx = (pl.N + CS - 1) / CS, ncy = (pl.M2 + CS - 1) / CS;
    std::vector<std::vector<int>> cell(ncx * ncy);
    for (size_t n = 0; n < pl.nodes.size(); ++n) {
      const NodeTap& t = pl.nodes[n];
      cell[(t.b2 / CS) * ncx + t.b1 / CS].push_back((int)n);
    }
    pl.gnodes.clear();
    pl.gitems.clear();
    const int BW = CS + pl.w - 1;
    for (int cy = 0; cy < ncy; ++cy)
      for (int cx = 0; cx < ncx; ++cx) {
        // Interleave nodes whose tap origin is on even and odd box columns: neighbouring
        // nodes are read by neighbouring lanes, and 128-byte rows of opposite parity fall
        // in opposite halves of the LDS banks.
        std::vector<int> lst;
        {
          std::vector<int> ev, od;
          for (int n : cell[cy * ncx + cx]) (((pl.nodes[n].b1 - cx * CS) & 1) ? od : ev).push_back(n);
          for (size_t i = 0; i < std::max(ev.size(), od.size()); ++i) {
            if (i < ev.size()) lst.push_back(ev[i]);
            if (i < od.size()) lst.push_back(od[i]);
          }
        }
        for (size_t a0 = 0; a0 < lst.size(); a0 += kGatherChunk) {
          GatherItem it{cx * CS, cy * CS, (int)pl.gnodes.size(), 0};
          for (size_t a = a0; a < std::min(lst.size(), a0 + kGatherChunk); ++a) {
            int n = lst[a];
            int j = n / pl.H, l = n % pl.H;
            double th = 2.0 * kPi * l / pl.n_theta;
            double t1 = pl.N * pl.xi[j] * std::cos(th), t2 = pl.N * pl.xi[j] * std::sin(th);
            double b1 = std::ceil(t1 - pl.w / 2.0), b2 = std::ceil(t2 - pl.w / 2.0);
            const NodeTap& t = pl.nodes[n];
            GatherNode g;
            g.j = (unsigned short)j;
            g.l = (unsigned short)l;
            g.off = (t.b2 - cy * CS) * BW + (t.b1 - cx * CS);
            for (int a2 = 0; a2 < pl.w; ++a2) {
              g.w1[a2] = (float)kb_kernel(2.0 * (t1 - (b1 + a2)) / pl.w, pl.beta);
              g.w2[a2] = (float)kb_kernel(2.0 * (t2 - (b2 + a2)) / pl.w, pl.beta);
            }
            pl.gnodes.push_back(g);
          }
          it.s1 = (int)pl.gnodes.size();
          pl.gitems.push_back(it);
        }
      }
    // the centred hull of the box columns read in each row (a box of a cell near m1 = N/2
    // wraps, and its row's hull is then the whole row)
    pl.gcols.assign(2 * (size_t)pl.M2, 0);
    for (int r = 0; r < pl.M2; ++r) {
      pl.gcols[2 * r] = pl.N;
      pl.gcols[2 * r + 1] = -pl.N - 1;
    }
    for (const GatherItem& it : pl.gitems)
      for (int r = it.c2; r < std::min(it.c2 + BW, pl.M2); ++r)
        for (int cc = 0; cc < BW; ++cc) {
          const int col = (it.c1 + cc) % pl.N, ic = col < pl.N / 2 ? col : col - pl.N;
          pl.gcols[2 * r] = std::min(pl.gcols[2 * r], ic);
          pl.gcols[2 * r + 1] = std::max(pl.gcols[2 * r + 1], ic);
        }
  }

  // FFTs: grid side N and the angular half length H
  pl.tw.clear();
  std::vector<int> rad;
  if (!fft_radices(pl.N, rad) || !fft_radices(pl.H, rad)) return FB_ERR_UNSUPPORTED;
  if ((int)rad.size() > kMaxRadices) return FB_ERR_UNSUPPORTED;
  add_fft(pl.fft_grid, pl.N, pl.tw);
  add_fft(pl.fft_ang, pl.H, pl.tw);
  pl.angtw.resize(2 * (pl.H + 1));
  for (int k = 0; k <= pl.H; ++k) {
    double a = -2.0 * kPi * k / pl.n_theta;
    pl.angtw[2 * k] = (float)std::cos(a);
    pl.angtw[2 * k + 1] = (float)std::sin(a);
  }

  // Adjoint spreading as a gather over the folded half plane m2 = 0..N/2.
  // A node with value Q and tap weight om at (m1, m2), m2 in [-hw, N/2 + hw], adds
  //   om/2 * Q       to (m1, m2)              when 0 <= m2 <= N/2
  //   om/2 * conj(Q) to (-m1, -m2) mod N      when m2 <= 0 or m2 >= N/2
  // so that the half plane holds X(m) = (G(m) + conj G(-m)) / 2 of the full spread G.
  {
    const int N = pl.N, Nh = N / 2 + 1;
    const size_t nrows = (size_t)N * Nh;
    std::vector<int> cnt(nrows + 1, 0);
    auto for_each_tap = [&](auto&& fn) {
      for (size_t n = 0; n < pl.nodes.size(); ++n) {
        int j = (int)(n / pl.H), l = (int)(n % pl.H);
        double th = 2.0 * kPi * l / pl.n_theta;
        double t1 = pl.N * pl.xi[j] * std::cos(th);
        double t2 = pl.N * pl.xi[j] * std::sin(th);
        int b1 = (int)std::ceil(t1 - pl.w / 2.0), b2 = (int)std::ceil(t2 - pl.w / 2.0);
        for (int bb = 0; bb < pl.w; ++bb) {
          int m2 = b2 + bb;
          double w2 = kb_kernel(2.0 * (t2 - m2) / pl.w, pl.beta);
          for (int a = 0; a < pl.w; ++a) {
            int m1 = b1 + a;
            double om = 0.5 * w2 * kb_kernel(2.0 * (t1 - m1) / pl.w, pl.beta);
            int m1p = ((m1 % N) + N) % N;
            if (m2 >= 0 && m2 <= N / 2) fn((size_t)m2 * N + m1p, (uint32_t)n, (float)om);
            if (m2 <= 0 || m2 >= N / 2) {
              int mm1 = ((-m1 % N) + N) % N, mm2 = ((-m2 % N) + N) % N;
              fn((size_t)mm2 * N + mm1, (uint32_t)n | 0x80000000u, (float)om);
            }
          }
        }
      }
    };
    for_each_tap([&](size_t row, uint32_t, float) { cnt[row + 1]++; });
    pl.csr_ptr.assign(nrows + 1, 0);
    for (size_t r = 0; r < nrows; ++r) pl.csr_ptr[r + 1] = pl.csr_ptr[r] + cnt[r + 1];
    pl.csr.resize(pl.csr_ptr[nrows]);
    std::vector<int> fill(pl.csr_ptr.begin(), pl.csr_ptr.end() - 1);
    for_each_tap([&](size_t row, uint32_t node, float om) { pl.csr[fill[row]++] = SpreadEntry{node, om}; });

    // tiled form: per output cell, the pair entries of its point pairs and the distinct
    // nodes they use, in chunks
    const int CR = kSpreadRows, CC = kSpreadCols, NP = kSpreadPairs;
    const int ncy = (Nh + CR - 1) / CR, ncx = (N + CC - 1) / CC;
    pl.stiles.clear();
    pl.sblocks.clear();
    pl.schunks.clear();
    pl.snodes.clear();
    pl.sseg.clear();
    pl.sslot.clear();
    pl.sent.clear();
    pl.sent.reserve(pl.csr.size());
    struct PairTmp {
      uint32_t key;  // node * 2 + conjugate flag
      float wa, wb;
    };
    std::vector<int> where(pl.nodes.size(), -1);  // node -> index in the cell's node list
    std::vector<int> cell_nodes;
    std::vector<std::vector<PairTmp>> plist(NP);
    std::vector<int> chunk_cnt;  // entries per (chunk, pair) of a trial chunk count
    std::vector<std::pair<uint32_t, float>> la, lb;
    auto point_list = [&](int m2, int m1, std::vector<std::pair<uint32_t, float>>& out) {
      out.clear();
      if (m2 >= Nh || m1 >= N) return;
      const size_t row = (size_t)m2 * N + m1;
      for (int e = pl.csr_ptr[row]; e < pl.csr_ptr[row + 1]; ++e) {
        const uint32_t nd = pl.csr[e].node & 0x7fffffffu, cj = pl.csr[e].node >> 31;
        out.push_back({nd * 2u + cj, pl.csr[e].weight});
      }
      std::stable_sort(out.begin(), out.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    };
    auto padded = [](int n) { return (n + kSpreadBatch - 1) / kSpreadBatch * kSpreadBatch; };
    // lane groups (slots) of a pair: the pairs of a cell are taken by 1, 2, 4 or 8 tiles of
    // kSpreadPairs slots each; in a tile every pair starts with one slot and the pair with
    // the most entries per slot has its slots doubled while slots remain (at most 8: one
    // wavefront); a pair's slots form an aligned run inside one wavefront, so the kernel adds
    // their partial sums with a butterfly over lanes.  Returns the most entries of one slot.
    std::vector<int> slot_of(NP), split_of(NP);
    auto allocate = [&](int p0, int np) {
      int left = NP - np;
      for (int p = p0; p < p0 + np; ++p) split_of[p] = 1;
      for (;;) {
        int best = -1;
        double bv = 0.0;
        for (int p = p0; p < p0 + np; ++p) {
          const double v = (double)plist[p].size() / split_of[p];
          if (split_of[p] < 8 && split_of[p] <= left && !plist[p].empty() && v > bv) {
            bv = v;
            best = p;
          }
        }
        if (best < 0) break;
        left -= split_of[best];
        split_of[best] *= 2;
      }
      size_t most = 0;
      for (int p = p0; p < p0 + np; ++p)
        most = std::max(most, (plist[p].size() + split_of[p] - 1) / split_of[p]);
      return most;
    };
    std::vector<int> order_p(NP);
    std::vector<uint16_t> tile_slots(NP);
    for (int cy = 0; cy < ncy; ++cy)
      for (int cx = 0; cx < ncx; ++cx) {
        for (int pp = 0; pp < NP; ++pp) {
          const int m2 = cy * CR + 2 * (pp / CC), m1 = cx * CC + pp % CC;
          point_list(m2, m1, la);
          point_list(m2 + 1, m1, lb);
          auto& L2 = plist[pp];
          L2.clear();
          size_t i = 0, k = 0;
          while (i < la.size() || k < lb.size()) {
            if (k >= lb.size() || (i < la.size() && la[i].first < lb[k].first)) {
              L2.push_back({la[i].first, la[i].second, 0.f});
              ++i;
            } else if (i >= la.size() || lb[k].first < la[i].first) {
              L2.push_back({lb[k].first, 0.f, lb[k].second});
              ++k;
            } else {
              L2.push_back({la[i].first, la[i].second, lb[k].second});
              ++i;
              ++k;
            }
          }
        }
        // tiles per cell: the smallest count that is at least 15 % cheaper than the previous
        // choice (the per-step time of a tile is set by its fullest slot; a tile stages the
        // node values of all its pairs, so splitting a cell is not free)
        int T = 1;
        size_t cost = allocate(0, NP);
        for (int tt = 2; tt <= 8; tt *= 2) {
          size_t c = 0;
          for (int k = 0; k < tt; ++k) c += allocate(k * (NP / tt), NP / tt);
          if ((double)c < 0.85 * (double)cost) {
            cost = c;
            T = tt;
          }
        }
        for (int tk = 0; tk < T; ++tk) {
          const int p0 = tk * (NP / T), np = NP / T;
          allocate(p0, np);
          // slot layout: larger runs first, each at the first free aligned position
          for (int i = 0; i < np; ++i) order_p[i] = p0 + i;
          std::stable_sort(order_p.begin(), order_p.begin() + np,
                           [&](int x, int y) { return split_of[x] > split_of[y]; });
          std::fill(tile_slots.begin(), tile_slots.end(), (uint16_t)kSpreadIdleSlot);
          int next = 0;
          for (int i = 0; i < np; ++i) {
            const int p = order_p[i], sp = split_of[p];
            next = (next + sp - 1) / sp * sp;
            slot_of[p] = next;
            int lg = 0;
            while ((1 << lg) < sp) ++lg;
            for (int j = 0; j < sp; ++j) tile_slots[next + j] = (uint16_t)(p | (lg << 8));
            next += sp;
          }
          // nodes of this tile, in the order in which they first reach one of its pairs
          cell_nodes.clear();
          for (int p = p0; p < p0 + np; ++p)
            for (const PairTmp& t : plist[p]) {
              const int nd = (int)(t.key >> 1);
              if (where[nd] < 0) {
                where[nd] = (int)cell_nodes.size();
                cell_nodes.push_back(nd);
              }
            }
          SpreadTile t{cy * CR, cx * CC, (int)pl.schunks.size(), 0, 1, (int)pl.sslot.size(), 1, 0};
          for (int p = p0; p < p0 + np; ++p) t.maxs = std::max(t.maxs, split_of[p]);
          pl.sslot.insert(pl.sslot.end(), tile_slots.begin(), tile_slots.end());
          const int nn = (int)cell_nodes.size();
          // chunks: the tile's nodes dealt round-robin (node li to chunk li % nch), so that
          // every chunk takes about the same share of each pair's entries and the slots of
          // one step stay balanced; a pair's entries of a chunk are cut into its slots in
          // order; nch is the smallest count whose chunks hold at most kSpreadNodes nodes and,
          // padded per slot, kSpreadEntries entries
          auto part = [](int n, int sp, int j) { return (int)((long long)n * j / sp); };
          int nch = 0;
          if (nn > 0) {
            long long tot = 0;
            for (int p = p0; p < p0 + np; ++p) tot += (long long)plist[p].size();
            nch = std::max((nn + kSpreadNodes - 1) / kSpreadNodes, (int)((tot + kSpreadEntries - 1) / kSpreadEntries));
            for (;; ++nch) {
              chunk_cnt.assign((size_t)nch * NP, 0);
              for (int p = p0; p < p0 + np; ++p)
                for (const PairTmp& e : plist[p]) chunk_cnt[(size_t)(where[(int)(e.key >> 1)] % nch) * NP + p]++;
              bool fits = true;
              for (int c = 0; c < nch && fits; ++c) {
                int used = 0;
                for (int p = p0; p < p0 + np; ++p) {
                  const int n = chunk_cnt[(size_t)c * NP + p];
                  for (int j = 0; j < split_of[p]; ++j)
                    used += padded(part(n, split_of[p], j + 1) - part(n, split_of[p], j));
                }
                fits = used <= kSpreadEntries;
              }
              if (fits) break;
            }
          }
          std::vector<PairTmp> mine;
          for (int c = 0; c < nch; ++c) {
            SpreadChunk ch{(int)pl.snodes.size(), 0, (int)pl.sseg.size(), 0};
            for (int li = c; li < nn; li += nch) {
              const int nd = cell_nodes[li];
              pl.snodes.push_back(((nd / pl.H) << 16) | (nd % pl.H));
            }
            ch.n1 = (int)pl.snodes.size();
            for (int sl = 0; sl < NP; ++sl) {
              pl.sseg.push_back((int)pl.sent.size());
              if (tile_slots[sl] == kSpreadIdleSlot) continue;
              const int p = tile_slots[sl] & 63, sp = split_of[p], j = sl - slot_of[p];
              mine.clear();
              for (const PairTmp& e : plist[p])
                if (where[(int)(e.key >> 1)] % nch == c) mine.push_back(e);
              const int n = (int)mine.size();
              for (int i = part(n, sp, j); i < part(n, sp, j + 1); ++i) {
                const PairTmp& e = mine[i];
                const int li = where[(int)(e.key >> 1)];
                const bool cj = e.key & 1u;
                pl.sent.push_back(SpreadLocal{(uint32_t)(li / nch) * kImgGroup * 8u, cj ? -e.wa : e.wa,
                                              cj ? -e.wb : e.wb});
              }
              while (pl.sent.size() % kSpreadBatch) pl.sent.push_back(SpreadLocal{0u, 0.f, 0.f});
            }
            pl.sseg.push_back((int)pl.sent.size());
            pl.schunks.push_back(ch);
          }
          t.c1 = (int)pl.schunks.size();
          t.nsub = nch <= 1 ? 1 : std::min(kSpreadSlice, std::max(kSpreadSlice / kSpreadHeavyGroups, nch));
          pl.stiles.push_back(t);
          for (int nd : cell_nodes) where[nd] = -1;
        }
      }
    // workgroups of one slice: cells with the most chunks first, then in grid order
    std::vector<int> order(pl.stiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return pl.stiles[x].c1 - pl.stiles[x].c0 > pl.stiles[y].c1 - pl.stiles[y].c0;
    });
    for (int ti : order)
      for (int r = 0; r < pl.stiles[ti].nsub; ++r) pl.sblocks.push_back(SpreadBlock{ti, r});
    // the tiled form replaces the per-point lists
    std::vector<int>().swap(pl.csr_ptr);
    std::vector<SpreadEntry>().swap(pl.csr);
  }

  // grouped-GEMM work items
  pl.items_fwd.clear();
  pl.items_adj.clear();
  pl.items_cov.clear();
  pl.items_spca.clear();
  for (int k = 0; k <= pl.k_max; ++k) {
    for (int n0 = 0; n0 < pl.p[k]; n0 += 64) pl.items_spca.push_back(GemmItem{k, n0, 0, 0});
    for (int m0 = 0; m0 < pl.p[k]; m0 += kRadialRows) pl.items_fwd.push_back(GemmItem{k, m0, 0, 0});
    for (int j0 = 0; j0 < pl.n_xi; j0 += pl.bm) pl.items_adj.push_back(GemmItem{k, j0, 0, 0});
  }
  // covariance items: blocks whose segments and tiles fit one item go whole, packed in k
  // order while an item's segments and tiles allow; larger blocks tile by tile (column by
  // column of the upper triangle), a segment loaded again by each item that needs it (its
  // S0 sums by the first)
  {
    CovItem cur{};
    int nseg = 0, ntile = 0;
    auto reset = [&]() {
      cur = CovItem{};
      for (int s = 0; s < kCovSegs; ++s) cur.k[s] = -1;
      for (int w = 0; w < kCovWaves; ++w) cur.ta[w] = cur.tb[w] = 255;
      nseg = ntile = 0;
    };
    auto flush = [&]() {
      if (nseg > 0) pl.items_cov.push_back(cur);
      reset();
    };
    std::vector<char> summed;
    auto seg_slot = [&](int k, int i) {  // slot of segment i of block k, added if absent
      for (int s = 0; s < nseg; ++s)
        if (cur.k[s] == k && cur.q0[s] == i * kCovSeg) return s;
      cur.k[nseg] = (short)k;
      cur.q0[nseg] = (unsigned char)(i * kCovSeg);
      cur.row[nseg] = (int)pl.coef_off[k] + i * kCovSeg;
      cur.sum0[nseg] = (k == 0 && !summed[i]) ? 1 : 0;
      if (k == 0) summed[i] = 1;
      return nseg++;
    };
    reset();
    for (int k = 0; k <= pl.k_max; ++k) {
      const int nb = (pl.p[k] + kCovSeg - 1) / kCovSeg, nt = nb * (nb + 1) / 2;
      if (k == 0) summed.assign(nb, 0);
      const bool whole = nb <= kCovSegs && nt <= kCovWaves;
      if (whole && (nseg + nb > kCovSegs || ntile + nt > kCovWaves)) flush();
      for (int j = 0; j < nb; ++j)
        for (int i = 0; i <= j; ++i) {
          const int need = (i == j) ? 1 : 2;
          int have = 0;
          for (int s = 0; s < nseg; ++s) have += cur.k[s] == k && (cur.q0[s] == i * kCovSeg || cur.q0[s] == j * kCovSeg);
          if (nseg + need - have > kCovSegs || ntile + 1 > kCovWaves) flush();
          const int a = seg_slot(k, i), b = seg_slot(k, j);
          cur.ta[ntile] = (unsigned char)a;
          cur.tb[ntile] = (unsigned char)b;
          ++ntile;
        }
    }
    flush();
  }
  return FB_OK;
}

#define FB_HIP_TRY(expr)                \
  do {                                  \
    hipError_t e_ = (expr);             \
    if (e_ != hipSuccess) {             \
      pl.last_hip = e_;                 \
      free_device(pl);                  \
      return e_ == hipErrorOutOfMemory ? FB_ERR_ALLOC : FB_ERR_HIP; \
    }                                   \
  } while (0)

template <class T>
static hipError_t upload(T** dptr, const T* src, size_t count) {
  hipError_t e = hipMalloc((void**)dptr, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return e;
  if (count) e = hipMemcpy(*dptr, src, count * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

int upload_plan(Plan& pl) {
  FB_HIP_TRY(hipGetDevice(&pl.device));
  FB_HIP_TRY(hipDeviceGetAttribute(&pl.num_cus, hipDeviceAttributeMultiprocessorCount, pl.device));
  FB_HIP_TRY(configure_kernels());
  FB_HIP_TRY(configure_svd_kernels());
  FB_HIP_TRY(configure_eig_kernels());
  size_t nb = (size_t)pl.p_half * pl.n_xi;
  std::vector<float> r32(nb);
  for (size_t i = 0; i < nb; ++i) r32[i] = (float)pl.radial[i];
  FB_HIP_TRY(upload(&pl.d_radial, r32.data(), nb));
  // the BF16x3 operand split of the FP32 table, x = hi + lo with hi = bf16(x) and lo =
  // bf16(x - hi), both rounded to nearest even (x - hi is exact in FP32)
  pl.n_xi_pad = (pl.n_xi + kRadialK - 1) / kRadialK * kRadialK;
  {
    const size_t nbp = (size_t)pl.p_half * pl.n_xi_pad;
    auto bf16_rne = [](float f) {
      uint32_t u;
      std::memcpy(&u, &f, sizeof u);
      u += 0x7fffu + ((u >> 16) & 1u);
      return (unsigned short)(u >> 16);
    };
    auto bf16_val = [](unsigned short h) {
      const uint32_t u = (uint32_t)h << 16;
      float f;
      std::memcpy(&f, &u, sizeof f);
      return f;
    };
    std::vector<unsigned short> bf(2 * nbp, 0);
    for (long long r = 0; r < pl.p_half; ++r)
      for (int j = 0; j < pl.n_xi; ++j) {
        const float x = r32[(size_t)r * pl.n_xi + j];
        const unsigned short h = bf16_rne(x);
        bf[(size_t)r * pl.n_xi_pad + j] = h;
        bf[nbp + (size_t)r * pl.n_xi_pad + j] = bf16_rne(x - bf16_val(h));
      }
    FB_HIP_TRY(upload(&pl.d_radial_bf, bf.data(), bf.size()));
    std::vector<float> pad(nbp, 0.f);
    for (long long r = 0; r < pl.p_half; ++r)
      std::copy(r32.begin() + (size_t)r * pl.n_xi, r32.begin() + (size_t)(r + 1) * pl.n_xi,
                pad.begin() + (size_t)r * pl.n_xi_pad);
    FB_HIP_TRY(upload(&pl.d_radial_pad, pad.data(), pad.size()));
  }
  std::vector<float> xw(pl.n_xi);
  for (int j = 0; j < pl.n_xi; ++j) xw[j] = (float)(pl.xi[j] * pl.wq[j]);
  FB_HIP_TRY(upload(&pl.d_xw, xw.data(), xw.size()));
  FB_HIP_TRY(upload(&pl.d_xi, pl.xi.data(), pl.xi.size()));
  FB_HIP_TRY(upload(&pl.d_wq, pl.wq.data(), pl.wq.size()));
  FB_HIP_TRY(upload(&pl.d_roots, pl.roots.data(), pl.roots.size()));
  std::vector<int> off32(pl.coef_off.begin(), pl.coef_off.end());
  FB_HIP_TRY(upload(&pl.d_coef_off, off32.data(), off32.size()));
  FB_HIP_TRY(upload(&pl.d_p, pl.p.data(), pl.p.size()));
  std::vector<long long> coff(pl.cov_off.begin(), pl.cov_off.end());
  FB_HIP_TRY(upload(&pl.d_cov_off, coff.data(), coff.size()));
  FB_HIP_TRY(upload(&pl.d_tri_off, pl.tri_off.data(), pl.tri_off.size()));
  std::vector<float> dc(pl.deconv.begin(), pl.deconv.end());
  FB_HIP_TRY(upload(&pl.d_deconv, dc.data(), dc.size()));
  FB_HIP_TRY(upload(&pl.d_gnodes, pl.gnodes.data(), pl.gnodes.size()));
  FB_HIP_TRY(upload(&pl.d_gitems, pl.gitems.data(), pl.gitems.size()));
  FB_HIP_TRY(upload(&pl.d_tw, (const float2*)pl.tw.data(), pl.tw.size() / 2));
  FB_HIP_TRY(upload(&pl.d_angtw, (const float2*)pl.angtw.data(), pl.angtw.size() / 2));
  FB_HIP_TRY(upload(&pl.d_stiles, pl.stiles.data(), pl.stiles.size()));
  FB_HIP_TRY(upload(&pl.d_sblocks, pl.sblocks.data(), pl.sblocks.size()));
  FB_HIP_TRY(upload(&pl.d_schunks, pl.schunks.data(), pl.schunks.size()));
  FB_HIP_TRY(upload(&pl.d_snodes, pl.snodes.data(), pl.snodes.size()));
  FB_HIP_TRY(upload(&pl.d_sseg, pl.sseg.data(), pl.sseg.size()));
  FB_HIP_TRY(upload(&pl.d_sslot, pl.sslot.data(), pl.sslot.size()));
  FB_HIP_TRY(upload(&pl.d_sent, pl.sent.data(), pl.sent.size()));
  FB_HIP_TRY(upload(&pl.d_items_fwd, pl.items_fwd.data(), pl.items_fwd.size()));
  FB_HIP_TRY(upload(&pl.d_items_adj, pl.items_adj.data(), pl.items_adj.size()));
  FB_HIP_TRY(upload(&pl.d_items_cov, pl.items_cov.data(), pl.items_cov.size()));
  FB_HIP_TRY(upload(&pl.d_items_spca, pl.items_spca.data(), pl.items_spca.size()));
  FB_HIP_TRY(upload(&pl.d_jmin, pl.jmin.data(), pl.jmin.size()));
  FB_HIP_TRY(upload(&pl.d_kring, pl.kring.data(), pl.kring.size()));
  FB_HIP_TRY(upload(&pl.d_gcols, pl.gcols.data(), pl.gcols.size()));
  pl.has_device = true;
  return FB_OK;
}

void free_device(Plan& pl) {
  if (pl.has_device) pl.prof.release();
  void* ptrs[] = {pl.d_radial,    pl.d_radial_bf, pl.d_radial_pad, pl.d_xw,        pl.d_xi,        pl.d_wq,        pl.d_roots,     pl.d_coef_off,  pl.d_p,         pl.d_cov_off,   pl.d_tri_off,
                  pl.d_deconv,    pl.d_gnodes,    pl.d_gitems,    pl.d_tw,        pl.d_angtw,
                  pl.d_stiles,    pl.d_sblocks,   pl.d_schunks,   pl.d_snodes,    pl.d_sseg,      pl.d_sslot,     pl.d_sent,
                  pl.d_items_fwd, pl.d_items_adj, pl.d_items_cov, pl.d_items_spca,
                  pl.d_jmin,      pl.d_kring,     pl.d_gcols};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  pl.d_radial = nullptr;
  pl.d_radial_bf = nullptr;
  pl.d_radial_pad = nullptr;
  pl.d_xw = nullptr;
  pl.d_xi = nullptr;
  pl.d_wq = nullptr;
  pl.d_roots = nullptr;
  pl.d_coef_off = pl.d_p = nullptr;
  pl.d_cov_off = nullptr;
  pl.d_tri_off = nullptr;
  pl.d_deconv = nullptr;
  pl.d_gnodes = nullptr;
  pl.d_gitems = nullptr;
  pl.d_tw = pl.d_angtw = nullptr;
  pl.d_stiles = nullptr;
  pl.d_sblocks = nullptr;
  pl.d_schunks = nullptr;
  pl.d_snodes = nullptr;
  pl.d_sseg = nullptr;
  pl.d_sslot = nullptr;
  pl.d_sent = nullptr;
  pl.d_items_fwd = pl.d_items_adj = pl.d_items_spca = nullptr;
  pl.d_items_cov = nullptr;
  pl.d_jmin = pl.d_kring = pl.d_gcols = nullptr;
  pl.has_device = false;
}

const char* stage_name(int s) {
  static const char* names[ST_COUNT] = {"fwd_rows",    "fwd_cols",   "fwd_gather", "fwd_angular",
                                        "radial_fwd",  "covariance", "radial_adj", "adj_angular",
                                        "adj_spread",  "adj_cols",   "adj_rows",   "eig",
                                        "spca",        "svd",        "estimate"};
  return (s >= 0 && s < ST_COUNT) ? names[s] : "unknown";
}

hipEvent_t Profiler::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void Profiler::begin(int stage, hipStream_t st) {
  if (!on) return;
  Rec r{stage, take(), take()};
  if (!r.a || !r.b) return;
  (void)hipEventRecord(r.a, st);
  recs.push_back(r);
}

void Profiler::end(hipStream_t st) {
  if (!on || recs.empty()) return;
  (void)hipEventRecord(recs.back().b, st);
}

int Profiler::collect() {
  int rc = FB_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) rc = FB_ERR_HIP;
    total_ms[r.stage] += ms;
    launches[r.stage] += 1;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
  return rc;
}

void Profiler::release() {
  collect();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

PassLayout pass_layout(const Plan& pl) {
  PassLayout lay;
  const size_t c8 = 8;  // complex64
  size_t a1 = (size_t)pl.M2 * pl.L;                    // forward row pass output
  size_t a2 = (size_t)pl.n_xi * pl.H;                  // polar samples / adjoint Q
  size_t a3 = (size_t)(pl.N / 2 + 1) * pl.L;           // adjoint column pass output
  size_t b1 = (size_t)pl.M2 * pl.N;                    // forward grid
  size_t b2 = (size_t)(pl.k_max + 1) * pl.n_xi;        // angular spectrum / adjoint D
  size_t b3 = (size_t)(pl.N / 2 + 1) * pl.N;           // adjoint folded grid
  lay.bytes_a = std::max(a1, std::max(a2, a3)) * c8;
  lay.bytes_b = std::max(b1, std::max(b2, b3)) * c8;
  lay.per_image = lay.bytes_a + lay.bytes_b;
  return lay;
}

}  // namespace fb
