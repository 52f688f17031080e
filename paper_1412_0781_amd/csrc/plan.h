// Internal plan of the library: FP64 host tables (Algorithm 1, steps 1-2) and
// their device copies, plus launch descriptors for the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ffbspca.h"

namespace fb {

constexpr int kMaxRadices = 24;

// Division by a divisor fixed on the host, for 0 <= x < 2^31 and 1 <= d < 2^31:
// q = floor(x * m / 2^s) with s = 31 + ceil(log2 d) and m = floor(2^s / d) + 1.
// The error term x (m - 2^s/d) / 2^s is below x / 2^s < 2^-ceil(log2 d) <= 1/d, so
// the floor equals floor(x / d).  m < 2^32 for every such d.
struct FastDiv {
  unsigned m;
  unsigned s;
  int d;
  int pad;
#ifdef __HIPCC__
  __host__ __device__
#endif
  inline int div(int x) const { return (int)(((unsigned long long)(unsigned)x * m) >> s); }
};
inline FastDiv make_fastdiv(int d) {
  unsigned c = 0;
  while ((1ull << c) < (unsigned long long)d) ++c;
  unsigned s = 31 + c;
  unsigned long long m = ((1ull << s) / (unsigned long long)d) + 1ull;
  return FastDiv{(unsigned)m, s, d, 0};
}

// One FFT length: its radix sequence and where its twiddles
// exp(-2 pi i t / n), t = 0..n-1, start in the plan's twiddle table.
struct FftDesc {
  int n;
  int nstage;
  int tw_off;
  int pad;
  int radix[kMaxRadices];
  FastDiv dnb[kMaxRadices];  // division by n / radix[s]
  FastDiv dns[kMaxRadices];  // division by radix[0] * ... * radix[s-1]
};

// Interpolation footprint of one polar node (j, l), l < n_theta/2, on the
// oversampled grid: grid coordinate t = grid_n * xi (first axis t1 = along i1,
// second t2 = along i2); the w x w taps start at integer b = ceil(t - w/2) and
// carry weights phi(2 (f - a) / w), a = 0..w-1, with f = t - b.
struct NodeTap {
  int b1;    // first tap column, reduced modulo grid_n into [0, grid_n)
  int b2;    // first tap row index into the stored half-plane rows (m2 + hw >= 0)
  float f1;  // t1 - ceil(t1 - w/2)
  float f2;  // t2 - ceil(t2 - w/2)
};

// Forward gather, LDS-tiled: nodes grouped by the kGatherCell x kGatherCell grid cell
// holding their tap origin.  A workgroup stages the cell's box of
// (kGatherCell + w - 1)^2 grid points (for a group of images) in LDS and
// interpolates its nodes from there.
constexpr int kGatherCell = 14;
// Pass buffers that keep images innermost store them in groups of kImgGroup:
// X[outer][group][inner][kImgGroup], a pass of m images using ceil(m / kImgGroup)
// groups (the slots past m hold zeros).  One group of one (outer, inner) entry is a
// 128-byte line, and a workgroup's tile of one group is one contiguous run.
constexpr int kImgGroup = 16;
constexpr int kGatherW = 7;                       // kernel width the gather kernels are built for
constexpr int kGatherChunk = 1024;                // nodes per work item at most
struct GatherNode {
  unsigned short j, l;   // polar node: ring j, angle l (< H)
  int off;               // tap origin inside the cell box: row * (cell + w - 1) + col
  float w1[kGatherW];    // weights along the first grid axis (i1 / x)
  float w2[kGatherW];    // weights along the second grid axis (i2 / y)
};
struct GatherItem {
  int c1, c2;  // cell origin in grid columns (m1, before wrap) and stored rows (m2 + hw)
  int s0, s1;  // node range in the cell-sorted node list
};

// Adjoint spreading, written as a gather: entry of grid point (m1, m2) of the
// folded half-plane m2 = 0..grid_n/2.  node index in bits 0..30, bit 31 set when
// the node's conjugate contributes (Hermitian fold of the m2 < 0 / m2 > n/2 taps).
struct SpreadEntry {
  uint32_t node;
  float weight;
};
// Tiled adjoint spread: the folded half-plane grid is cut into cells of kSpreadRows x
// kSpreadCols output points, taken as pairs of vertically neighbouring points (m2, m2 + 1),
// which share most of the nodes that reach them.  The nodes that reach a cell are listed
// once (packed j << 16 | l) and split into chunks of at most kSpreadNodes nodes and
// kSpreadEntries pair entries; a workgroup stages one chunk's node values (one image
// group) and entries in LDS, and every pair sums its entries of that chunk: one entry per
// (node, conjugate flag) reaching either point, with the LDS offset of the node's values
// and one weight per point (0 where the node misses that point), in node order.  Each
// pair's entries of a chunk are padded with zero-weight entries to a multiple of
// kSpreadBatch, so that they are read in aligned batches.  A cell with several chunks is
// split over nsub >= kSpreadSlice / kSpreadHeavyGroups workgroups per slice of
// kSpreadSlice image groups (workgroup r of the cell takes groups r, r + nsub, ...), each
// walking the chunks in order with the next image group's values prefetched and
// per-group partial sums in registers.  The pairs of a cell whose entry counts differ
// widely (near the origin, where the rings crowd) are shared out over up to 8 tiles, and in
// a tile a pair may take 1, 2, 4 or 8 of the kSpreadPairs lane groups (slots), each summing
// a contiguous part of the pair's entries; the slot table of a tile maps slot -> pair.
constexpr int kSpreadRows = 16;
constexpr int kSpreadCols = 8;
constexpr int kSpreadPairs = kSpreadRows / 2 * kSpreadCols;
constexpr int kSpreadNodes = 256;
constexpr int kSpreadEntries = 4096;
constexpr int kSpreadBatch = 4;
constexpr int kSpreadSlice = 16;
constexpr int kSpreadHeavyGroups = 2;
// slot table entry: pair index in the cell (bits 0-5) | log2 of the pair's slot count << 8,
// or kSpreadIdleSlot for a slot without a pair
constexpr uint16_t kSpreadIdleSlot = 0x8000;
struct SpreadTile {
  int m2, m1;    // cell origin (row m2 of the half plane, column m1)
  int c0, c1;    // chunk range
  int nsub;      // workgroups per slice of image groups
  int slots;     // first of its kSpreadPairs slot table entries
  int maxs;      // most slots of one pair (1: slot = pair)
  int pad;
};
struct SpreadBlock {
  int tile;      // index into the cell list
  int sub;       // 0 .. nsub-1
};
struct SpreadChunk {
  int n0, n1;    // node range in the chunk node list
  int seg;       // kSpreadPairs + 1 entry offsets of this chunk's pairs start here
  int pad;
};
struct SpreadLocal {
  uint32_t off;   // byte offset of the node's values (one image group) in the chunk's LDS copy
  float wa, wb;   // spreading weights (>= 0) of the upper and lower point, each negated when
                  // that point takes the conjugate of the node value
};

// Kernel stages, in launch order (names in stage_name()).
enum Stage {
  ST_FWD_ROWS = 0,
  ST_FWD_COLS,
  ST_FWD_GATHER,
  ST_FWD_ANGULAR,
  ST_RADIAL_FWD,
  ST_COVARIANCE,
  ST_RADIAL_ADJ,
  ST_ADJ_ANGULAR,
  ST_ADJ_SPREAD,
  ST_ADJ_COLS,
  ST_ADJ_ROWS,
  ST_EIG,
  ST_SPCA,
  ST_SVD,
  ST_ESTIMATE,
  ST_COUNT
};
const char* stage_name(int s);

// Optional per-kernel timing: HIP events recorded on the caller's stream around
// every kernel launch of a plan while enabled.  Not for concurrent use of one
// plan from several streams.
struct Profiler {
  bool on = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double total_ms[ST_COUNT] = {};
  long long launches[ST_COUNT] = {};
  hipEvent_t take();
  void begin(int stage, hipStream_t st);
  void end(hipStream_t st);
  int collect();  // folds completed records into the totals; returns FB_OK or FB_ERR_HIP
  void release();
};

constexpr int kRadialRows = 128;  // row tile of the radial quadrature GEMM
constexpr int kRadialK = 32;      // K chunk of the radial quadrature GEMM (rows of the BF16 table padded to it)
// Radial table entries below this fraction of their row's largest entry are treated as zero:
// J_k(x) decays faster than exponentially for x below its turning point x ~ k, so for large k
// the inner rings add nothing an FP32 sum can hold (the dropped terms of a row sum to less
// than n_xi 2^-30 of its largest term).
constexpr double kRadialNegligible = 1.0 / (1u << 30);

struct GemmItem {  // one (k, tile) work item of a grouped GEMM
  int k;
  int t0;  // first row (or first row tile) of the tile
  int t1;  // second tile coordinate (unused)
  int pad;
};

// Covariance work item: up to kCovSegs segments of kCovSeg consecutive coefficients, each
// inside one block k (starting at a multiple of kCovSeg in the block), staged together for
// every chunk of images, and up to kCovWaves tiles (one per wave): the kCovSeg x kCovSeg
// products of two segments of the same block.  A block of at most 3 kCovSeg coefficients
// sits in one item (all its tiles, every coefficient read once); small blocks share items.
constexpr int kCovSeg = 32;
constexpr int kCovSegs = 4;
constexpr int kCovWaves = 8;
struct CovItem {
  int row[kCovSegs];                // first coefficient of the segment (index < p_half)
  short k[kCovSegs];                // its block, -1 for an unused slot
  unsigned char q0[kCovSegs];       // its first row inside the block (blocks hold <= 256 rows)
  unsigned char sum0[kCovSegs];     // 1: this item adds the segment's k = 0 sums (S0)
  unsigned char ta[kCovWaves], tb[kCovWaves];  // segments of wave w's tile (ta <= tb), 255: none
};
static_assert(sizeof(CovItem) == 48, "a covariance item is three 16-byte words");

struct Plan {
  // problem
  int L = 0;
  double c = 0, R = 0;
  int n_xi = 0, n_theta = 0, k_max = 0, p0 = 0;
  int64_t p_half = 0, p_total = 0, cov_size = 0;
  std::vector<int> p;               // p_k
  std::vector<int64_t> coef_off;    // k_max + 2
  std::vector<int64_t> cov_off;     // k_max + 2
  std::vector<long long> tri_off;   // k_max + 2: offsets of packed p_k x p_k upper triangles
  std::vector<int> kq_k, kq_q;      // p_half
  std::vector<double> roots, norms; // p_half
  std::vector<double> xi, wq;       // n_xi
  std::vector<double> radial;       // p_half x n_xi

  // non-uniform FFT
  int N = 0;        // oversampled grid side
  int w = 0;        // kernel width
  double beta = 0;  // kernel shape
  int hw = 0;       // half-plane rows stored: m2 = -hw .. N/2 + hw
  int M2 = 0;       // = N/2 + 2 hw + 1
  int H = 0;        // n_theta / 2: half-ring nodes, also the complex FFT length of the angular step
  std::vector<double> deconv;      // 1 / phi_hat(x / N), x over pixel indices
  std::vector<NodeTap> nodes;      // n_xi * H, node n = j * H + l
  std::vector<GatherNode> gnodes;  // nodes sorted by gather cell
  std::vector<GatherItem> gitems;  // (cell, node chunk) work items
  // per stored grid row m2 (M2 rows): the centred m1 range [lo, hi] (m1 - N for m1 >= N/2)
  // that holds every point some gather box reads (lo > hi if none); the streaming column
  // pass stores only these points of G
  std::vector<int> gcols;          // 2 * M2: lo, hi
  FftDesc fft_grid{}, fft_ang{};
  std::vector<float> tw;           // interleaved (re, im) twiddles of both FFT lengths
  std::vector<float> angtw;        // exp(-2 pi i k / n_theta), k = 0..H, interleaved
  std::vector<int> csr_ptr;        // N * (N/2 + 1) + 1
  std::vector<SpreadEntry> csr;    // spreading entries, by grid point
  std::vector<SpreadTile> stiles;  // tiled form of the same entries
  std::vector<SpreadBlock> sblocks; // workgroups of one image-group slice, heaviest cells first
  std::vector<SpreadChunk> schunks;
  std::vector<int> snodes;         // j << 16 | l
  std::vector<int> sseg;
  std::vector<uint16_t> sslot;     // kSpreadPairs slot table entries per tile
  std::vector<SpreadLocal> sent;
  std::vector<GemmItem> items_fwd, items_adj, items_spca;
  std::vector<CovItem> items_cov;
  // rings the radial sum of block k reads: j >= jmin[k] (the first ring where some row of
  // block k reaches kRadialNegligible of its largest entry); kring[j] = the largest k with
  // jmin[k] <= j (-1 if none): the angular step writes F-hat(j, k) for k <= kring[j] only
  std::vector<int> jmin, kring;
  int bm = 64, bn = 64;            // GEMM tile

  mutable Profiler prof;

  // device
  bool has_device = false;
  int device = -1;
  int num_cus = 256;                  // compute units of the device (sizes persistent launches)
  hipError_t last_hip = hipSuccess;
  float* d_radial = nullptr;          // FP32 copy of radial, p_half x n_xi
  unsigned short* d_radial_bf = nullptr;  // its BF16 hi parts, then its lo parts: 2 x p_half x n_xi_pad, zero-padded
  float* d_radial_pad = nullptr;      // FP32 radial with rows zero-padded to n_xi_pad, p_half x n_xi_pad
  int n_xi_pad = 0;                   // n_xi rounded up to kRadialK
  float* d_xw = nullptr;              // xi_j w_j, n_xi (the radial table's quadrature factor)
  double* d_roots = nullptr;          // R_{k,q} at coef_off[k] + q - 1 (FP64, p_half)
  double* d_xi = nullptr;             // Gauss-Legendre nodes xi_j (FP64, n_xi)
  double* d_wq = nullptr;             // Gauss-Legendre weights w_j (FP64, n_xi)
  int* d_coef_off = nullptr;          // k_max + 2 (fits int32)
  int* d_p = nullptr;                 // k_max + 1
  long long* d_cov_off = nullptr;     // k_max + 2
  long long* d_tri_off = nullptr;     // k_max + 2
  float* d_deconv = nullptr;
  GatherNode* d_gnodes = nullptr;
  GatherItem* d_gitems = nullptr;
  float2* d_tw = nullptr;
  float2* d_angtw = nullptr;
  SpreadTile* d_stiles = nullptr;
  SpreadBlock* d_sblocks = nullptr;
  SpreadChunk* d_schunks = nullptr;
  int* d_snodes = nullptr;
  int* d_sseg = nullptr;
  uint16_t* d_sslot = nullptr;
  SpreadLocal* d_sent = nullptr;
  GemmItem* d_items_fwd = nullptr;
  GemmItem* d_items_adj = nullptr;
  CovItem* d_items_cov = nullptr;
  GemmItem* d_items_spca = nullptr;   // (k, 64-wide column tile) of the steerable-PCA products
  int* d_jmin = nullptr;              // k_max + 1
  int* d_kring = nullptr;             // n_xi
  int* d_gcols = nullptr;             // 2 * M2
};

// Build host tables; returns FB_OK or an FB_ERR_* code.
int build_host_plan(int L, double c, double R, Plan& pl);
// Upload to the current device; returns FB_OK / FB_ERR_HIP / FB_ERR_ALLOC.
int upload_plan(Plan& pl);
void free_device(Plan& pl);

// Per-image workspace layout of one expand/adjoint pass.
struct PassLayout {
  size_t bytes_a;   // buffer A: row-pass output, later polar samples
  size_t bytes_b;   // buffer B: grid, later angular spectrum
  size_t per_image;
};
PassLayout pass_layout(const Plan& pl);

}  // namespace fb

// The handle behind fb_plan_t.
struct fb_plan_s {
  fb::Plan pl;
};
