// Output-stationary grouped GEMM on gfx950 MFMA.
//
// A launch is a list of output tiles.  Each tile owns a rectangle of one
// output matrix C and a contiguous range of segments; every segment adds
// alpha * A * B (A: m x k, B: k x n, either may be stored transposed) to the
// same tile, so all contributions to a tile accumulate in registers and the
// tile is written once.  No two tiles of one launch may overlap in C.
#pragma once
#include <algorithm>
#include <cstdint>
#include <vector>

#include "common.h"

namespace dmrg {

enum SegFlags : int32_t {
  kTransA = 1,  // A stored k x m: A[i][k] = a[k * lda + i]
  kTransB = 2,  // B stored n x k: B[k][j] = b[j * ldb + k]
};

struct GemmSeg {
  const void* a;
  const void* b;
  int32_t lda, ldb, k, flags;
  double alpha;
};

struct GemmTile {
  void* c;
  int32_t ldc;
  int32_t m, n;        // valid rows / cols of this tile
  int32_t row0, col0;  // tile origin inside the problem (offsets A rows / B cols)
  int32_t seg_begin, seg_end;
  int32_t beta;        // 0: C = sum, 1: C += sum
  int32_t pad;
};

constexpr int kTileM = 64;
constexpr int kTileN = 64;

// Host-side accumulation of one launch.
struct GemmBatch {
  std::vector<GemmSeg> segs;
  std::vector<GemmTile> tiles;
  double flops = 0;  // algorithmic 2*m*n*k over all segments
  // output tile of the launch (rows x cols): 64 x 64 (4 waves), 128 x 128,
  // 128 x 64 or 64 x 128 (8 waves)
  int tile = kTileM, tile_n = kTileN;

  // Adds one output problem C (m x n, ldc) += sum over segs [s0, s1).
  // The problem is split into tile x tile_n pieces that share the segments.
  void add_problem(void* c, int ldc, int m, int n, size_t s0, size_t s1, int beta) {
    if (m <= 0 || n <= 0 || s1 <= s0) return;
    for (int r = 0; r < m; r += tile)
      for (int q = 0; q < n; q += tile_n) {
        GemmTile t;
        t.c = c;
        t.ldc = ldc;
        t.m = std::min(tile, m - r);
        t.n = std::min(tile_n, n - q);
        t.row0 = r;
        t.col0 = q;
        t.seg_begin = (int32_t)s0;
        t.seg_end = (int32_t)s1;
        t.beta = beta;
        t.pad = 0;
        tiles.push_back(t);
      }
    for (size_t s = s0; s < s1; ++s) flops += 2.0 * m * n * segs[s].k;
  }
  void clear() { segs.clear(); tiles.clear(); flops = 0; }
};

// MI355X hands the workgroups of a launch to its 8 XCDs round-robin by block
// index (block b runs on XCD b mod 8), and each XCD has its own L2.
constexpr int kXcds = 8;

// Reorders a launch's tiles for L2 locality.  key[t] names a locality group
// (tiles of one group share operands: the caller emits them consecutively,
// problem by problem, each problem's tiles row by row).  A group runs on one
// XCD, in emission order; groups are spread over the XCDs longest first onto
// the least loaded one, a group larger than a quarter of an XCD's share being
// cut at problem boundaries into pieces of about that size (cost(tile)
// estimates a tile's time).  Queues are interleaved so that block b takes the
// next tile of XCD b mod 8's queue; shorter queues are padded with empty
// tiles (m = 0), which the kernels skip.
template <class Tile, class Cost>
void xcd_order(std::vector<Tile>& tiles, const std::vector<int>& key, Cost&& cost) {
  struct Group {
    size_t t0, t1;
    double c;
  };
  const size_t nt = tiles.size();
  std::vector<double> tc(nt);
  double total = 0;
  for (size_t i = 0; i < nt; ++i) total += (tc[i] = cost(tiles[i]));
  const double cap = std::max(1.0, total / (4.0 * kXcds));
  auto same_problem = [&](size_t a, size_t b) {
    return tiles[a].c == tiles[b].c && tiles[a].seg_begin == tiles[b].seg_begin &&
           tiles[a].seg_end == tiles[b].seg_end;
  };
  std::vector<Group> groups;
  for (size_t i = 0; i < nt;) {
    size_t j = i;
    double c = 0;
    // extend over whole problems of the same key up to the cap
    while (j < nt && key[j] == key[i]) {
      size_t e = j + 1;
      while (e < nt && same_problem(e, j)) ++e;
      double pc = 0;
      for (size_t k = j; k < e; ++k) pc += tc[k];
      if (j > i && c + pc > cap) break;
      c += pc;
      j = e;
    }
    groups.push_back({i, j, c});
    i = j;
  }
  std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.c > b.c; });
  std::vector<std::vector<size_t>> queue(kXcds);
  double load[kXcds] = {};
  for (const Group& g : groups) {
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (load[y] < load[x]) x = y;
    for (size_t k = g.t0; k < g.t1; ++k) queue[x].push_back(k);
    load[x] += g.c;
  }
  size_t len = 0;
  for (auto& q : queue) len = std::max(len, q.size());
  Tile empty{};
  std::vector<Tile> out;
  out.reserve(len * kXcds);
  for (size_t i = 0; i < len; ++i)
    for (int x = 0; x < kXcds; ++x) out.push_back(i < queue[x].size() ? tiles[queue[x][i]] : empty);
  tiles.swap(out);
}

// Launch (stream-ordered, no host synchronisation).  The descriptors are
// copied into pinned staging memory of the library, so the caller may
// release b as soon as the call returns; operand and output buffers must stay
// valid until the launch has run.
void launch_gemm_f64(const GemmBatch& b, hipStream_t stream);

// Descriptors uploaded once and launched many times (no host work per launch).
struct DevGemm {
  DevBuf buf;
  GemmSeg* segs = nullptr;
  GemmTile* tiles = nullptr;
  size_t ntiles = 0, nsegs = 0;
  double flops = 0;
  int tile = kTileM, tile_n = kTileN;
  bool lds = false;  // every segment suits the direct-to-LDS kernel
};
void upload_gemm(const GemmBatch& b, DevGemm& d);
void launch_gemm_f64(const DevGemm& d, hipStream_t stream, int role = 0);

// ---- elementwise / BLAS-1 helpers (FP64) ----------------------------------
void launch_scale(double* x, double a, int64_t n, hipStream_t s);
void launch_axpy(double* y, double a, const double* x, int64_t n, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
// z = a x + b y (z may alias x or y)
void launch_axpby(double* z, double a, const double* x, double b, const double* y, int64_t n,
                  hipStream_t s);
// out[j] = sum_i X[j][i] * y[i] for j < nv (X rows of length n, row stride ldx)
void launch_multidot(double* out, const double* X, int64_t ldx, int nv, const double* y,
                     int64_t n, hipStream_t s);
// y = sum_j c[j] * X[j] (+ beta * y)
void launch_lincomb(double* y, const double* X, int64_t ldx, int nv, const double* c,
                    int64_t n, double beta, hipStream_t s);
// block copies (one workgroup per task), optionally transposing
struct CopyTask;
void launch_copy_tasks(const CopyTask* tasks, int ntasks, bool transpose, hipStream_t s);
// scatter-add rows: dst[idx[r]] += src[r]   (rows of length n)
void launch_row_scatter_add(double* dst, const double* src, const int64_t* dst_off, int nrows,
                            int64_t n, hipStream_t s);

}  // namespace dmrg
