// Output-stationary grouped GEMM on gfx950 MFMA.
//
// A launch is a list of output tiles.  Each tile owns a rectangle of one
// output matrix C and a contiguous range of segments; every segment adds
// alpha * A * B (A: m x k, B: k x n, either may be stored transposed) to the
// same tile, so all contributions to a tile accumulate in registers and the
// tile is written once.  No two tiles of one launch may overlap in C.
#pragma once
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

  // Adds one output problem C (m x n, ldc) += sum over segs [s0, s1).
  // The problem is split into kTileM x kTileN tiles that share the segments.
  void add_problem(void* c, int ldc, int m, int n, size_t s0, size_t s1, int beta) {
    if (m <= 0 || n <= 0 || s1 <= s0) return;
    for (int r = 0; r < m; r += kTileM)
      for (int q = 0; q < n; q += kTileN) {
        GemmTile t;
        t.c = c;
        t.ldc = ldc;
        t.m = std::min(kTileM, m - r);
        t.n = std::min(kTileN, n - q);
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

// Launch (stream-ordered).  dev_scratch holds the uploaded descriptors; it is
// grown as needed; the call returns after the launch is enqueued and the
// descriptor copies have completed.
void launch_gemm_f64(const GemmBatch& b, DevBuf& dev_scratch, hipStream_t stream);

// Descriptors uploaded once and launched many times (no host work per launch).
struct DevGemm {
  DevBuf buf;
  GemmSeg* segs = nullptr;
  GemmTile* tiles = nullptr;
  size_t ntiles = 0, nsegs = 0;
  double flops = 0;
};
void upload_gemm(const GemmBatch& b, DevGemm& d);
void launch_gemm_f64(const DevGemm& d, hipStream_t stream, int role = 0);

// ---- elementwise / BLAS-1 helpers (FP64) ----------------------------------
void launch_scale(double* x, double a, int64_t n, hipStream_t s);
void launch_axpy(double* y, double a, const double* x, int64_t n, hipStream_t s);
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
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
