// FP64 matrix products emulated on INT8 MFMA (Ozaki scheme).
//
// Every row of an operand (rows of A, rows of the n x k storage of B) is
// scaled by a power of two 2^-e, |x| < 2^e over the row, and rounded to an
// integer X = round(x 2^(p - e)) of p = 8 kappa - 1 bits.  X is split into
// kappa signed base-256 digits d_0 .. d_(kappa-1) in [-128, 127]
// (X = sum_s d_s 256^s), one int8 plane per digit.  A product then is
//   (A B)_ij = 2^(e_i + f_j - 2p) sum_(s,t) 256^(s+t) (D_s^A D_t^B)_ij,
// of which the kappa (kappa + 1) / 2 digit products with s + t >= kappa - 1
// are kept (the dropped ones lie below the rounding of X).  Each digit
// product is exact in INT32 (|d| <= 128, k < 2^31 / (kappa 2^14) for the
// products of one weight s + t summed together); the weights are combined in
// FP64 at the end of each segment, scaled by the row exponents.
#pragma once
#include <cstdint>
#include <vector>

#include "gemm_bf16.h"

namespace dmrg {

constexpr int kOzMinKappa = 3, kOzMaxKappa = 7;
constexpr int kOzTile = 64;  // output tile rows and columns
constexpr int kOzBK = 64;    // int8 k entries per slab

// Segment: A (m x k) and B (stored n x k) as digit planes, kp = k rounded up
// to 16 bytes per row; plane s of A at a + s * a_plane (row stride lda);
// ea[i], eb[j]: the row exponents.
struct GemmSegO {
  const int8_t* a;
  const int8_t* b;
  const int32_t* ea;
  const int32_t* eb;
  int64_t a_plane, b_plane;
  int32_t lda, ldb, k, pad;
  double alpha;
};

struct GemmBatchO {
  std::vector<GemmSegO> segs;
  std::vector<GemmTileB> tiles;
  void add_problem(void* c, int ldc, int m, int n, size_t s0, size_t s1, int beta) {
    if (m <= 0 || n <= 0 || s1 <= s0) return;
    for (int r = 0; r < m; r += kOzTile)
      for (int q = 0; q < n; q += kOzTile) {
        GemmTileB t;
        t.c = c;
        t.clo = 0;
        t.ldc = ldc;
        t.m = std::min(kOzTile, m - r);
        t.n = std::min(kOzTile, n - q);
        t.row0 = r;
        t.col0 = q;
        t.seg_begin = (int32_t)s0;
        t.seg_end = (int32_t)s1;
        t.beta = beta;
        tiles.push_back(t);
      }
  }
};

struct DevGemmO {
  DevBuf buf;
  GemmSegO* segs = nullptr;
  GemmTileB* tiles = nullptr;
  size_t ntiles = 0, nsegs = 0;
};

// One operand to slice: the rows x k matrix X (element (i, kk) at
// src[kk * ld + i] if colmajor, else src[i * ld + kk]) -> digit planes at
// arena + dst + s * plane (rows of kp bytes, zero past k) and exponents at
// exps[exp + i].  row0: its first row in the slicing pass.
struct SliceOp {
  const double* src;
  int64_t dst, plane, exp, row0;
  int32_t ld, rows, k, kp, colmajor, pad;
};
__host__ __device__ inline int oz_kp(int k) { return (k + 15) & ~15; }

void launch_slice_oz(const SliceOp* ops, int nops, int64_t rows, int8_t* arena, int32_t* exps, int kappa,
                     hipStream_t s);
void upload_gemm_oz(const GemmBatchO& b, int kappa, DevGemmO& d);
void launch_gemm_oz(const DevGemmO& d, int kappa, hipStream_t s);

}  // namespace dmrg
