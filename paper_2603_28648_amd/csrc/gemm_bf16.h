// BF16 / split-BF16 grouped GEMM (task model of gemm.h with BF16 operands).
#pragma once
#include <cstdint>
#include <vector>

#include "gemm.h"

namespace dmrg {

enum : int { kOutBf16 = 0, kOutF64 = 1 };
// Workgroup tile shapes of the BF16 kernel (rows x columns of the output).
// kShape128x128s3: the 128 x 128 tile with three LDS stages instead of two;
// kShape256x256: eight waves, FP64 output only (sigma stage 2).
enum : int {
  kShape128x64 = 0, kShape64x64 = 1, kShape64x128 = 2, kShape128x128 = 3, kShape128x128s3 = 4,
  kShape256x256 = 5, kNumShapes = 6
};
inline int shape_rows(int s) {
  return s == kShape256x256 ? 256 : (s == kShape128x64 || s >= kShape128x128) ? 128 : 64;
}
inline int shape_cols(int s) {
  return s == kShape256x256 ? 256 : (s == kShape64x128 || s >= kShape128x128) ? 128 : 64;
}

// NT operands: A row-major m x k (stride lda), B stored n x k (stride ldb),
// rows 16-byte aligned and zero-padded in k to a multiple of 8.
struct GemmSegB {
  const uint16_t* a;  // bf16 hi; the lo part (split mode) is at a + alo
  const uint16_t* b;
  int64_t alo, blo;
  int32_t lda, ldb, k, flags;
  double alpha;
};

struct GemmTileB {
  void* c;        // FP64 (kOutF64) or bf16 hi (kOutBf16; lo at c + clo)
  int64_t clo;
  int32_t ldc, m, n, row0, col0, seg_begin, seg_end, beta;
};

struct GemmBatchB {
  std::vector<GemmSegB> segs;
  std::vector<GemmTileB> tiles;
  int shape = kShape128x64;  // tile of the NT kernel
  void add_problem(void* c, int64_t clo, int ldc, int m, int n, size_t s0, size_t s1, int beta) {
    add_region(c, clo, ldc, 0, m, 0, n, s0, s1, beta);
  }
  // Tiles over rows [r0, r1) and columns [q0, q1) of an output problem (the
  // rest of the problem is tiled by other launches).
  void add_region(void* c, int64_t clo, int ldc, int r0, int r1, int q0, int q1, size_t s0, size_t s1,
                  int beta) {
    if (r1 <= r0 || q1 <= q0 || s1 <= s0) return;
    const int TM = shape_rows(shape), TN = shape_cols(shape);
    for (int r = r0; r < r1; r += TM)
      for (int q = q0; q < q1; q += TN) {
        GemmTileB t;
        t.c = c;
        t.clo = clo;
        t.ldc = ldc;
        t.m = std::min(TM, r1 - r);
        t.n = std::min(TN, q1 - q);
        t.row0 = r;
        t.col0 = q;
        t.seg_begin = (int32_t)s0;
        t.seg_end = (int32_t)s1;
        t.beta = beta;
        tiles.push_back(t);
      }
  }
};

struct DevGemmB {
  DevBuf buf;
  GemmSegB* segs = nullptr;
  GemmTileB* tiles = nullptr;
  size_t ntiles = 0, nsegs = 0;
  int shape = kShape128x64;
};

// One operand of a repacking pass: the rows x k matrix X (element (i, kk) at
// src[kk * ld + i] if colmajor, else src[i * ld + kk]) written as BF16 hi
// (at base + dst) and lo (at base + dst + rows * kp) planes, rows of kp
// (k rounded up to 8, zero-padded) elements.  chunk0: the first of its
// rows * kp / 8 16-byte chunks in the pass.
struct PackOp {
  const double* src;
  int64_t dst, chunk0;
  int32_t ld, rows, k, kp, colmajor, pad;
};
void launch_pack_bf16(const PackOp* ops, int nops, int64_t chunks, uint16_t* base, hipStream_t s);

void upload_gemm_bf16(const GemmBatchB& b, DevGemmB& d);
void launch_gemm_bf16(const DevGemmB& d, bool x3, int out, int role, hipStream_t s);
void launch_split_bf16(uint16_t* out, const double* x, int64_t n, hipStream_t s);

// ---- FP64 task lists executed on the BF16 kernel -----------------------------
// launch_gemm runs a GemmBatch of FP64 operands (any storage order) with the
// FP64 kernel, or, inside a GemmPrecisionScope for BF16 / split-BF16x3, with
// the BF16 kernel: every distinct operand is repacked once per launch into
// k-contiguous hi/lo planes, products accumulate in FP32, are flushed into an
// FP64 register accumulator every few segments and added to the FP64 output
// (64 x 64 tiles; segment scales applied in FP64 at the flush).
struct GemmPrecisionScope {
  explicit GemmPrecisionScope(int precision);  // 0 FP64, 1 BF16, 2 split-BF16x3
  ~GemmPrecisionScope();
  GemmPrecisionScope(const GemmPrecisionScope&) = delete;
  GemmPrecisionScope& operator=(const GemmPrecisionScope&) = delete;
  int precision, prev;
  DevBuf pack, ops, desc;
  double ms_pack = 0;  // host time of the repacking passes
};
void launch_gemm(const GemmBatch& b, DevBuf& desc, hipStream_t s);

}  // namespace dmrg
