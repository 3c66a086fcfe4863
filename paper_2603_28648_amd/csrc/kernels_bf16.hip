// gfx950 BF16 MFMA grouped GEMM for the mixed-precision sigma.
//
// Same task model as the FP64 kernel (one workgroup per 64x64 output tile,
// a list of segments accumulated in registers).  Operands are BF16; with
// X3 every operand x is split as x ~ hi + lo (hi = bf16(x), lo =
// bf16(x - hi)) and the product uses hi*hi + hi*lo + lo*hi (16-bit
// effective mantissa).  Each segment is accumulated in FP32 by the MFMA
// (K of one segment is one operator block, <= a few hundred), then scaled
// by its alpha and flushed into an FP64 tile accumulator, so the sum over
// thousands of segments carries no FP32 error growth.
//
// Output modes: OUT_BF16 stores the tile as BF16 hi/lo pairs (stage-1
// intermediates), OUT_F64 adds it into an FP64 matrix (sigma).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_bf16.h"

namespace dmrg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16_rn(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan pass through
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kBK = 32;            // k per slab (one 16x16x32 MFMA)
constexpr int kBLd = kBK + 8;      // LDS row stride in bf16 (16-byte aligned, skewed)

// MFMA 16x16x32 bf16 (wave64): lane l supplies A[l%16][8*(l/16) .. +7] and
// B[8*(l/16) .. +7][l%16]; accumulator element v holds D[4*(l/16)+v][l%16].
template <bool X3, int OUT, int ROLE>
__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmTileB* __restrict__ tiles,
                                                    const GemmSegB* __restrict__ segs) {
  __shared__ __attribute__((aligned(16))) uint16_t As[X3 ? 2 : 1][kTileM][kBLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[X3 ? 2 : 1][kTileN][kBLd];
  const GemmTileB t = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  double acc[2][2][4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;

  for (int s = t.seg_begin; s < t.seg_end; ++s) {
    const GemmSegB g = segs[s];
    const bool ta = g.flags & kTransA, tb = g.flags & kTransB;
    f32x4 sacc[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) sacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.k; k0 += kBK) {
      // stage A (64 x 32) and B (32 x 64, stored [j][k]) for hi (and lo)
#pragma unroll
      for (int r = 0; r < (kTileM * kBK) / 256; ++r) {
        const int e = r * 256 + tid;
        int i, kk;
        if (!ta) { i = e / kBK; kk = e % kBK; }
        else { kk = e / kTileM; i = e % kTileM; }
        const int gk = k0 + kk;
        uint16_t hi = 0, lo = 0;
        if (i < t.m && gk < g.k) {
          const int64_t gi = (int64_t)t.row0 + i;
          const int64_t idx = ta ? (int64_t)gk * g.lda + gi : gi * g.lda + gk;
          hi = g.a[idx];
          if (X3) lo = g.a[idx + g.alo];
        }
        As[0][i][kk] = hi;
        if (X3) As[X3 ? 1 : 0][i][kk] = lo;
      }
#pragma unroll
      for (int r = 0; r < (kTileN * kBK) / 256; ++r) {
        const int e = r * 256 + tid;
        int j, kk;
        if (!tb) { kk = e / kTileN; j = e % kTileN; }
        else { j = e / kBK; kk = e % kBK; }
        const int gk = k0 + kk;
        uint16_t hi = 0, lo = 0;
        if (j < t.n && gk < g.k) {
          const int64_t gj = (int64_t)t.col0 + j;
          const int64_t idx = tb ? gj * g.ldb + gk : (int64_t)gk * g.ldb + gj;
          hi = g.b[idx];
          if (X3) lo = g.b[idx + g.blo];
        }
        Bs[0][j][kk] = hi;
        if (X3) Bs[X3 ? 1 : 0][j][kk] = lo;
      }
      __syncthreads();
      bf16x8 ah[2], bh[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ah[x] = *reinterpret_cast<const bf16x8*>(&As[0][wm + 16 * x + lr][8 * lk]);
        bh[x] = *reinterpret_cast<const bf16x8*>(&Bs[0][wn + 16 * x + lr][8 * lk]);
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], sacc[a][b], 0, 0, 0);
      if (X3) {
        bf16x8 al[2], bl[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          al[x] = *reinterpret_cast<const bf16x8*>(&As[X3 ? 1 : 0][wm + 16 * x + lr][8 * lk]);
          bl[x] = *reinterpret_cast<const bf16x8*>(&Bs[X3 ? 1 : 0][wn + 16 * x + lr][8 * lk]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], sacc[a][b], 0, 0, 0);
            sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], sacc[a][b], 0, 0, 0);
          }
      }
      __syncthreads();
    }
    const double al = g.alpha;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][b][v] += al * (double)sacc[a][b][v];
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wm + a * 16 + 4 * lk + v;
        const int j = wn + b * 16 + lr;
        if (i >= t.m || j >= t.n) continue;
        const int64_t idx = ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
        if (OUT == kOutF64) {
          double* C = static_cast<double*>(t.c);
          C[idx] = t.beta ? C[idx] + acc[a][b][v] : acc[a][b][v];
        } else {
          uint16_t* C = static_cast<uint16_t*>(t.c);
          const double x = acc[a][b][v];
          const uint16_t hi = f32_to_bf16_rn((float)x);
          C[idx] = hi;
          C[idx + t.clo] = f32_to_bf16_rn((float)(x - (double)bf16_to_f32(hi)));
        }
      }
}

void launch_gemm_bf16(const DevGemmB& d, bool x3, int out, int role, hipStream_t s) {
  for (size_t off = 0; off < d.ntiles; off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(d.ntiles - off, (size_t)1 << 30);
    const GemmTileB* tl = d.tiles + off;
#define DMRG_LB(X, O, R) hipLaunchKernelGGL((k_gemm_bf16<X, O, R>), dim3(cnt), dim3(256), 0, s, tl, d.segs)
    if (x3) {
      if (out == kOutF64) { if (role == 2) DMRG_LB(true, kOutF64, 2); else DMRG_LB(true, kOutF64, 0); }
      else { if (role == 1) DMRG_LB(true, kOutBf16, 1); else DMRG_LB(true, kOutBf16, 0); }
    } else {
      if (out == kOutF64) { if (role == 2) DMRG_LB(false, kOutF64, 2); else DMRG_LB(false, kOutF64, 0); }
      else { if (role == 1) DMRG_LB(false, kOutBf16, 1); else DMRG_LB(false, kOutBf16, 0); }
    }
#undef DMRG_LB
  }
  DMRG_HIP(hipGetLastError());
}

void upload_gemm_bf16(const GemmBatchB& b, DevGemmB& d) {
  const size_t sb = b.segs.size() * sizeof(GemmSegB);
  const size_t tb = b.tiles.size() * sizeof(GemmTileB);
  const size_t sba = ((sb + 255) / 256) * 256;
  d.buf.alloc(sba + tb + 256);
  d.segs = reinterpret_cast<GemmSegB*>(d.buf.as<char>());
  d.tiles = reinterpret_cast<GemmTileB*>(d.buf.as<char>() + sba);
  if (sb) DMRG_HIP(hipMemcpy(d.segs, b.segs.data(), sb, hipMemcpyHostToDevice));
  if (tb) DMRG_HIP(hipMemcpy(d.tiles, b.tiles.data(), tb, hipMemcpyHostToDevice));
  d.ntiles = b.tiles.size();
  d.nsegs = b.segs.size();
}

// x (FP64) -> hi = bf16(x), lo = bf16(x - hi); lo stored at hi + n.
__global__ void k_split_bf16(uint16_t* out, const double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    const uint16_t hi = f32_to_bf16_rn((float)v);
    out[i] = hi;
    out[i + n] = f32_to_bf16_rn((float)(v - (double)bf16_to_f32(hi)));
  }
}
void launch_split_bf16(uint16_t* out, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t g = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
  hipLaunchKernelGGL(k_split_bf16, dim3((unsigned)g), dim3(256), 0, s, out, x, n);
  DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
