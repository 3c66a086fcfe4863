// Repacking of FP64 operands into the BF16 hi/lo planes of the BF16 grouped
// GEMM (the mixed-precision task lists of gemm_mixed.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_bf16.h"

namespace dmrg {
namespace {

// Round-to-nearest-even FP32 -> BF16 (inf / nan pass through).
__device__ __forceinline__ uint16_t bf16_rn(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct __attribute__((aligned(16))) Chunk8 { uint32_t w[4]; };

// FP64 operands (either storage order) -> k-contiguous BF16 hi/lo planes,
// one 16-byte chunk of eight k entries per thread: hi = bf16(x),
// lo = bf16(x - hi).
__global__ void k_pack_bf16(const PackOp* __restrict__ ops, int nops, int64_t chunks, uint16_t* base) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < chunks;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nops - 1;  // last op with chunk0 <= g (ops without chunks are never picked)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ops[mid].chunk0 <= g) lo = mid; else hi = mid - 1;
    }
    const PackOp op = ops[lo];
    const int64_t c = g - op.chunk0;
    const int per_row = op.kp >> 3;
    const int i = (int)(c / per_row), k0 = 8 * (int)(c % per_row);
    Chunk8 vh, vl;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      uint16_t h[2], l[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kk = k0 + e + u;
        double x = 0.0;
        if (kk < op.k) x = op.colmajor ? op.src[(int64_t)kk * op.ld + i] : op.src[(int64_t)i * op.ld + kk];
        h[u] = bf16_rn((float)x);
        l[u] = bf16_rn((float)(x - (double)bf16_f32(h[u])));
      }
      vh.w[e >> 1] = h[0] | ((uint32_t)h[1] << 16);
      vl.w[e >> 1] = l[0] | ((uint32_t)l[1] << 16);
    }
    uint16_t* dh = base + op.dst + (int64_t)i * op.kp + k0;
    *reinterpret_cast<Chunk8*>(dh) = vh;
    *reinterpret_cast<Chunk8*>(dh + (int64_t)op.rows * op.kp) = vl;
  }
}

}  // namespace

void launch_pack_bf16(const PackOp* ops, int nops, int64_t chunks, uint16_t* base, hipStream_t s) {
  if (chunks <= 0 || nops <= 0) return;
  const int64_t g = std::max<int64_t>(1, std::min<int64_t>((chunks + 255) / 256, 16384));
  hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)g), dim3(256), 0, s, ops, nops, chunks, base);
  DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
