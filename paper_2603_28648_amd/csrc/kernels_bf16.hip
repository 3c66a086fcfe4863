// gfx950 BF16 MFMA grouped GEMM for the mixed-precision sigma.
//
// Same task model as the FP64 kernel (one workgroup per output tile, a list
// of segments accumulated in registers).  Operands are BF16; with
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

// NT products only: A row-major (m x k, row stride lda), B stored n x k (row
// stride ldb); both k-contiguous, 16-byte aligned rows with zero padding up
// to a multiple of 8 in k (the layouts of the sigma guarantee this).
//
// Workgroup tile 128 x 64, four waves as 2 x 2, each wave 64 x 32 = 4 x 2
// MFMA 16x16x32 blocks.  k advances in slabs of 32 through two LDS buffers;
// the next slab's global loads are issued before the current slab's MFMAs
// (register prefetch), so one barrier per slab suffices.
constexpr int kBM = 128, kBN = 64, kBK = 32, kBLd = kBK + 8;

struct __attribute__((aligned(16))) V8 { uint32_t x, y, z, w; };

template <bool X3>
struct SlabRegs {
  V8 a[2][X3 ? 2 : 1];  // two 16-byte vectors of A per thread (hi, lo)
  V8 b[1][X3 ? 2 : 1];  // one of B
};

__device__ __forceinline__ V8 ld16(const uint16_t* p) { return *reinterpret_cast<const V8*>(p); }

template <bool X3>
__device__ __forceinline__ void load_slab(SlabRegs<X3>& R, const GemmSegB& g, const GemmTileB& t,
                                          int k0, int kpad, int tid) {
  // A: 128 rows x 4 vectors; thread covers vectors tid and tid + 256
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int v = tid + 256 * q;
    const int row = v >> 2, kk = k0 + 8 * (v & 3);
    V8 hi{0, 0, 0, 0}, lo{0, 0, 0, 0};
    if (row < t.m && kk < kpad) {
      const int64_t idx = ((int64_t)t.row0 + row) * g.lda + kk;
      hi = ld16(g.a + idx);
      if (X3) lo = ld16(g.a + g.alo + idx);
    }
    R.a[q][0] = hi;
    if (X3) R.a[q][X3 ? 1 : 0] = lo;
  }
  {
    const int row = tid >> 2, kk = k0 + 8 * (tid & 3);
    V8 hi{0, 0, 0, 0}, lo{0, 0, 0, 0};
    if (row < t.n && kk < kpad) {
      const int64_t idx = ((int64_t)t.col0 + row) * g.ldb + kk;
      hi = ld16(g.b + idx);
      if (X3) lo = ld16(g.b + g.blo + idx);
    }
    R.b[0][0] = hi;
    if (X3) R.b[0][X3 ? 1 : 0] = lo;
  }
}

template <bool X3, int OUT, int ROLE>
__global__ __launch_bounds__(256, 2) void k_gemm_bf16(const GemmTileB* __restrict__ tiles,
                                                       const GemmSegB* __restrict__ segs) {
  constexpr int NP = X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][NP][kBM][kBLd];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NP][kBN][kBLd];
  const GemmTileB t = tiles[blockIdx.x];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  double acc[4][2][4];
  f32x4 sacc[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      sacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
    }

  int s = t.seg_begin;
  if (s < t.seg_end) {
    GemmSegB g = segs[s];
    int kpad = (g.k + 7) & ~7;
    int k0 = 0;
    SlabRegs<X3> R;
    load_slab<X3>(R, g, t, 0, kpad, tid);
    int buf = 0;
    auto store = [&](int bb) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = tid + 256 * q;
        const int row = v >> 2, kc = 8 * (v & 3);
        *reinterpret_cast<V8*>(&As[bb][0][row][kc]) = R.a[q][0];
        if (X3) *reinterpret_cast<V8*>(&As[bb][NP - 1][row][kc]) = R.a[q][NP - 1];
      }
      const int row = tid >> 2, kc = 8 * (tid & 3);
      *reinterpret_cast<V8*>(&Bs[bb][0][row][kc]) = R.b[0][0];
      if (X3) *reinterpret_cast<V8*>(&Bs[bb][NP - 1][row][kc]) = R.b[0][NP - 1];
    };
    store(0);
    __syncthreads();
    for (;;) {
      // coordinates of the next slab
      int ns = s, nk = k0 + kBK, nkpad = kpad;
      GemmSegB ng = g;
      if (nk >= kpad) {
        ns = s + 1;
        nk = 0;
        if (ns < t.seg_end) {
          ng = segs[ns];
          nkpad = (ng.k + 7) & ~7;
        }
      }
      const bool has_next = ns < t.seg_end;
      if (has_next) load_slab<X3>(R, ng, t, nk, nkpad, tid);
      // MFMAs on the current slab
      bf16x8 ah[4], bh[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) ah[x] = *reinterpret_cast<const bf16x8*>(&As[buf][0][wm + 16 * x + lr][8 * lk]);
#pragma unroll
      for (int x = 0; x < 2; ++x) bh[x] = *reinterpret_cast<const bf16x8*>(&Bs[buf][0][wn + 16 * x + lr][8 * lk]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], sacc[a][b], 0, 0, 0);
      if (X3) {
        bf16x8 al[4], bl[2];
#pragma unroll
        for (int x = 0; x < 4; ++x) al[x] = *reinterpret_cast<const bf16x8*>(&As[buf][NP - 1][wm + 16 * x + lr][8 * lk]);
#pragma unroll
        for (int x = 0; x < 2; ++x) bl[x] = *reinterpret_cast<const bf16x8*>(&Bs[buf][NP - 1][wn + 16 * x + lr][8 * lk]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], sacc[a][b], 0, 0, 0);
            sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], sacc[a][b], 0, 0, 0);
          }
      }
      if (ns != s) {
        // segment finished: scale by alpha and flush into the FP64 accumulator
        const double al = g.alpha;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[a][b][v] += al * (double)sacc[a][b][v];
            sacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
      }
      if (!has_next) break;
      store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
      s = ns;
      k0 = nk;
      g = ng;
      kpad = nkpad;
    }
  }

#pragma unroll
  for (int a = 0; a < 4; ++a)
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
