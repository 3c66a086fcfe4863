// gfx950 BF16 MFMA grouped GEMM for the mixed-precision sigma.
//
// Same task model as the FP64 kernel (one workgroup per output tile, a list
// of segments accumulated in registers).  Operands are BF16; with
// X3 every operand x is split as x ~ hi + lo (hi = bf16(x), lo =
// bf16(x - hi)) and the product uses hi*hi + hi*lo + lo*hi (16-bit
// effective mantissa).  The MFMAs accumulate in FP32; the FP32 tile is
// flushed into an FP64 accumulator every kFlush segments, so the sum over
// thousands of segments grows no FP32 error beyond that of kFlush of them.
// Segment scales of +-1 (all of the sigma's) are folded into the sign of
// the A fragments, so consecutive segments share the FP32 accumulator; any
// other scale gets an FP32 pass of its own, scaled at its flush.
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
// Workgroup tile BM x BN (128 x 64, 64 x 64 or 64 x 128), four waves as
// 2 x 2, each wave (BM/2) x (BN/2) in MFMA 16x16x32 blocks.  k advances in
// slabs of 32 over the concatenated segments of the tile.  Operand slabs go
// straight from global memory to LDS (global_load_lds, 16 bytes a lane, no
// register staging) through a ring of kStages buffers, so two slabs are in
// flight while the third is multiplied: enough bytes in flight to cover
// HBM latency at two workgroups per CU.
//
// LDS slab layout: rows of 32 bf16 (64 bytes), A hi | A lo | B hi | B lo.  A
// load instruction of a wave fills 1 KB = 16 rows, lane i writing bytes
// 16 i .. 16 i + 15, i.e. row i / 4, slot i % 4.  Slot s of row r holds the
// k-chunk s ^ sw(r), sw(r) = (r / 2) mod 4 (an XOR swizzle), which makes the
// 16-byte fragment reads of eight consecutive rows hit distinct banks.
// Chunks outside the operand (rows beyond the tile, k beyond its padding)
// are loaded from a zero buffer, so every address stays inside an operand
// and the padding is exactly zero.
constexpr int kBK = 32;
constexpr int kFlush = 8;  // segments accumulated in FP32 between FP64 flushes

// Per tile shape: the 64-row and 128 x 64 tiles keep an FP64 register
// accumulator (FP32 MFMA partials flushed into it every kFlush segments)
// and three LDS stages; the 128 x 128 tile gives each wave a 64 x 64 block
// (twice the operand reuse per LDS byte of a 64 x 32 block) and accumulates
// in FP32 only (its registers go to the larger block), with two LDS stages
// (two workgroups per CU) or three (one slab more in flight, one workgroup
// per CU in split-BF16x3).
// The 256 x 256 tile (FP64 output only) runs eight waves as 2 x 4, each a
// 128 x 64 block (four times the operand reuse per LDS byte of a 64 x 32
// block), FP32 accumulation, two LDS stages of 64 KB: one workgroup per CU,
// two waves per SIMD.
constexpr int waves_of(int BM, int BN) { return (BM == 256 && BN == 256) ? 8 : 4; }
template <int BM, int BN, int ST>
struct TileCfg {
  static constexpr bool ACC64 = !(BM >= 128 && BN >= 128);
  static constexpr int STAGES = ST;
  static constexpr int WAVES = waves_of(BM, BN);
  static constexpr int MIN_BLOCKS = (BM * BN <= 4096) ? 3 : ((ST == 3 && !ACC64) || WAVES == 8 ? 1 : 2);
};

__device__ __attribute__((aligned(16))) uint32_t g_zero16[4];  // 16 zero bytes (static storage)
struct __attribute__((aligned(16))) V8s { uint32_t x, y, z, w; };  // eight bf16

// Negates eight bf16 values (sign bits) when mask is 0x80008000.
__device__ __forceinline__ bf16x8 neg_if(bf16x8 x, uint32_t mask) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 u = __builtin_bit_cast(u32x4, x);
  u ^= mask;
  return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ bool unit_scale(double a) { return a == 1.0 || a == -1.0; }
__device__ __forceinline__ int swz(int row) { return (row >> 1) & 3; }

// Waits until at most n of this lane's vector memory operations are pending
// (gfx9 encoding of s_waitcnt: vmcnt low bits [3:0], high bits [15:14];
// expcnt and lgkmcnt left at their maxima, i.e. not waited for).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

template <bool X3, int BM, int BN>
struct SlabShape {
  static constexpr int NP = X3 ? 2 : 1;
  static constexpr int ROWS = NP * (BM + BN);    // 64-byte rows per slab
  static constexpr int BLOCKS = ROWS / 16;       // 1 KB load blocks per slab
  static constexpr int WAVES = waves_of(BM, BN);
  static constexpr int PER_WAVE = BLOCKS / WAVES;  // load instructions per lane
  static constexpr int ELEMS = ROWS * 32;        // bf16 per slab buffer
  static_assert(BLOCKS % WAVES == 0, "slab blocks split over the waves");
};

// Per-lane sources of the slab loads: load j of a lane covers row
// 16 (wave PER_WAVE + j) + lane / 4 of the slab and the k-chunk
// (lane % 4) ^ sw(row); base[j] points at that row and chunk of the current
// segment (k offset 0), or is null for a row outside the tile.
template <bool X3, int BM, int BN>
struct LaneLoads {
  using SS = SlabShape<X3, BM, BN>;
  const uint16_t* base[SS::PER_WAVE];
  int c8[SS::PER_WAVE];  // k offset of the lane's chunk

  __device__ __forceinline__ void segment(const GemmSegB& g, const GemmTileB& t, int wave, int lane) {
#pragma unroll
    for (int j = 0; j < SS::PER_WAVE; ++j) {
      const int rr = 16 * (wave * SS::PER_WAVE + j) + (lane >> 2);
      if (rr < SS::NP * BM) {
        const int row = rr & (BM - 1);
        c8[j] = 8 * ((lane & 3) ^ swz(row));
        base[j] = row < t.m ? g.a + (rr >= BM ? g.alo : 0) + ((int64_t)t.row0 + row) * g.lda + c8[j]
                            : nullptr;
      } else {
        const int r2 = rr - SS::NP * BM;
        const int row = r2 & (BN - 1);
        c8[j] = 8 * ((lane & 3) ^ swz(row));
        base[j] = row < t.n ? g.b + (r2 >= BN ? g.blo : 0) + ((int64_t)t.col0 + row) * g.ldb + c8[j]
                            : nullptr;
      }
    }
  }
  // Issues the loads of the slab at k offset k0 (segment padded to kpad)
  // into the buffer buf; chunks outside the operand read the zero buffer.
  __device__ __forceinline__ void issue(uint16_t* buf, int k0, int kpad, int wave) const {
    const uint16_t* zero = reinterpret_cast<const uint16_t*>(g_zero16);
#pragma unroll
    for (int j = 0; j < SS::PER_WAVE; ++j) {
      const uint16_t* src = (base[j] && k0 + c8[j] < kpad) ? base[j] + k0 : zero;
      __builtin_amdgcn_global_load_lds(src, buf + 512 * (wave * SS::PER_WAVE + j), 16, 0, 0);
    }
  }
};

__device__ __forceinline__ bf16x8 frag(const uint16_t* part, int row, int q) {
  return *reinterpret_cast<const bf16x8*>(part + row * 32 + 8 * (q ^ swz(row)));
}

template <bool X3, int OUT, int ROLE, int BM, int BN, int ST>
__global__ __launch_bounds__(64 * waves_of(BM, BN), (TileCfg<BM, BN, ST>::MIN_BLOCKS)) void k_gemm_bf16(
    const GemmTileB* __restrict__ tiles, const GemmSegB* __restrict__ segs) {
  using SS = SlabShape<X3, BM, BN>;
  using TC = TileCfg<BM, BN, ST>;
  constexpr int NP = SS::NP;
  constexpr int kStages = TC::STAGES;
  constexpr int WV = TC::WAVES;
  static_assert(WV == 4 || OUT == kOutF64, "eight-wave tiles write FP64 only");
  // waves as 2 x 2 (or 2 x 4): each wave (BM / 2) x (BN / (WV / 2)) in 16x16 blocks
  constexpr int FM = BM / 32, FN = BN / (8 * WV);
  constexpr int AM = TC::ACC64 ? FM : 1, AN = TC::ACC64 ? FN : 1;
  __shared__ __attribute__((aligned(16))) uint16_t smem[kStages][SS::ELEMS];
  const GemmTileB t = tiles[blockIdx.x];
  if (t.m <= 0) return;  // padding tile of the XCD-ordered launch
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wm = (wave / (WV / 2)) * (BM / 2), wn = (wave % (WV / 2)) * (BN / (WV / 2));
  const int lr = lane & 15, lk = lane >> 4;
  double acc[AM][AN][4];  // FP64 accumulator (ACC64 shapes only)
  f32x4 sacc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) sacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < AM; ++a)
#pragma unroll
    for (int b = 0; b < AN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][b][v] = 0.0;
  int pend = 0;  // segments held in the FP32 accumulator
  auto flush = [&](double scale) {
    if constexpr (TC::ACC64) {
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a][b][v] += scale * (double)sacc[a][b][v];
          sacc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    pend = 0;
  };
  // FP32-only shapes: a tile with one segment of scale other than +-1 is
  // scaled at the end (multi-segment tiles have +-1 scales, checked on upload)
  double fscale = 1.0;

  // A wave whose rows or columns all lie outside the tile's valid part
  // multiplies zero rows of the slab only: it skips its fragment reads and
  // MFMAs (and still loads its share of each slab)
  const bool idle = __builtin_amdgcn_readfirstlane((int)(wm >= t.m || wn >= t.n)) != 0;

  if (t.seg_begin < t.seg_end) {
    // producer cursor: next slab to load; consumer cursor: next slab to multiply
    int ps = t.seg_begin, pk0 = 0;
    GemmSegB pg = segs[ps];
    int pkpad = (pg.k + 7) & ~7;
    int cs = ps, ck0 = 0;
    GemmSegB cg = pg;
    int ckpad = pkpad;
    int issued = 0, done = 0;  // slabs
    LaneLoads<X3, BM, BN> ld;
    ld.segment(pg, t, wave, lane);
    auto produce = [&]() {
      ld.issue(&smem[issued % kStages][0], pk0, pkpad, wave);
      ++issued;
      pk0 += kBK;
      if (pk0 >= pkpad) {
        pk0 = 0;
        if (++ps < t.seg_end) {
          pg = segs[ps];
          pkpad = (pg.k + 7) & ~7;
          ld.segment(pg, t, wave, lane);
        }
      }
    };
    if constexpr (!TC::ACC64) {
      if (!unit_scale(cg.alpha)) fscale = cg.alpha;
    }
    produce();
    if (kStages == 3 && ps < t.seg_end) produce();
    while (cs < t.seg_end) {
      // slab `done` is complete once at most kStages - 2 newer slabs are pending
      if (kStages == 3 && issued > done + 1) wait_vm<SS::PER_WAVE>();
      else wait_vm<0>();
      // Workgroup barrier without a memory fence (a fence would wait for the
      // newer slabs in flight as well): after it every wave's loads of this
      // slab have landed in LDS, and every wave has consumed its fragment
      // reads of the buffer that the next load overwrites (fragments are
      // waited for before the MFMAs use them).
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      if (ps < t.seg_end) produce();
      const uint16_t* st = &smem[done % kStages][0];
      const uint16_t* Ahi = st;
      const uint16_t* Alo = st + BM * 32 * (NP - 1);
      const uint16_t* Bhi = st + NP * BM * 32;
      const uint16_t* Blo = Bhi + BN * 32 * (NP - 1);
      // MFMAs on the slab; a -1 scale flips the sign of A
      const uint32_t nmask = cg.alpha == -1.0 ? 0x80008000u : 0u;
      if (!idle) {
        bf16x8 ah[FM], bh[FN];
#pragma unroll
        for (int x = 0; x < FM; ++x) ah[x] = neg_if(frag(Ahi, wm + 16 * x + lr, lk), nmask);
#pragma unroll
        for (int x = 0; x < FN; ++x) bh[x] = frag(Bhi, wn + 16 * x + lr, lk);
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], sacc[a][b], 0, 0, 0);
        if (X3) {
          bf16x8 al[FM], bl[FN];
#pragma unroll
          for (int x = 0; x < FM; ++x) al[x] = neg_if(frag(Alo, wm + 16 * x + lr, lk), nmask);
#pragma unroll
          for (int x = 0; x < FN; ++x) bl[x] = frag(Blo, wn + 16 * x + lr, lk);
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b) {
              sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], sacc[a][b], 0, 0, 0);
              sacc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], sacc[a][b], 0, 0, 0);
            }
        }
      }
      ++done;
      ck0 += kBK;
      if (ck0 >= ckpad) {
        // segment finished
        ck0 = 0;
        const double alpha = cg.alpha;
        if constexpr (TC::ACC64) {
          if (!unit_scale(alpha)) flush(alpha);  // it had the accumulator to itself
          else if (++pend >= kFlush) flush(1.0);
        }
        if (++cs < t.seg_end) {
          cg = segs[cs];
          ckpad = (cg.k + 7) & ~7;
          if (TC::ACC64 && pend > 0 && !unit_scale(cg.alpha)) flush(1.0);
        }
      }
    }
    if (TC::ACC64 && pend > 0) flush(1.0);
  }
  // final value of accumulator element (a, b, v)
  auto value = [&](int a, int b, int v) -> double {
    if constexpr (TC::ACC64) return acc[a][b][v];
    else return fscale * (double)sacc[a][b][v];
  };

  if (OUT == kOutF64) {
    // FP64 output: sixteen lanes write 128 consecutive bytes of a row
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = wm + a * 16 + 4 * lk + v;
          const int j = wn + b * 16 + lr;
          if (i >= t.m || j >= t.n) continue;
          const int64_t idx = ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
          double* C = static_cast<double*>(t.c);
          C[idx] = t.beta ? C[idx] + value(a, b, v) : value(a, b, v);
        }
  } else {
    // BF16 hi/lo output (stage-1 intermediates): the tile is staged in LDS as
    // two planes and written with 16-byte stores (rows of the output are
    // 16-byte aligned and t.n is a multiple of 8 in the sigma layouts, which
    // the launcher checks).
    uint16_t* hi_pl = &smem[0][0];
    uint16_t* lo_pl = hi_pl + BM * BN;
    __syncthreads();  // every wave is done with the operand buffers
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = wm + a * 16 + 4 * lk + v;
          const int j = wn + b * 16 + lr;
          const double x = value(a, b, v);
          const uint16_t hi = f32_to_bf16_rn((float)x);
          hi_pl[i * BN + j] = hi;
          lo_pl[i * BN + j] = f32_to_bf16_rn((float)(x - (double)bf16_to_f32(hi)));
        }
    __syncthreads();
    uint16_t* C = static_cast<uint16_t*>(t.c);
    for (int c = tid; c < BM * BN / 8; c += 64 * WV) {
      const int i = c / (BN / 8), j = 8 * (c % (BN / 8));
      if (i >= t.m || j >= t.n) continue;
      const int64_t idx = ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
      *reinterpret_cast<V8s*>(C + idx) = *reinterpret_cast<const V8s*>(hi_pl + i * BN + j);
      *reinterpret_cast<V8s*>(C + idx + t.clo) = *reinterpret_cast<const V8s*>(lo_pl + i * BN + j);
    }
  }
}

// Every variant is instantiated explicitly: it forces both the device code
// and the host launch stub of each one into this object.
#define DMRG_INST_SHAPE(BM, BN, ST)                                                                 \
  template __global__ void k_gemm_bf16<true, kOutF64, 2, BM, BN, ST>(const GemmTileB*, const GemmSegB*);  \
  template __global__ void k_gemm_bf16<true, kOutF64, 0, BM, BN, ST>(const GemmTileB*, const GemmSegB*);  \
  template __global__ void k_gemm_bf16<true, kOutBf16, 1, BM, BN, ST>(const GemmTileB*, const GemmSegB*); \
  template __global__ void k_gemm_bf16<true, kOutBf16, 0, BM, BN, ST>(const GemmTileB*, const GemmSegB*); \
  template __global__ void k_gemm_bf16<false, kOutF64, 2, BM, BN, ST>(const GemmTileB*, const GemmSegB*); \
  template __global__ void k_gemm_bf16<false, kOutF64, 0, BM, BN, ST>(const GemmTileB*, const GemmSegB*); \
  template __global__ void k_gemm_bf16<false, kOutBf16, 1, BM, BN, ST>(const GemmTileB*, const GemmSegB*); \
  template __global__ void k_gemm_bf16<false, kOutBf16, 0, BM, BN, ST>(const GemmTileB*, const GemmSegB*);
DMRG_INST_SHAPE(128, 64, 3)
DMRG_INST_SHAPE(64, 64, 3)
DMRG_INST_SHAPE(64, 128, 3)
DMRG_INST_SHAPE(128, 128, 2)
DMRG_INST_SHAPE(128, 128, 3)
#undef DMRG_INST_SHAPE
template __global__ void k_gemm_bf16<true, kOutF64, 2, 256, 256, 2>(const GemmTileB*, const GemmSegB*);
template __global__ void k_gemm_bf16<true, kOutF64, 0, 256, 256, 2>(const GemmTileB*, const GemmSegB*);
template __global__ void k_gemm_bf16<false, kOutF64, 2, 256, 256, 2>(const GemmTileB*, const GemmSegB*);
template __global__ void k_gemm_bf16<false, kOutF64, 0, 256, 256, 2>(const GemmTileB*, const GemmSegB*);

template <int BM, int BN, int ST>
static void launch_shape(const GemmTileB* tl, unsigned cnt, const GemmSegB* sg, bool x3, int out,
                         int role, hipStream_t s) {
#define DMRG_LB(X, O, R) \
  hipLaunchKernelGGL((k_gemm_bf16<X, O, R, BM, BN, ST>), dim3(cnt), dim3(64 * waves_of(BM, BN)), 0, s, tl, sg)
  if (x3) {
    if (out == kOutF64) { if (role == 2) DMRG_LB(true, kOutF64, 2); else DMRG_LB(true, kOutF64, 0); }
    else { if (role == 1) DMRG_LB(true, kOutBf16, 1); else DMRG_LB(true, kOutBf16, 0); }
  } else {
    if (out == kOutF64) { if (role == 2) DMRG_LB(false, kOutF64, 2); else DMRG_LB(false, kOutF64, 0); }
    else { if (role == 1) DMRG_LB(false, kOutBf16, 1); else DMRG_LB(false, kOutBf16, 0); }
  }
#undef DMRG_LB
}

void launch_gemm_bf16(const DevGemmB& d, bool x3, int out, int role, hipStream_t s) {
  for (size_t off = 0; off < d.ntiles; off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(d.ntiles - off, (size_t)1 << 30);
    const GemmTileB* tl = d.tiles + off;
    switch (d.shape) {
      case kShape128x128: launch_shape<128, 128, 2>(tl, cnt, d.segs, x3, out, role, s); break;
      case kShape128x128s3: launch_shape<128, 128, 3>(tl, cnt, d.segs, x3, out, role, s); break;
      case kShape256x256:
        DMRG_REQUIRE(out == kOutF64, kErrState, "gemm_bf16: the 256 x 256 tile writes FP64 only");
        if (x3) {
          if (role == 2) hipLaunchKernelGGL((k_gemm_bf16<true, kOutF64, 2, 256, 256, 2>), dim3(cnt), dim3(512), 0, s, tl, d.segs);
          else hipLaunchKernelGGL((k_gemm_bf16<true, kOutF64, 0, 256, 256, 2>), dim3(cnt), dim3(512), 0, s, tl, d.segs);
        } else {
          if (role == 2) hipLaunchKernelGGL((k_gemm_bf16<false, kOutF64, 2, 256, 256, 2>), dim3(cnt), dim3(512), 0, s, tl, d.segs);
          else hipLaunchKernelGGL((k_gemm_bf16<false, kOutF64, 0, 256, 256, 2>), dim3(cnt), dim3(512), 0, s, tl, d.segs);
        }
        break;
      case kShape64x64: launch_shape<64, 64, 3>(tl, cnt, d.segs, x3, out, role, s); break;
      case kShape64x128: launch_shape<64, 128, 3>(tl, cnt, d.segs, x3, out, role, s); break;
      default: launch_shape<128, 64, 3>(tl, cnt, d.segs, x3, out, role, s); break;
    }
  }
  DMRG_HIP(hipGetLastError());
}

void upload_gemm_bf16(const GemmBatchB& b, DevGemmB& d) {
  if (b.shape == kShape128x128 || b.shape == kShape128x128s3 || b.shape == kShape256x256)  // FP32 accumulation: +-1 scales only
    for (const GemmTileB& t : b.tiles)
      if (t.seg_end - t.seg_begin > 1)
        for (int k = t.seg_begin; k < t.seg_end; ++k)
          DMRG_REQUIRE(b.segs[k].alpha == 1.0 || b.segs[k].alpha == -1.0, kErrState,
                       "gemm_bf16: 128x128 tiles need +-1 scales on multi-segment tiles");
  for (const GemmTileB& t : b.tiles)
    // BF16 hi/lo outputs (clo != 0) are written with 16-byte stores
    DMRG_REQUIRE(t.m <= 0 || t.clo == 0 ||
                     (t.ldc % 8 == 0 && t.clo % 8 == 0 && t.col0 % 8 == 0 && t.n % 8 == 0 &&
                      reinterpret_cast<uintptr_t>(t.c) % 16 == 0),
                 kErrState, "gemm_bf16: BF16 output tile not 16-byte aligned");
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
  d.shape = b.shape;
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
