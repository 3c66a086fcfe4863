// Ozaki-scheme FP64 emulation on gfx950 INT8 MFMA (see gemm_oz.h).
//
// k_slice_oz: one workgroup per operand, each wave four rows at a time: the
// row maximum (wave reduction) gives the exponent e with |x| < (127/128) 2^e,
// so that every rounded X = round(x 2^(p - e)) has a kappa-digit signed
// base-256 expansion; the digits are written as kappa int8 planes (four
// entries a lane, one 32-bit store per plane, coalesced along k).
//
// k_gemm_oz: the task model of the other grouped GEMMs (one workgroup per
// 64 x 64 output tile, a list of segments), four waves as 2 x 2 with 32 x 32
// each in MFMA 16x16x64 INT8 blocks.  A slab holds 64 k entries of every
// digit plane of both operands (kappa (64 + 64) rows of 64 bytes), loaded
// straight into LDS (global_load_lds, 16 bytes a lane, XOR-swizzled rows,
// chunks outside the operand read a zero buffer) through three LDS stages
// (two for kappa = 7).
// Per slab and 16 x 16 block the kappa (kappa + 1) / 2 digit products with
// s + t >= kappa - 1 accumulate in INT32, one accumulator per weight s + t;
// at the end of a segment the weights are combined in FP64 (Horner in 256),
// scaled by 2^(e_i + f_j - 2p) and the segment scale, and added to an FP64
// register accumulator, which is written (or added) once per tile.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gemm_oz.h"

namespace dmrg {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));

__device__ __attribute__((aligned(16))) uint32_t g_oz_zero[4];  // 16 zero bytes

template <int N>
__device__ __forceinline__ void oz_wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
__device__ __forceinline__ int oz_swz(int row) { return (row >> 1) & 3; }
__device__ __forceinline__ i32x4 oz_frag(const int8_t* part, int row, int q) {
  return *reinterpret_cast<const i32x4*>(part + row * 64 + 16 * (q ^ oz_swz(row)));
}

// Digits of four consecutive entries (X: rounded integers) as one 32-bit
// store per plane.
__device__ __forceinline__ void oz_store_digits(int8_t* dst, int64_t plane, int kappa, int64_t X[4]) {
  for (int s = 0; s < kappa; ++s) {
    uint32_t w = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t d = ((X[u] + 128) & 255) - 128;
      w |= (uint32_t)(uint8_t)(int8_t)d << (8 * u);
      X[u] = (X[u] - d) >> 8;
    }
    *reinterpret_cast<uint32_t*>(dst + (int64_t)s * plane) = w;
  }
}

// A wave takes kRows rows at once (their loads in flight together) and holds
// up to kHeld entries of each row per lane (rows of up to 64 kHeld entries
// are read once; longer rows read their remainder twice).
constexpr int kRows = 4, kHeld = 8;

__global__ void k_slice_oz(const SliceOp* __restrict__ ops, int8_t* arena, int32_t* exps, int kappa) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int P = 8 * kappa - 1;
  const SliceOp op = ops[blockIdx.x];  // one workgroup per operand, its waves over the rows
  auto x_at = [&](int i, int kk) -> double {
    return op.colmajor ? op.src[(int64_t)kk * op.ld + i] : op.src[(int64_t)i * op.ld + kk];
  };
  // held entry q of a lane: k = 256 (q / 4) + 4 lane + q % 4
  auto k_of = [&](int q) { return 256 * (q >> 2) + 4 * lane + (q & 3); };
  for (int i0 = wave * kRows; i0 < op.rows; i0 += wpb * kRows) {
    double v[kRows][kHeld], mx[kRows];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int i = i0 + r;
      mx[r] = 0.0;
#pragma unroll
      for (int q = 0; q < kHeld; ++q) {
        const int kk = k_of(q);
        v[r][q] = (i < op.rows && kk < op.k) ? x_at(i, kk) : 0.0;
        mx[r] = fmax(mx[r], fabs(v[r][q]));
      }
      for (int kk = 64 * kHeld + lane; kk < op.k && i < op.rows; kk += 64) mx[r] = fmax(mx[r], fabs(x_at(i, kk)));
    }
#pragma unroll
    for (int r = 0; r < kRows; ++r)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) mx[r] = fmax(mx[r], __shfl_xor(mx[r], off));
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      const int i = i0 + r;
      if (i >= op.rows) break;
      // |x| <= mx < (127/128) 2^e keeps X inside the kappa-digit range
      const int e = mx[r] > 0.0 ? ilogb(mx[r] * (128.0 / 127.0)) + 1 : 0;
      if (lane == 0) exps[op.exp + i] = e;
      int8_t* row = arena + op.dst + (int64_t)i * op.kp;
#pragma unroll
      for (int h = 0; h < kHeld / 4; ++h) {
        const int k4 = 256 * h + 4 * lane;
        if (k4 >= op.kp) break;
        int64_t X[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) X[u] = (int64_t)rint(ldexp(v[r][4 * h + u], P - e));
        oz_store_digits(row + k4, op.plane, kappa, X);
      }
      for (int k4 = 64 * kHeld + 4 * lane; k4 < op.kp; k4 += 256) {
        int64_t X[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) X[u] = (int64_t)rint(ldexp(k4 + u < op.k ? x_at(i, k4 + u) : 0.0, P - e));
        oz_store_digits(row + k4, op.plane, kappa, X);
      }
    }
  }
}

template <int KAPPA>
__global__ __launch_bounds__(256, 1) void k_gemm_oz(const GemmTileB* __restrict__ tiles,
                                                    const GemmSegO* __restrict__ segs) {
  constexpr int BM = kOzTile, BN = kOzTile;
  constexpr int ROWS = KAPPA * (BM + BN);  // 64-byte rows per slab
  static_assert(ROWS % 64 == 0, "slab rows split over four waves in 16-row loads");
  constexpr int PER_WAVE = ROWS / 64;
  constexpr int BYTES = ROWS * 64;
  constexpr int ST = 3 * BYTES <= 160 * 1024 ? 3 : 2;  // LDS stages that fit
  constexpr int P = 8 * KAPPA - 1;
  __shared__ __attribute__((aligned(16))) int8_t smem[ST][BYTES];
  const GemmTileB t = tiles[blockIdx.x];
  if (t.m <= 0) return;  // padding tile of an XCD-ordered launch
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  i32x4 acc[KAPPA][2][2];  // by weight s + t - (KAPPA - 1)
  double acc64[2][2][4];
#pragma unroll
  for (int w = 0; w < KAPPA; ++w)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[w][a][b] = i32x4{0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[a][b][v] = 0.0;

  if (t.seg_begin < t.seg_end) {
    // per-lane sources: load j covers slab row 16 (wave PER_WAVE + j) + lane / 4
    const int8_t* base[PER_WAVE];
    int c16[PER_WAVE];
    auto segment = [&](const GemmSegO& g) {
#pragma unroll
      for (int j = 0; j < PER_WAVE; ++j) {
        const int rr = 16 * (wave * PER_WAVE + j) + (lane >> 2);
        if (rr < KAPPA * BM) {
          const int s = rr / BM, row = rr % BM;
          c16[j] = 16 * ((lane & 3) ^ oz_swz(row));
          base[j] = row < t.m ? g.a + s * g.a_plane + (int64_t)(t.row0 + row) * g.lda + c16[j] : nullptr;
        } else {
          const int r2 = rr - KAPPA * BM;
          const int s = r2 / BN, row = r2 % BN;
          c16[j] = 16 * ((lane & 3) ^ oz_swz(row));
          base[j] = row < t.n ? g.b + s * g.b_plane + (int64_t)(t.col0 + row) * g.ldb + c16[j] : nullptr;
        }
      }
    };
    const int8_t* zero = reinterpret_cast<const int8_t*>(g_oz_zero);
    int ps = t.seg_begin, pk0 = 0;
    GemmSegO pg = segs[ps];
    int pkpad = oz_kp(pg.k);
    segment(pg);
    int cs = ps, ck0 = 0;
    GemmSegO cg = pg;
    int ckpad = pkpad;
    int issued = 0, done = 0;
    auto produce = [&]() {
      int8_t* buf = &smem[issued % ST][0];
#pragma unroll
      for (int j = 0; j < PER_WAVE; ++j) {
        const int8_t* src = (base[j] && pk0 + c16[j] < pkpad) ? base[j] + pk0 : zero;
        __builtin_amdgcn_global_load_lds(src, buf + 1024 * (wave * PER_WAVE + j), 16, 0, 0);
      }
      ++issued;
      pk0 += kOzBK;
      if (pk0 >= pkpad) {
        pk0 = 0;
        if (++ps < t.seg_end) {
          pg = segs[ps];
          pkpad = oz_kp(pg.k);
          segment(pg);
        }
      }
    };
    produce();
    if (ST == 3 && ps < t.seg_end) produce();
    while (cs < t.seg_end) {
      // slab `done` is complete once at most ST - 2 newer slabs are pending
      if (ST == 3 && issued > done + 1) oz_wait_vm<PER_WAVE>();
      else oz_wait_vm<0>();
      // barrier without a memory fence: every wave's loads of this slab are
      // in LDS, and every wave has read the buffer the next load overwrites
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      if (ps < t.seg_end) produce();
      const int8_t* st = &smem[done % ST][0];
      i32x4 bf[KAPPA][2];
#pragma unroll
      for (int s = 0; s < KAPPA; ++s)
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[s][b] = oz_frag(st + (KAPPA * BM + s * BN) * 64, wn + 16 * b + lr, lk);
#pragma unroll
      for (int s = 0; s < KAPPA; ++s) {
        i32x4 af[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = oz_frag(st + s * BM * 64, wm + 16 * a + lr, lk);
#pragma unroll
        for (int u = KAPPA - 1 - s; u < KAPPA; ++u) {
          const int w = s + u - (KAPPA - 1);
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
              acc[w][a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a], bf[u][b], acc[w][a][b], 0, 0, 0);
        }
      }
      ++done;
      ck0 += kOzBK;
      if (ck0 >= ckpad) {
        // segment finished: combine the weights in FP64 with the row scales
        int ea[2][4], eb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = wm + 16 * a + 4 * lk + v;
            ea[a][v] = i < t.m ? cg.ea[t.row0 + i] : 0;
          }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int j = wn + 16 * b + lr;
          eb[b] = j < t.n ? cg.eb[t.col0 + j] : 0;
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              double x = 0.0;
#pragma unroll
              for (int w = KAPPA - 1; w >= 0; --w) x = x * 256.0 + (double)acc[w][a][b][v];
              acc64[a][b][v] += cg.alpha * ldexp(x, ea[a][v] + eb[b] - 2 * P + 8 * (KAPPA - 1));
            }
#pragma unroll
        for (int w = 0; w < KAPPA; ++w)
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[w][a][b] = i32x4{0, 0, 0, 0};
        ck0 = 0;
        if (++cs < t.seg_end) {
          cg = segs[cs];
          ckpad = oz_kp(cg.k);
        }
      }
    }
  }
  double* C = static_cast<double*>(t.c);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wm + 16 * a + 4 * lk + v;
        const int j = wn + 16 * b + lr;
        if (i >= t.m || j >= t.n) continue;
        const int64_t idx = ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
        C[idx] = t.beta ? C[idx] + acc64[a][b][v] : acc64[a][b][v];
      }
}

template __global__ void k_gemm_oz<3>(const GemmTileB*, const GemmSegO*);
template __global__ void k_gemm_oz<4>(const GemmTileB*, const GemmSegO*);
template __global__ void k_gemm_oz<5>(const GemmTileB*, const GemmSegO*);
template __global__ void k_gemm_oz<6>(const GemmTileB*, const GemmSegO*);
template __global__ void k_gemm_oz<7>(const GemmTileB*, const GemmSegO*);

}  // namespace

void launch_slice_oz(const SliceOp* ops, int nops, int64_t rows, int8_t* arena, int32_t* exps, int kappa,
                     hipStream_t s) {
  if (rows <= 0 || nops <= 0) return;
  DMRG_REQUIRE(kappa >= kOzMinKappa && kappa <= kOzMaxKappa, kErrInvalidArg, "slice_oz: kappa out of range");
  hipLaunchKernelGGL(k_slice_oz, dim3((unsigned)nops), dim3(256), 0, s, ops, arena, exps, kappa);
  DMRG_HIP(hipGetLastError());
}

void upload_gemm_oz(const GemmBatchO& b, int kappa, DevGemmO& d) {
  // the INT32 accumulator of one weight sums up to kappa digit products of
  // one segment: kappa * k * 2^14 < 2^31
  for (const GemmSegO& g : b.segs)
    DMRG_REQUIRE((int64_t)kappa * g.k * 16384 < ((int64_t)1 << 31), kErrShape,
                 "gemm_oz: segment k too large for exact INT32 accumulation");
  const size_t sb = b.segs.size() * sizeof(GemmSegO);
  const size_t tb = b.tiles.size() * sizeof(GemmTileB);
  const size_t sba = ((sb + 255) / 256) * 256;
  d.buf.alloc(sba + tb + 256);
  d.segs = reinterpret_cast<GemmSegO*>(d.buf.as<char>());
  d.tiles = reinterpret_cast<GemmTileB*>(d.buf.as<char>() + sba);
  if (sb) DMRG_HIP(hipMemcpy(d.segs, b.segs.data(), sb, hipMemcpyHostToDevice));
  if (tb) DMRG_HIP(hipMemcpy(d.tiles, b.tiles.data(), tb, hipMemcpyHostToDevice));
  d.ntiles = b.tiles.size();
  d.nsegs = b.segs.size();
}

void launch_gemm_oz(const DevGemmO& d, int kappa, hipStream_t s) {
  for (size_t off = 0; off < d.ntiles; off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(d.ntiles - off, (size_t)1 << 30);
    const GemmTileB* tl = d.tiles + off;
    switch (kappa) {
      case 3: hipLaunchKernelGGL(k_gemm_oz<3>, dim3(cnt), dim3(256), 0, s, tl, d.segs); break;
      case 4: hipLaunchKernelGGL(k_gemm_oz<4>, dim3(cnt), dim3(256), 0, s, tl, d.segs); break;
      case 5: hipLaunchKernelGGL(k_gemm_oz<5>, dim3(cnt), dim3(256), 0, s, tl, d.segs); break;
      case 6: hipLaunchKernelGGL(k_gemm_oz<6>, dim3(cnt), dim3(256), 0, s, tl, d.segs); break;
      case 7: hipLaunchKernelGGL(k_gemm_oz<7>, dim3(cnt), dim3(256), 0, s, tl, d.segs); break;
      default: DMRG_REQUIRE(false, kErrInvalidArg, "gemm_oz: kappa out of range");
    }
  }
  DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
