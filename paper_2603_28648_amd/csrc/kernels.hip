// gfx950 kernels: FP64-MFMA grouped GEMM and FP64 BLAS-1 helpers.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <map>

#include <algorithm>

#include "gemm.h"
#include "davidson.h"
#include "engine.h"

namespace dmrg {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// One workgroup per TM x TN output tile: 64 x 64 with 4 waves (each a
// 32 x 32 quarter as 2 x 2 blocks of v_mfma_f64_16x16x4f64), 128 x 128 with
// 8 waves (each 64 x 32 as 4 x 2 blocks; twice the operand reuse per loaded
// byte), or 128 x 64 / 64 x 128 with 8 waves of 32 x 32 (4/3 of the reuse at
// the register count of the 64 x 64 tile).
// Operands are staged through LDS in k-slabs of 16 with bounds-checked
// (zero-filled) loads, so ragged m, n, k need no padding in memory.  alpha is
// folded into A.  The slabs of all segments of a tile form one sequence,
// double-buffered: the global loads of the next slab are issued into
// registers before the MFMAs of the current one, then stored into the other
// LDS buffer (one barrier per slab).
//
// MFMA operand layout (16x16x4 f64, wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator element v of lane l holds D[4*v + l/16][l%16]
// (rows interleaved across the four 16-lane groups).
constexpr int kTK = 16;
constexpr int f64_waves(int TM, int TN) { return TM == 64 && TN == 64 ? 4 : 8; }
constexpr int f64_wave_rows(int TM, int TN) { return TM == 128 && TN == 64 ? 4 : 2; }

// ROLE only names the kernel for profilers: 0 = operator construction,
// 1 = sigma stage 1 (psi x right operator), 2 = sigma stage 2 (left operator x T).
template <int ROLE, int TM, int TN>
__global__ __launch_bounds__(64 * f64_waves(TM, TN)) void k_gemm_f64(const GemmTile* __restrict__ tiles,
                                                                     const GemmSeg* __restrict__ segs) {
  constexpr int WV = f64_waves(TM, TN), NT = 64 * WV;
  constexpr int WR = f64_wave_rows(TM, TN), WC = WV / WR;  // waves down the rows / across the columns
  constexpr int FM = TM / (16 * WR), FN = TN / (16 * WC);  // 16x16 blocks of a wave
  constexpr int kLoadsA = (TM * kTK) / NT, kLoadsB = (TN * kTK) / NT;
  static_assert(FM >= 1 && FN >= 1 && kLoadsA >= 1 && kLoadsB >= 1, "k_gemm_f64: tile shape");
  __shared__ double As[2][kTK][TM + 1];
  __shared__ double Bs[2][kTK][TN + 1];
  const GemmTile t = tiles[blockIdx.x];
  if (t.m <= 0) return;  // padding tile of the XCD-ordered launch
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wm = (wave / WC) * (TM / WR), wn = (wave % WC) * (TN / WC);
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  if (t.seg_begin < t.seg_end) {
    double ra[kLoadsA], rb[kLoadsB];
    // global loads of the slab at k offset k0 of segment g into ra, rb
    auto load = [&](const GemmSeg& g, int k0) {
      const double* __restrict__ A = static_cast<const double*>(g.a);
      const double* __restrict__ B = static_cast<const double*>(g.b);
      const bool ta = g.flags & kTransA, tb = g.flags & kTransB;
#pragma unroll
      for (int r = 0; r < kLoadsA; ++r) {
        const int e = r * NT + tid;
        int i, kk;
        if (!ta) { i = e / kTK; kk = e % kTK; }
        else { kk = e / TM; i = e % TM; }
        const int gk = k0 + kk;
        double v = 0.0;
        if (i < t.m && gk < g.k) {
          const int64_t gi = (int64_t)t.row0 + i;
          v = ta ? A[(int64_t)gk * g.lda + gi] : A[gi * g.lda + gk];
        }
        ra[r] = v * g.alpha;
      }
#pragma unroll
      for (int r = 0; r < kLoadsB; ++r) {
        const int e = r * NT + tid;
        int j, kk;
        if (!tb) { kk = e / TN; j = e % TN; }
        else { j = e / kTK; kk = e % kTK; }
        const int gk = k0 + kk;
        double v = 0.0;
        if (j < t.n && gk < g.k) {
          const int64_t gj = (int64_t)t.col0 + j;
          v = tb ? B[gj * g.ldb + gk] : B[(int64_t)gk * g.ldb + gj];
        }
        rb[r] = v;
      }
    };
    // ra, rb into LDS buffer buf (same element placement as the loads)
    auto store = [&](const GemmSeg& g, int buf) {
      const bool ta = g.flags & kTransA, tb = g.flags & kTransB;
#pragma unroll
      for (int r = 0; r < kLoadsA; ++r) {
        const int e = r * NT + tid;
        if (!ta) As[buf][e % kTK][e / kTK] = ra[r];
        else As[buf][e / TM][e % TM] = ra[r];
      }
#pragma unroll
      for (int r = 0; r < kLoadsB; ++r) {
        const int e = r * NT + tid;
        if (!tb) Bs[buf][e / TN][e % TN] = rb[r];
        else Bs[buf][e % kTK][e / kTK] = rb[r];
      }
    };
    int s = t.seg_begin, k0 = 0, buf = 0;
    GemmSeg g = segs[s];
    load(g, 0);
    store(g, 0);
    __syncthreads();
    while (true) {
      // position of the next slab in the tile's sequence
      int ns = s, nk0 = k0 + kTK;
      GemmSeg ng = g;
      if (nk0 >= g.k) {
        nk0 = 0;
        if (++ns < t.seg_end) ng = segs[ns];
      }
      const bool more = ns < t.seg_end;
      if (more) load(ng, nk0);  // in flight during the MFMAs below
      // MFMAs only on 16x16 blocks and k-steps of 4 that meet the tile's
      // valid rows, columns and the segment's k (the rest of the LDS slab is
      // zero padding); the conditions are uniform over the wave, so the
      // skipped MFMAs leave the SIMD's matrix pipe to the other waves
      if (wm < t.m && wn < t.n) {
        const int kv = g.k - k0;  // valid k of this slab (>= 1)
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 4) {
          if (kk >= kv) break;
          double a[FM], b[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) a[i] = As[buf][kk + lk][wm + 16 * i + lr];
#pragma unroll
          for (int j = 0; j < FN; ++j) b[j] = Bs[buf][kk + lk][wn + 16 * j + lr];
#pragma unroll
          for (int i = 0; i < FM; ++i)
            if (wm + 16 * i < t.m)
#pragma unroll
              for (int j = 0; j < FN; ++j)
                if (wn + 16 * j < t.n)
                  acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
      if (!more) break;
      // the other buffer was last read before the previous barrier
      store(ng, buf ^ 1);
      __syncthreads();
      buf ^= 1;
      s = ns;
      k0 = nk0;
      g = ng;
    }
  }
  double* __restrict__ C = static_cast<double*>(t.c);
#pragma unroll
  for (int bi = 0; bi < FM; ++bi)
#pragma unroll
    for (int bj = 0; bj < FN; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wm + bi * 16 + 4 * v + lk;
        const int j = wn + bj * 16 + lr;
        if (i < t.m && j < t.n) {
          double* p = C + ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
          const double val = acc[bi][bj][v];
          *p = t.beta ? (*p + val) : val;
        }
      }
}

// Direct-to-LDS variant for NT segments (A m x k and B stored n x k, both k
// contiguous, with even leading dimensions and 16-byte aligned bases, so
// that every 16-byte chunk of a row lies inside the row).  Each lane moves 16
// bytes of a slab from global memory straight into LDS (global_load_lds): no
// registers stage the operands, and a ring of three LDS stages keeps two
// slabs in flight during the MFMAs of a third (two stages for 128 x 128, so
// that two workgroups fit a CU).  A slab holds kTK = 16 k of
// the TM rows of A and the TN rows of B, 128 bytes a row; chunk c (k 2c,
// 2c + 1) of LDS row r sits at position c ^ ((r >> 1) & 7), so that the
// fragment reads of 16 consecutive rows at one k (half a wave) meet each
// bank once.  Chunks outside the operands read a zero buffer; k entries past
// a segment's k that share a chunk with valid ones are zeroed in the
// fragments, and alpha scales the A fragments.  The MFMA sequence (k-steps of
// 4, segment by segment) is that of k_gemm_f64, so both give the same bits.
__device__ __attribute__((aligned(16))) double g_f64_zero[2];  // 16 zero bytes (static storage)

template <int N>
__device__ __forceinline__ void f64_wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  // gfx9 encoding of s_waitcnt: vmcnt low bits [3:0], high bits [15:14];
  // expcnt and lgkmcnt at their maxima (not waited on)
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
__device__ __forceinline__ int f64_swz(int row) { return (row >> 1) & 7; }

template <int ROLE, int TM, int TN>
__global__ __launch_bounds__(64 * f64_waves(TM, TN)) void k_gemm_f64_lds(const GemmTile* __restrict__ tiles,
                                                                         const GemmSeg* __restrict__ segs) {
  constexpr int WV = f64_waves(TM, TN);
  constexpr int WR = f64_wave_rows(TM, TN), WC = WV / WR;
  constexpr int FM = TM / (16 * WR), FN = TN / (16 * WC);
  constexpr int ROWS = TM + TN;        // 128-byte LDS rows of a slab
  constexpr int NL = ROWS / (8 * WV);  // wave loads (8 rows each) per wave and slab
  static_assert(NL >= 1 && NL * 8 * WV == ROWS && kTK == 16, "k_gemm_f64_lds: slab layout");
  // three LDS stages where two workgroups still fit a CU, else two
  constexpr int ST = 3 * ROWS * kTK * 8 <= 80 * 1024 ? 3 : 2;
  __shared__ __attribute__((aligned(16))) double sm[ST][ROWS * kTK];
  const GemmTile t = tiles[blockIdx.x];
  if (t.m <= 0) return;  // padding tile of the XCD-ordered launch
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int wm = (wave / WC) * (TM / WR), wn = (wave % WC) * (TN / WC);
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  if (t.seg_begin < t.seg_end) {
    // load j of a lane: LDS row 8 (wave NL + j) + lane / 8, position lane % 8
    const double* src[NL];
    int kc[NL];
    auto segment = [&](const GemmSeg& g) {
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const int r = 8 * (wave * NL + j) + (lane >> 3);
        const int c = (lane & 7) ^ f64_swz(r);
        kc[j] = 2 * c;
        if (r < TM)
          src[j] = r < t.m ? static_cast<const double*>(g.a) + (int64_t)(t.row0 + r) * g.lda + 2 * c : nullptr;
        else
          src[j] = r - TM < t.n ? static_cast<const double*>(g.b) + (int64_t)(t.col0 + r - TM) * g.ldb + 2 * c
                                : nullptr;
      }
    };
    int ps = t.seg_begin, pk0 = 0;
    GemmSeg pg = segs[ps];
    segment(pg);
    int cs = ps, ck0 = 0;
    GemmSeg cg = pg;
    int issued = 0, done = 0;
    auto produce = [&]() {
      double* buf = &sm[issued % ST][0];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const double* p = (src[j] && pk0 + kc[j] < pg.k) ? src[j] + pk0 : g_f64_zero;
        __builtin_amdgcn_global_load_lds(p, buf + 128 * (wave * NL + j), 16, 0, 0);
      }
      ++issued;
      pk0 += kTK;
      if (pk0 >= pg.k) {
        pk0 = 0;
        if (++ps < t.seg_end) {
          pg = segs[ps];
          segment(pg);
        }
      }
    };
    produce();
    if (ST == 3 && ps < t.seg_end) produce();
    while (cs < t.seg_end) {
      // slab `done` is complete once at most ST - 2 newer slabs are pending
      if (ST == 3 && issued > done + 1) f64_wait_vm<NL>();
      else f64_wait_vm<0>();
      // barrier without a memory fence: every wave's loads of this slab are
      // in LDS, and every wave has read the buffer the next load overwrites
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
      if (ps < t.seg_end) produce();
      const double* st = &sm[done % ST][0];
      if (wm < t.m && wn < t.n) {
        const int kv = cg.k - ck0;  // valid k of this slab
#pragma unroll
        for (int kk = 0; kk < kTK; kk += 4) {
          if (kk >= kv) break;
          const int k = kk + lk, c = k >> 1, h = k & 1;
          double a[FM], b[FN];
#pragma unroll
          for (int i = 0; i < FM; ++i) {
            const int r = wm + 16 * i + lr;
            a[i] = st[r * kTK + 2 * (c ^ f64_swz(r)) + h];
          }
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            const int r = TM + wn + 16 * j + lr;
            b[j] = st[r * kTK + 2 * (c ^ f64_swz(r)) + h];
          }
          if (kv - kk < 4) {  // the segment's last k-step: entries past k are zero
            const bool ok = k < kv;
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = ok ? a[i] : 0.0;
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = ok ? b[j] : 0.0;
          }
#pragma unroll
          for (int i = 0; i < FM; ++i) a[i] *= cg.alpha;
#pragma unroll
          for (int i = 0; i < FM; ++i)
            if (wm + 16 * i < t.m)
#pragma unroll
              for (int j = 0; j < FN; ++j)
                if (wn + 16 * j < t.n)
                  acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
      }
      ++done;
      ck0 += kTK;
      if (ck0 >= cg.k) {
        ck0 = 0;
        if (++cs < t.seg_end) cg = segs[cs];
      }
    }
  }
  double* __restrict__ C = static_cast<double*>(t.c);
#pragma unroll
  for (int bi = 0; bi < FM; ++bi)
#pragma unroll
    for (int bj = 0; bj < FN; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wm + bi * 16 + 4 * v + lk;
        const int j = wn + bj * 16 + lr;
        if (i < t.m && j < t.n) {
          double* p = C + ((int64_t)t.row0 + i) * t.ldc + (t.col0 + j);
          const double val = acc[bi][bj][v];
          *p = t.beta ? (*p + val) : val;
        }
      }
}

// Whether every segment of a launch suits k_gemm_f64_lds: NT operands with
// even leading dimensions and 16-byte aligned bases.  DMRG_F64_LDS=0 keeps
// every launch on k_gemm_f64.
static bool f64_lds_ok(const GemmSeg* segs, size_t n) {
  const char* e = std::getenv("DMRG_F64_LDS");
  if (e && std::atoi(e) == 0) return false;
  for (size_t i = 0; i < n; ++i) {
    const GemmSeg& g = segs[i];
    if ((g.flags & kTransA) || !(g.flags & kTransB) || (g.lda & 1) || (g.ldb & 1) ||
        (reinterpret_cast<uintptr_t>(g.a) & 15) || (reinterpret_cast<uintptr_t>(g.b) & 15))
      return false;
  }
  return true;
}

// One launch of cnt tiles of the given shape (rows x cols) and role.
static void launch_f64_tiles(int role, int tm, int tn, bool lds, unsigned cnt, hipStream_t s, const GemmTile* tiles,
                             const GemmSeg* segs) {
#define DMRG_LF(R, TM, TN)                                                                                       \
  do {                                                                                                          \
    if (lds)                                                                                                    \
      hipLaunchKernelGGL((k_gemm_f64_lds<R, TM, TN>), dim3(cnt), dim3(64 * f64_waves(TM, TN)), 0, s, tiles, segs); \
    else                                                                                                        \
      hipLaunchKernelGGL((k_gemm_f64<R, TM, TN>), dim3(cnt), dim3(64 * f64_waves(TM, TN)), 0, s, tiles, segs);     \
  } while (0)
#define DMRG_LF_ROLES(TM, TN)               \
  do {                                      \
    if (role == 1) DMRG_LF(1, TM, TN);      \
    else if (role == 2) DMRG_LF(2, TM, TN); \
    else DMRG_LF(0, TM, TN);                \
  } while (0)
  if (tm == 128 && tn == 128) DMRG_LF_ROLES(128, 128);
  else if (tm == 128 && tn == 64) DMRG_LF_ROLES(128, 64);
  else if (tm == 64 && tn == 128) DMRG_LF_ROLES(64, 128);
  else {
    DMRG_REQUIRE(tm == 64 && tn == 64, kErrInvalidArg, "k_gemm_f64: tile must be 64x64, 128x128, 128x64 or 64x128");
    DMRG_LF_ROLES(64, 64);
  }
#undef DMRG_LF_ROLES
#undef DMRG_LF
}

// Descriptors of one-off launches go through a ring of pinned host buffers
// copied asynchronously to device buffers, so that a launch needs no host
// synchronisation: a slot is reused only after the event recorded behind
// the launch that read it has completed.  One ring per device and host
// thread, kept until the process ends.
namespace {
struct DescSlot {
  char* host = nullptr;
  DevBuf dev;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool used = false;
};
constexpr int kDescSlots = 8;
struct DescRing {
  DescSlot slot[kDescSlots];
  int next = 0;
};
DescRing& desc_ring() {
  static thread_local std::map<int, DescRing*> rings;
  int dev = 0;
  DMRG_HIP(hipGetDevice(&dev));
  DescRing*& r = rings[dev];
  if (!r) r = new DescRing();  // process lifetime
  return *r;
}
}  // namespace

void launch_gemm_f64(const GemmBatch& b, hipStream_t stream) {
  if (b.tiles.empty()) return;
  const size_t sb = b.segs.size() * sizeof(GemmSeg);
  const size_t sba = ((sb + 255) / 256) * 256;
  const size_t tb = b.tiles.size() * sizeof(GemmTile);
  const size_t need = sba + tb;
  DescRing& ring = desc_ring();
  DescSlot& sl = ring.slot[ring.next];
  ring.next = (ring.next + 1) % kDescSlots;
  if (sl.used) DMRG_HIP(hipEventSynchronize(sl.ev));
  if (!sl.ev) DMRG_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  if (sl.cap < need) {
    const size_t cap = std::max(need, (size_t)1 << 16);
    if (sl.host) DMRG_HIP(hipHostFree(sl.host));
    sl.host = nullptr;
    DMRG_HIP(hipHostMalloc(reinterpret_cast<void**>(&sl.host), cap));
    sl.dev.alloc(cap);
    sl.cap = cap;
  }
  std::memcpy(sl.host, b.segs.data(), sb);
  std::memcpy(sl.host + sba, b.tiles.data(), tb);
  DMRG_HIP(hipMemcpyAsync(sl.dev.p, sl.host, need, hipMemcpyHostToDevice, stream));
  GemmSeg* dsegs = sl.dev.as<GemmSeg>();
  GemmTile* dtiles = reinterpret_cast<GemmTile*>(sl.dev.as<char>() + sba);
  const size_t nt = b.tiles.size();
  const bool lds = f64_lds_ok(b.segs.data(), b.segs.size());
  for (size_t off = 0; off < nt; off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(nt - off, (size_t)1 << 30);
    launch_f64_tiles(0, b.tile, b.tile_n, lds, cnt, stream, dtiles + off, dsegs);
  }
  DMRG_HIP(hipGetLastError());
  DMRG_HIP(hipEventRecord(sl.ev, stream));
  sl.used = true;
}

void upload_gemm(const GemmBatch& b, DevGemm& d) {
  const size_t sb = b.segs.size() * sizeof(GemmSeg);
  const size_t tb = b.tiles.size() * sizeof(GemmTile);
  const size_t sba = ((sb + 255) / 256) * 256;
  d.buf.alloc(sba + tb + 256);
  d.segs = reinterpret_cast<GemmSeg*>(d.buf.as<char>());
  d.tiles = reinterpret_cast<GemmTile*>(d.buf.as<char>() + sba);
  if (sb) DMRG_HIP(hipMemcpy(d.segs, b.segs.data(), sb, hipMemcpyHostToDevice));
  if (tb) DMRG_HIP(hipMemcpy(d.tiles, b.tiles.data(), tb, hipMemcpyHostToDevice));
  d.ntiles = b.tiles.size();
  d.nsegs = b.segs.size();
  d.flops = b.flops;
  d.tile = b.tile;
  d.tile_n = b.tile_n;
  d.lds = f64_lds_ok(b.segs.data(), b.segs.size());
}

void launch_gemm_f64(const DevGemm& d, hipStream_t stream, int role) {
  for (size_t off = 0; off < d.ntiles; off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(d.ntiles - off, (size_t)1 << 30);
    launch_f64_tiles(role, d.tile, d.tile_n, d.lds, cnt, stream, d.tiles + off, d.segs);
  }
  DMRG_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
__global__ void k_scale(double* x, double a, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= a;
}
__global__ void k_axpy(double* y, double a, const double* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}
__global__ void k_axpby(double* z, double a, const double* x, double b, const double* y,
                        int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    z[i] = a * x[i] + b * y[i];
}
__global__ void k_fill(double* x, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

static unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

void launch_scale(double* x, double a, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, s, x, a, n);
  DMRG_HIP(hipGetLastError());
}
void launch_axpy(double* y, double a, const double* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, y, a, x, n);
  DMRG_HIP(hipGetLastError());
}
void launch_axpby(double* z, double a, const double* x, double b, const double* y, int64_t n,
                  hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, s, z, a, x, b, y, n);
  DMRG_HIP(hipGetLastError());
}
void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, x, v, n);
  DMRG_HIP(hipGetLastError());
}

// Deterministic two-pass dot products: block partials, then one block per row.
constexpr int kDotBlocks = 512;
__global__ __launch_bounds__(256) void k_multidot_partial(double* part, const double* X,
                                                          int64_t ldx, const double* y,
                                                          int64_t n) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const double* x = X + j * ldx;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += x[i] * y[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void k_reduce_rows(double* out, const double* part, int nb) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[(int64_t)j * nb + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

void launch_multidot(double* out, const double* X, int64_t ldx, int nv, const double* y,
                     int64_t n, hipStream_t s) {
  if (nv <= 0) return;
  static thread_local DevBuf part;
  const size_t need = (size_t)nv * kDotBlocks * sizeof(double);
  if (part.bytes < need) {
    DMRG_HIP(hipStreamSynchronize(s));
    part.alloc(need);
  }
  int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (n + 255) / 256));
  hipLaunchKernelGGL(k_multidot_partial, dim3(nb, nv), dim3(256), 0, s, part.as<double>(), X,
                     ldx, y, n);
  hipLaunchKernelGGL(k_reduce_rows, dim3(nv), dim3(256), 0, s, out, part.as<double>(), nb);
  DMRG_HIP(hipGetLastError());
}

__global__ void k_lincomb(double* y, const double* X, int64_t ldx, int nv, const double* c,
                          int64_t n, double beta) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = beta == 0.0 ? 0.0 : beta * y[i];
    for (int j = 0; j < nv; ++j) acc += c[j] * X[j * ldx + i];
    y[i] = acc;
  }
}
void launch_lincomb(double* y, const double* X, int64_t ldx, int nv, const double* c,
                    int64_t n, double beta, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, s, y, X, ldx, nv, c, n, beta);
  DMRG_HIP(hipGetLastError());
}

__global__ void k_row_scatter_add(double* dst, const double* src, const int64_t* off, int64_t n) {
  const int r = blockIdx.y;
  double* d = dst + off[r];
  const double* x = src + (int64_t)r * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] += x[i];
}
void launch_row_scatter_add(double* dst, const double* src, const int64_t* dst_off, int nrows,
                            int64_t n, hipStream_t s) {
  if (nrows <= 0 || n <= 0) return;
  unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 64));
  hipLaunchKernelGGL(k_row_scatter_add, dim3(gx, nrows), dim3(256), 0, s, dst, src, dst_off, n);
  DMRG_HIP(hipGetLastError());
}

__global__ void k_copy_tasks(const CopyTask* tasks, int transpose) {
  const CopyTask t = tasks[blockIdx.x];
  const int64_t n = (int64_t)t.rows * t.cols;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = (int)(e / t.cols), c = (int)(e % t.cols);
    if (transpose) t.dst[(int64_t)c * t.dld + r] = t.src[(int64_t)r * t.sld + c];
    else t.dst[(int64_t)r * t.dld + c] = t.src[(int64_t)r * t.sld + c];
  }
}
void launch_copy_tasks(const CopyTask* tasks, int ntasks, bool transpose, hipStream_t s) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_copy_tasks, dim3(ntasks), dim3(256), 0, s, tasks, (int)transpose);
  DMRG_HIP(hipGetLastError());
}

// ---- Davidson helpers --------------------------------------------------------
__global__ void k_extract_diag(const DiagTask* tasks) {
  const DiagTask t = tasks[blockIdx.x];
  for (int i = threadIdx.x; i < t.d; i += blockDim.x) t.dst[i] = t.src[(int64_t)i * (t.ld + 1)];
}
void launch_extract_diag(const DiagTask* tasks, int ntasks, hipStream_t s) {
  for (int off = 0; off < ntasks; off += 1 << 30) {
    const int cnt = std::min(ntasks - off, 1 << 30);
    hipLaunchKernelGGL(k_extract_diag, dim3(cnt), dim3(64), 0, s, tasks + off);
  }
  DMRG_HIP(hipGetLastError());
}

// diag[row][col] = sum_p yd[p][n(row)] * Ld[p][aL(row)] * Zd[p][offR + col]
__global__ __launch_bounds__(256) void k_heff_diag(double* out, int64_t rows, int dr,
                                                   const int64_t* rowinfo, int64_t offR,
                                                   int npairs, const double* yd,
                                                   const double* Ld, int64_t DL,
                                                   const double* Zd, int64_t DR) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= rows * dr) return;
  const int64_t row = e / dr;
  const int col = (int)(e % dr);
  const int64_t aL = rowinfo[2 * row];
  const int n = (int)rowinfo[2 * row + 1];
  double acc = 0.0;
  for (int p = 0; p < npairs; ++p)
    acc += yd[p * 16 + n] * Ld[p * DL + aL] * Zd[p * DR + offR + col];
  out[e] = acc;
}
void launch_heff_diag(double* out, int64_t rows, int dr, const int64_t* rowinfo, int64_t offR,
                      int npairs, const double* yd, const double* Ld, int64_t DL,
                      const double* Zd, int64_t DR, hipStream_t s) {
  const int64_t n = rows * dr;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_heff_diag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, rows, dr,
                     rowinfo, offR, npairs, yd, Ld, DL, Zd, DR);
  DMRG_HIP(hipGetLastError());
}

// t = r / (theta - d), the denominator clamped to |.| >= 1e-8 keeping its sign
__global__ void k_precondition(double* t, const double* r, const double* d, double theta,
                               int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double den = theta - d[i];
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    t[i] = r[i] / den;
  }
}
void launch_precondition(double* t, const double* r, const double* d, double theta, int64_t n,
                         hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_precondition, dim3(grid_for(n)), dim3(256), 0, s, t, r, d, theta, n);
  DMRG_HIP(hipGetLastError());
}

}  // namespace dmrg
