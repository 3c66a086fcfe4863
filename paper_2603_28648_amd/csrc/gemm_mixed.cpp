// FP64 grouped-GEMM task lists run on the BF16 kernel (see gemm_bf16.h).
#include <map>
#include <tuple>

#include "gemm_bf16.h"

namespace dmrg {
namespace {
thread_local GemmPrecisionScope* g_scope = nullptr;

void grow_buf(DevBuf& b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return;
  DMRG_HIP(hipStreamSynchronize(s));
  b.alloc(bytes);
}

void launch_gemm_lowp(const GemmBatch& b, GemmPrecisionScope& sc, hipStream_t s) {
  // output problems: tiles sharing (c, segment range), extents from the tiles
  struct Prob {
    void* c;
    int ldc, m = 0, n = 0, beta;
    int32_t s0, s1;
  };
  std::vector<Prob> probs;
  std::map<std::tuple<void*, int32_t, int32_t>, size_t> pidx;
  for (const GemmTile& t : b.tiles) {
    if (t.m <= 0) continue;
    auto key = std::make_tuple(t.c, t.seg_begin, t.seg_end);
    auto it = pidx.find(key);
    if (it == pidx.end()) {
      it = pidx.emplace(key, probs.size()).first;
      probs.push_back({t.c, t.ldc, 0, 0, t.beta, t.seg_begin, t.seg_end});
    }
    Prob& p = probs[it->second];
    DMRG_REQUIRE(p.beta == t.beta && p.ldc == t.ldc, kErrState, "launch_gemm: inconsistent tiles");
    p.m = std::max(p.m, t.row0 + t.m);
    p.n = std::max(p.n, t.col0 + t.n);
  }
  if (probs.empty()) return;
  // distinct operands (source, ld, order, k) with the rows they need
  std::map<std::tuple<const void*, int, int, int>, int> opidx;
  std::vector<PackOp> ops;
  auto operand = [&](const void* src, int ld, int colmajor, int k, int rows) {
    auto key = std::make_tuple(src, ld, colmajor, k);
    auto it = opidx.find(key);
    if (it == opidx.end()) {
      it = opidx.emplace(key, (int)ops.size()).first;
      PackOp o{};
      o.src = static_cast<const double*>(src);
      o.ld = ld;
      o.colmajor = colmajor;
      o.k = k;
      o.kp = (k + 7) & ~7;
      ops.push_back(o);
    }
    ops[it->second].rows = std::max(ops[it->second].rows, rows);
    return it->second;
  };
  std::vector<std::pair<int, int>> segop(b.segs.size(), {-1, -1});
  for (const Prob& p : probs)
    for (int j = p.s0; j < p.s1; ++j) {
      const GemmSeg& g = b.segs[(size_t)j];
      DMRG_REQUIRE(g.k >= 0, kErrState, "launch_gemm: negative k");
      segop[(size_t)j] = {operand(g.a, g.lda, (g.flags & kTransA) ? 1 : 0, g.k, p.m),
                          operand(g.b, g.ldb, (g.flags & kTransB) ? 0 : 1, g.k, p.n)};
    }
  int64_t elems = 0, chunks = 0;
  for (PackOp& o : ops) {
    o.dst = elems;
    o.chunk0 = chunks;
    const int64_t n = (int64_t)o.rows * o.kp;
    elems += 2 * n;
    chunks += n / 8;
  }
  grow_buf(sc.pack, (size_t)std::max<int64_t>(elems, 8) * sizeof(uint16_t), s);
  grow_buf(sc.ops, std::max<size_t>(1, ops.size()) * sizeof(PackOp), s);
  uint16_t* base = sc.pack.as<uint16_t>();
  DMRG_HIP(hipMemcpyAsync(sc.ops.p, ops.data(), ops.size() * sizeof(PackOp), hipMemcpyHostToDevice, s));
  launch_pack_bf16(sc.ops.as<PackOp>(), (int)ops.size(), chunks, base, s);
  GemmBatchB bb;
  bb.shape = kShape64x64;
  for (const Prob& p : probs) {
    const size_t s0 = bb.segs.size();
    for (int j = p.s0; j < p.s1; ++j) {
      const GemmSeg& g = b.segs[(size_t)j];
      const PackOp& oa = ops[(size_t)segop[(size_t)j].first];
      const PackOp& ob = ops[(size_t)segop[(size_t)j].second];
      GemmSegB sb;
      sb.a = base + oa.dst;
      sb.b = base + ob.dst;
      sb.alo = (int64_t)oa.rows * oa.kp;
      sb.blo = (int64_t)ob.rows * ob.kp;
      sb.lda = oa.kp;
      sb.ldb = ob.kp;
      sb.k = g.k;
      sb.flags = 0;
      sb.alpha = g.alpha;
      bb.segs.push_back(sb);
    }
    bb.add_problem(p.c, 0, p.ldc, p.m, p.n, s0, bb.segs.size(), p.beta);
  }
  DevGemmB d;
  upload_gemm_bf16(bb, d);
  launch_gemm_bf16(d, sc.precision == 2, kOutF64, 0, s);
  // the descriptors and packed operands are released or reused after this
  DMRG_HIP(hipStreamSynchronize(s));
}
}  // namespace

GemmPrecisionScope::GemmPrecisionScope(int p) : precision(p), prev(0) {
  DMRG_REQUIRE(p >= 0 && p <= 2, kErrInvalidArg, "GemmPrecisionScope: precision must be 0, 1 or 2");
  DMRG_REQUIRE(!g_scope, kErrState, "GemmPrecisionScope: scopes do not nest");
  g_scope = this;
}
GemmPrecisionScope::~GemmPrecisionScope() { g_scope = nullptr; }

void launch_gemm(const GemmBatch& b, DevBuf& desc, hipStream_t s) {
  if (!g_scope || g_scope->precision == 0 || b.tiles.empty()) {
    launch_gemm_f64(b, s);
    return;
  }
  launch_gemm_lowp(b, *g_scope, s);
}

}  // namespace dmrg
