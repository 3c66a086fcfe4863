// Block-sparse renormalised operators, their construction along the chain,
// and the two-site sigma plan.
#pragma once
#include <map>
#include <memory>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "gemm.h"
#include "gemm_bf16.h"
#include "gemm_oz.h"
#include "strings.h"

namespace dmrg {

// ---- problem (integrals) ----------------------------------------------------
struct Problem {
  int K = 0, N = 0, tsz = 0;
  bool all_terms = false;  // enumerate terms with zero integrals too (backward)
  double e_core = 0;
  std::vector<double> h, eri;  // K*K and K^4, chemists' (pq|rs)
  double t(int P, int Q) const {
    return ((P ^ Q) & 1) ? 0.0 : h[(size_t)(P >> 1) * K + (Q >> 1)];
  }
};

// Calls f(coef, str, entry, factor) for every nonzero term of
//   H = sum t_PQ a+_P a_Q + 1/2 sum V_PQRS a+_P a+_Q a_R a_S,
//   V_PQRS = (ps|qr) d(s_P,s_S) d(s_Q,s_R)
// restricted to spatial-index tuples accepted by keep(list, count).
// coef = factor * (integral entry): entry indexes [h (K*K) | eri (K^4)].
template <class Keep, class F>
void for_each_term(const Problem& P, Keep&& keep, F&& f) {
  const int K = P.K;
  const int64_t K2 = (int64_t)K * K;
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < K; ++q) {
      const int ix[2] = {p, q};
      if (!keep(ix, 2)) continue;
      const double t = P.h[(size_t)p * K + q];
      if (t == 0.0 && !P.all_terms) continue;
      for (int a = 0; a < 2; ++a) {
        Str s;
        s.push(2 * p + a, 1);
        s.push(2 * q + a, 0);
        f(t, s, (int64_t)p * K + q, 1.0);
      }
    }
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < K; ++q)
      for (int r = 0; r < K; ++r)
        for (int u = 0; u < K; ++u) {
          const int ix[4] = {p, q, r, u};
          if (!keep(ix, 4)) continue;
          const int64_t e = (((int64_t)p * K + u) * K + q) * K + r;  // (pu|qr)
          const double g = P.eri[(size_t)e];
          if (g == 0.0 && !P.all_terms) continue;
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              const int A = 2 * p + a, B = 2 * q + b, C = 2 * r + b, D = 2 * u + a;
              if (A == B || C == D) continue;
              Str s;
              s.push(A, 1);
              s.push(B, 1);
              s.push(C, 0);
              s.push(D, 0);
              f(0.5 * g, s, K2 + e, 0.5);
            }
        }
}

// ---- bonds and layouts --------------------------------------------------------
struct Bond {
  std::vector<QN> q;
  std::vector<int> d;
  std::vector<int64_t> off;  // state offset of each sector
  int64_t total = 0;
  std::map<QN, int> idx;
  void finish() {
    off.assign(q.size(), 0);
    total = 0;
    idx.clear();
    for (size_t k = 0; k < q.size(); ++k) {
      off[k] = total;
      total += d[k];
      idx[q[k]] = (int)k;
    }
  }
  int find(QN x) const {
    auto it = idx.find(x);
    return it == idx.end() ? -1 : it->second;
  }
  size_t size() const { return q.size(); }
};

// Blocks of an operator with own quantum-number change dq acting on the
// states of one bond.  Bond labels are the quantum numbers of the part left
// of the bond, so for a left block row = col + dq and for a right block
// row = col - dq.  Block rows are padded to a multiple of 8 elements (the
// padding stays zero) so that every block row starts 16-byte aligned in the
// BF16 copies and vector loads along a row never leave the block.
inline int pad8(int x) { return (x + 7) & ~7; }
inline int64_t pad8(int64_t x) { return (x + 7) & ~(int64_t)7; }

struct Layout {
  QN dq;
  int side = +1;
  struct Blk {
    int r, c, dr, dc, ld;
    int64_t off;
  };
  std::vector<Blk> blk;
  std::vector<int> by_col;
  int64_t nnz = 0;
  void build(const Bond& b, QN dq_, int side_) {
    dq = dq_;
    side = side_;
    blk.clear();
    by_col.assign(b.size(), -1);
    nnz = 0;
    for (size_t c = 0; c < b.size(); ++c) {
      QN rq = side > 0 ? b.q[c] + dq : b.q[c] - dq;
      int r = b.find(rq);
      if (r < 0) continue;
      by_col[c] = (int)blk.size();
      const int ld = pad8(b.d[c]);
      blk.push_back({r, (int)c, b.d[r], b.d[c], ld, nnz});
      nnz += (int64_t)b.d[r] * ld;
    }
  }
  const Blk* col(int c) const { return (c >= 0 && by_col[c] >= 0) ? &blk[by_col[c]] : nullptr; }
};

// ---- operators ----------------------------------------------------------------
enum OpKind : uint8_t { kIdent = 0, kHam = 1, kNormal = 2, kComp = 3, kPsum = 4 };

struct OpKey {
  uint8_t kind = 0;
  uint64_t s = 0;
  bool operator==(const OpKey& o) const { return kind == o.kind && s == o.s; }
};
struct OpKeyHash {
  size_t operator()(const OpKey& k) const { return std::hash<uint64_t>()(k.s * 8 + k.kind); }
};

struct OpClass {
  Layout L;
  int nops = 0;
  DevBuf data;  // nops x nnz, FP64
  double* op(int i) const { return data.as<double>() + (int64_t)i * L.nnz; }
};

struct OpRef {
  int cls = -1, idx = -1;
};

// A set of renormalised operators on one block.
struct Env {
  int side = +1;  // +1: sites [0, bond); -1: sites [bond, K)
  int bond = 0;
  Bond basis;
  std::vector<std::unique_ptr<OpClass>> classes;
  std::map<QN, int> class_of_dq;
  std::unordered_map<OpKey, OpRef, OpKeyHash> ops;
  int class_for(QN dq) {
    auto it = class_of_dq.find(dq);
    if (it != class_of_dq.end()) return it->second;
    auto c = std::make_unique<OpClass>();
    c->L.build(basis, dq, side);
    classes.push_back(std::move(c));
    class_of_dq[dq] = (int)classes.size() - 1;
    return (int)classes.size() - 1;
  }
  OpRef add(OpKey k, QN dq) {
    auto it = ops.find(k);
    if (it != ops.end()) return it->second;
    int c = class_for(dq);
    OpRef r{c, classes[c]->nops++};
    ops[k] = r;
    return r;
  }
  const OpRef* get(OpKey k) const {
    auto it = ops.find(k);
    return it == ops.end() ? nullptr : &it->second;
  }
  void allocate(hipStream_t s);  // device arrays for every class, zeroed
  size_t bytes() const {
    size_t b = 0;
    for (auto& c : classes) b += c->data.bytes;
    return b;
  }
};

// Device copy of one site tensor: blocks (l, n) -> r packed in (l, n) order.
struct SiteTensor {
  std::vector<int64_t> off;  // offset of block (l, n) at index 4*l+n, -1 if absent
  DevBuf data;
};

struct Mps {
  int K = 0, N = 0, tsz = 0;
  std::vector<Bond> bonds;       // K+1
  std::vector<SiteTensor> site;  // K (window sites may be empty)
};

// A projection dst += alpha * Proj(src (x) y) onto the next bond; side +1
// projects a left-block operator with A_site, side -1 a right-block one with
// B_site (dst and src are operators of the layouts dl / sl).
struct Projection {
  const double* src;
  const Layout* sl;
  Mat4 y;
  int ypar;
  double* dst;
  const Layout* dl;
  double alpha;
};
void run_projections(int side, const Mps& m, int site, const std::vector<Projection>& projs,
                     DevBuf& desc, DevBuf& uws, int64_t budget, hipStream_t s);

// Provenance of component coefficients, for the backward:
// (target cls, target idx, source cls, source idx, site string) -> list of
// (integral entry, d coefficient / d entry).
using CompKey = std::tuple<int, int, int, int, uint64_t>;
struct CompProv {
  std::map<CompKey, double> coef;                                  // total coefficients
  std::map<CompKey, std::vector<std::pair<int64_t, double>>> prov;  // integral dependence
};

// Builds the operators of sites [0, b+1) from those of [0, b) and site b.
// When rec is given, every component and its integral dependence is recorded.
std::unique_ptr<Env> left_start(const Mps& m, hipStream_t s);
std::unique_ptr<Env> right_start(const Mps& m, hipStream_t s);
std::unique_ptr<Env> grow_left(const Problem& P, const Mps& m, const Env& old, DevBuf& scratch,
                               hipStream_t s, CompProv* rec = nullptr);
std::unique_ptr<Env> grow_right(const Problem& P, const Mps& m, const Env& old, DevBuf& scratch,
                                hipStream_t s, CompProv* rec = nullptr);

// ---- sigma ----------------------------------------------------------------------
// psi of window (i, i+1) is stored right-sector-major: for each sector r of
// bond i+2 the rows (l, n1, n2) with Q_l + Q_n1 + Q_n2 = Q_r in ascending
// order form a dense M_r x d_r row-major matrix Psi_r; the Psi_r follow each
// other in ascending r.
//
// Internally the sigma works on a padded copy: every (l, n1, n2) row group
// starts at a multiple of 8 rows and holds pad8(d_l) rows (zero padding),
// and rows have pad8(d_r) columns.  PsiT_r (d_r x rows_pad) is its transpose.
struct PsiLayout {
  std::vector<int64_t> rows_of;  // M_r
  std::vector<int64_t> off;      // element offset of Psi_r (API layout)
  std::vector<std::map<std::pair<int, int>, int64_t>> row_of;  // per r: (l, 4*n1+n2) -> row
  int64_t size = 0;
  // padded copy
  std::vector<int64_t> rows_pad, off_pad, offT;
  std::vector<int> ld;
  std::vector<std::map<std::pair<int, int>, int64_t>> row_pad_of;
  int64_t size_pad = 0, sizeT = 0;
  void build(const Bond& bl, const Bond& br);
};

// Row-group copy task: rows x cols from src (row stride sld) to dst (dld),
// optionally transposed (dst[c][r] = src[r][c]).
struct CopyTask {
  const double* src;
  double* dst;
  int32_t rows, cols, sld, dld;
};

struct OpView {
  const double* data = nullptr;
  const Layout* lay = nullptr;
};

struct SigmaPair {
  OpView L;  // left operator (stored, or a window partial sum)
  int z;     // index into SigmaPlan::zops, -1 = identity
  Mat16 y;   // site matrix, coefficient folded in
  int ypar;  // fermion parity of the site string
  bool pinned = false;  // always FP64 (block Hamiltonians: energy-sized diagonals)
  int lsrc = 0;         // 0: stored left operator, 1: window partial sum
  OpRef lref;           // the left operator in the left block or in psums
};

// The sigma schedule is kept precision-agnostic: operands are (buffer id,
// element offset) and are turned into device descriptors per precision.
struct BufRef {
  int buf = -1;
  int64_t off = 0;
};
struct ASeg {
  BufRef a, b;
  int32_t lda, ldb, k, flags;
  double alpha;
};
struct AProb {
  BufRef c;
  int32_t ldc, m, n;
  int64_t s0, s1;
  int32_t beta;
  int32_t key = 0;  // locality group: problems of one key run on one XCD
};
struct AStage {
  std::vector<ASeg> segs;
  std::vector<AProb> probs;
  double flops = 0;
};
struct PlanBuf {
  double* f64 = nullptr;  // FP64 data (not owned unless in own)
  int64_t n = 0;          // elements
  DevBuf own;             // storage when the plan owns the buffer
  DevBuf bf;              // BF16 copy: hi at [0, n), lo at [n, 2n) (uint16)
  bool is_operator = false;
};

// Optional kernel timing of run_sigma: HIP events recorded on the launch
// stream around every grouped-GEMM launch (role 1 / 2: main stages, role 3:
// the FP64 launches of the pinned pairs).
struct SigmaTiming {
  bool on = false;
  int calls = 0;
  double ms[4] = {0, 0, 0, 0};  // by role
  int launches[4] = {0, 0, 0, 0};
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;  // (role, begin/end)
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void record(int role, hipEvent_t a, hipEvent_t b) { pending.push_back({role, {a, b}}); }
  void collect(hipStream_t s);  // waits for the stream, folds pending events into ms
  void reset();
  SigmaTiming() = default;
  SigmaTiming(const SigmaTiming&) = delete;
  SigmaTiming& operator=(const SigmaTiming&) = delete;
  ~SigmaTiming();
};

// Launch configuration of the BF16 stages (chosen by the autotuner).
constexpr int kShapeMixed = kNumShapes;  // tile shape chosen per output problem
// 128 x 128 tiles over whole 128-blocks of each output problem; remainders
// of at most 64 rows or columns on 64-wide tiles (one launch per shape)
constexpr int kShapeSplit = kNumShapes + 1;
struct BfChoice {
  int shape = kShape128x64;  // tile shape, kShapeMixed or kShapeSplit
  int order = 0;             // 0: per-problem XCD groups, 1: groups by locality key
  int sort_a = 0;            // 1: segments of a problem sorted by their A operand
};
struct TuneEntry {
  int stage;
  BfChoice choice;
  double ms;
};

// Executable graphs of the sigma, one per precision (captured on first use).
struct SigmaGraphs {
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  hipStream_t capture = nullptr;  // stream the graphs are captured on
  SigmaGraphs() = default;
  SigmaGraphs(const SigmaGraphs&) = delete;
  SigmaGraphs& operator=(const SigmaGraphs&) = delete;
  ~SigmaGraphs();
};

// Ozaki-scheme sigma (precision 3): digit planes and row exponents of every
// distinct operand of the two stages in one arena: operators and window
// partial sums (sliced once per plan), psi (sliced per sigma) and the
// stage-1 workspace (sliced per chunk, a region shared by the chunks).
struct OzPlan {
  int kappa = 0;  // 0: not prepared
  DevBuf arena, exps;
  DevBuf ops_static, ops_psi;
  int n_static = 0, n_psi = 0;
  int64_t rows_static = 0, rows_psi = 0;
  std::vector<DevBuf> ops_ws;  // per chunk
  std::vector<int> n_ws;
  std::vector<int64_t> rows_ws;
  std::vector<DevGemmO> s1, s2;  // per chunk
  bool statics_sliced = false;
  int64_t arena_bytes = 0;
};

struct SigmaPlan {
  int window = -1;
  bool use_graphs = false;  // replay each sigma from a HIP graph
  SigmaGraphs graphs;
  BfChoice bf_choice[2];            // stage 1, stage 2
  std::vector<TuneEntry> tune_log;  // autotuner trials
  double tune_ms = 0;
  SigmaTiming timing;
  PsiLayout psi;
  std::unique_ptr<Env> psums;  // window partial sums of left operators
  std::vector<OpView> zops;    // distinct right operators
  std::vector<int> zpar;
  std::vector<SigmaPair> pairs;
  std::vector<PlanBuf> bufs;
  int buf_psi = -1, buf_sig = -1, buf_ws = -1, buf_psit = -1;
  DevBuf pack_tasks, unpack_tasks, trans_tasks;  // CopyTask arrays
  int n_pack = 0, n_trans = 0;
  std::vector<CopyTask> pack_host, unpack_host;  // API side as byte offsets
  const double* bound_psi = nullptr;
  const double* bound_sigma = nullptr;
  std::vector<AStage> s1, s2;  // per chunk (pairs not pinned to FP64)
  AStage p1, p2;               // pairs pinned to FP64 (one chunk)
  double flops_s2_ident = 0;  // stage-2 FLOPs whose left operand is the identity
  // materialised descriptors
  std::vector<DevGemm> f64_s1, f64_s2;
  DevGemm f64_p1, f64_p2;
  std::vector<std::vector<DevGemmB>> bf_s1, bf_s2;  // per chunk: one launch per tile shape
  bool bf_ready = false;
  OzPlan oz;
  // FP64 schedule with the stage-1 workspace at a caller-given fixed address
  // (descriptors built at plan time, so running it allocates nothing)
  std::vector<DevGemm> fx_s1, fx_s2;
  DevGemm fx_p1, fx_p2;
  bool fx_ready = false;
  DevBuf diag;                 // diag(H_eff) for the Davidson preconditioner
  bool diag_ready = false;
  double flops = 0;            // algorithmic FLOPs of one sigma
  double flops_stage1 = 0, flops_stage2 = 0;
  // sum over (term, psi block) of the cheaper of the two association orders
  double flops_terms = 0;
  // stage-1 FLOPs of the rows stage 2 reads (stage 1 multiplies whole psi sectors)
  double flops_s1_used = 0;
  int64_t ws_doubles = 0;
  // kept for the backward
  std::vector<OpRef> zrefs;    // right-block operator of each zops entry
  bool record = false;
  using PsumKey = std::pair<uint64_t, uint64_t>;  // (site string, right string)
  std::map<PsumKey, std::map<std::pair<int, int>, std::vector<std::pair<int64_t, double>>>> psum_prov;
  std::vector<std::pair<PsumKey, OpRef>> wkeys;    // partial sum of each key
  std::map<int, int> w_src_cls;                    // psums class -> left class of its sources
};

// Plans the sigma of window (i, i+1) from the left block at bond i and the
// right block at bond i+2 (both renormalised).
// With record set, the plan also keeps the integral dependence of the
// partial-sum coefficients (for the backward).
std::unique_ptr<SigmaPlan> plan_sigma(const Problem& P, const Mps& m, const Env& L, const Env& R,
                                      int64_t ws_budget_doubles, hipStream_t s, bool record = false);
// Copies psi (API layout) into the plan's padded psi buffer and its transpose.
void plan_load_psi(SigmaPlan& plan, const double* psi, hipStream_t s);
// sigma = H_eff psi (device pointers, right-sector-major psi layout).
// precision: 0 FP64, 1 BF16, 2 split-BF16x3, 3 Ozaki-scheme FP64 emulation
// on INT8 (block Hamiltonian pairs stay FP64 in 1-3).
void run_sigma(SigmaPlan& plan, const double* psi, double* sigma, int precision, hipStream_t s);
void prepare_bf16(SigmaPlan& plan, hipStream_t s);
// Builds the FP64 descriptors of the plan's schedule with the stage-1
// workspace at ws (ws_doubles doubles) instead of the plan's own buffer;
// false (and nothing built) when the plan's workspace does not fit.
bool plan_fixed_workspace(SigmaPlan& plan, double* ws, int64_t ws_doubles);
// FP64 sigma on that schedule: host work only binds the caller's buffers
// (task-list copies when the pointers change); no device allocation.
void run_sigma_fixed_workspace(SigmaPlan& plan, const double* psi, double* sigma, hipStream_t s);
// Slices per operand (kappa digits, DMRG_OZAKI_SLICES, default 6) and the
// Ozaki task lists of both stages.
void prepare_ozaki(SigmaPlan& plan, hipStream_t s);
int ozaki_kappa();

}  // namespace dmrg
