// Spin-adapted (SU(2)) contraction on the FP64 grouped GEMM.
//
// The reduced window vector holds coupled blocks (a, b) of a left multiplet
// sector a = (N_a, 2S_a, d_a) and a right sector b (total N and S).  A scalar
// product c [A^k x B^k]^0 of a left and a right tensor operator acts block by
// block as
//   sigma[a', b'] += c (-1)^(p N_a) W(S_a', S_b', S_a, S_b, S, k) A[a', a] psi[a, b] B[b', b]^T
// with the recoupling factor
//   W = (-1)^(S_a + S_b' + S + k) sqrt((2 S_a' + 1)(2 S_b' + 1) / (2k + 1)) {S_a S_b S; S_b' S_a' k}
// for reduced matrices in the Clebsch-Gordan convention of the Wigner-Eckart
// theorem (the 6j symbol from Racah's formula).  The two stages are the ones
// of the U(1) sigma: stage 1 forms T = psi[., b] B[b', b]^T once per right
// operator block, over the blocks (a, b) of its right sector stacked by a
// (NT products), stage 2 accumulates W c (-1)^(p N_a) A[a', a] T[a] into
// each output block (NN products).  A plan keeps both stages' descriptors per
// chunk of right operators, whose stage-1 products fit the workspace budget;
// stage 1 only forms the rows some pair's stage 2 reads, and long stage-2
// product lists are split over partial sums of sigma.  Split-BF16x3 plans
// run the same products on the BF16 kernel from packed hi/lo copies.
#include "su2.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"
#include "engine.h"
#include "gemm.h"
#include "gemm_bf16.h"

namespace dmrg {

namespace {

bool triangle(int ta, int tb, int tc) { return tc >= std::abs(ta - tb) && tc <= ta + tb && (ta + tb + tc) % 2 == 0; }

// n! for n = t2 / 2 (t2 even and >= 0), in double (the spins here are small)
double fact_half(int t2) {
  double f = 1.0;
  for (int i = 2; i <= t2 / 2; ++i) f *= i;
  return f;
}

double delta(int ta, int tb, int tc) {
  return std::sqrt(fact_half(ta + tb - tc) * fact_half(ta - tb + tc) * fact_half(-ta + tb + tc) /
                   fact_half(ta + tb + tc + 2));
}

// W above (doubled spins: primed first, then unprimed, then S and k)
double recoupling(int tSa2, int tSb2, int tSa, int tSb, int tS, int tk) {
  const int ph = (tSa + tSb2 + tS + tk) / 2;
  return ((ph & 1) ? -1.0 : 1.0) * std::sqrt((tSa2 + 1.0) * (tSb2 + 1.0) / (tk + 1.0)) *
         wigner_6j(tSa, tSb, tS, tSb2, tSa2, tk);
}

struct Window {
  std::vector<int> ln, ls, ld, rn, rs, rd;
  int n, ts;
  std::vector<int64_t> off;  // coupled block (a, b) -> element offset at a * n_right + b, or -1
  int64_t size = 0;
  int64_t at(int a, int b) const { return off[(size_t)a * rn.size() + b]; }
};

Window parse(const dmrg_su2_window& w) {
  DMRG_REQUIRE(w.n_left > 0 && w.n_right > 0, kErrInvalidArg, "su2: a window needs left and right sectors");
  DMRG_REQUIRE(w.left_n && w.left_two_s && w.left_dim && w.right_n && w.right_two_s && w.right_dim,
               kErrInvalidArg, "su2: NULL sector array");
  DMRG_REQUIRE(w.n_elec >= 0 && w.two_s >= 0 && (w.n_elec - w.two_s) % 2 == 0, kErrInvalidArg,
               "su2: total N and 2S must be non-negative with equal parity");
  Window W;
  W.n = w.n_elec;
  W.ts = w.two_s;
  auto side = [&](int k, const int32_t* n, const int32_t* s, const int32_t* d, std::vector<int>& on,
                  std::vector<int>& os, std::vector<int>& od) {
    for (int i = 0; i < k; ++i) {
      DMRG_REQUIRE(n[i] >= 0 && s[i] >= 0 && (n[i] - s[i]) % 2 == 0 && d[i] > 0, kErrInvalidArg,
                   "su2: a sector needs N, 2S >= 0 of equal parity and a positive dimension");
      on.push_back(n[i]);
      os.push_back(s[i]);
      od.push_back(d[i]);
    }
  };
  side(w.n_left, w.left_n, w.left_two_s, w.left_dim, W.ln, W.ls, W.ld);
  side(w.n_right, w.right_n, w.right_two_s, w.right_dim, W.rn, W.rs, W.rd);
  W.off.assign((size_t)w.n_left * w.n_right, -1);
  for (int a = 0; a < w.n_left; ++a)
    for (int b = 0; b < w.n_right; ++b)
      if (W.ln[a] + W.rn[b] == W.n && triangle(W.ls[a], W.rs[b], W.ts)) {
        W.off[(size_t)a * w.n_right + b] = W.size;
        W.size += (int64_t)W.ld[a] * W.rd[b];
      }
  return W;
}

// Blocks of an operator grouped by their ket (in) sector.
std::vector<std::vector<int>> by_in_sector(const dmrg_su2_operator& o, int ns) {
  std::vector<std::vector<int>> v(ns);
  for (int i = 0; i < o.n_blocks; ++i) v[o.in_sector[i]].push_back(i);
  return v;
}

// A stage-2 product: pair, block of its right operator B, block of its left
// operator A, and the scale c (-1)^(p N_a) W.
struct Prod {
  int p, i, j;
  double scale;
};
// The stage-1 product of a right-operator block: rows [lo, hi) of psi_b and
// the workspace offset of T(r, i).
struct S1 {
  int64_t lo = -1, hi = -1, off = 0;
};
inline int64_t pad8(int64_t x) { return (x + 7) & ~(int64_t)7; }

// Output tiles (rows, cols) of the two stages: 128 x 64 with eight waves
// for both, measured at the CAS(89,102)-shaped workload (ms per sigma):
// 170.7, against 178.3 with 64 x 64, 177.3 with 128 x 64 for stage 1 only,
// 186.4 with 128 x 128 and 182.7 with 64 x 128 for stage 1.
// DMRG_SU2_TILE="t1,t2" overrides, each 64, 128 (square), 128x64 or 64x128.
std::pair<std::pair<int, int>, std::pair<int, int>> su2_tiles() {
  std::pair<int, int> t[2] = {{128, 64}, {128, 64}};
  if (const char* e = std::getenv("DMRG_SU2_TILE")) {
    auto parse = [](const std::string& w, std::pair<int, int>& o) {
      int a = 0, b = 0;
      if (std::sscanf(w.c_str(), "%dx%d", &a, &b) == 2) o = {a, b};
      else if (std::sscanf(w.c_str(), "%d", &a) == 1) o = {a, a};
      else return false;
      return (o.first == 64 || o.first == 128) && (o.second == 64 || o.second == 128);
    };
    const std::string v(e);
    const size_t comma = v.find(',');
    DMRG_REQUIRE(comma != std::string::npos && parse(v.substr(0, comma), t[0]) && parse(v.substr(comma + 1), t[1]),
                 kErrInvalidArg, "DMRG_SU2_TILE must be \"t1,t2\", each 64, 128, 128x64 or 64x128");
  }
  return {t[0], t[1]};
}

// BF16 tile shapes of the split-BF16x3 stages: 64 x 128 for stage 1 (its
// BF16 hi/lo output), 64 x 64 for stage 2 (FP64 flush with each product's
// scale), measured at the CAS(89,102)-shaped workload (ms per sigma): 85.6,
// against 117.9 with 128 x 128 and 90.0 with 128 x 64 for stage 1, 89.6
// with 128 x 64 and 86.2 with 64 x 128 for stage 2.
// DMRG_SU2_BF16_SHAPE="s1,s2" overrides, each 64x64, 128x64 or 64x128
// (stage 1 also 128x128).
std::pair<int, int> su2_bf16_shapes() {
  int sh[2] = {kShape64x128, kShape64x64};
  if (const char* e = std::getenv("DMRG_SU2_BF16_SHAPE")) {
    auto parse = [](const std::string& w, int& o, bool square) {
      if (w == "64x64") o = kShape64x64;
      else if (w == "128x64") o = kShape128x64;
      else if (w == "64x128") o = kShape64x128;
      else if (square && w == "128x128") o = kShape128x128s3;
      else return false;
      return true;
    };
    const std::string v(e);
    const size_t comma = v.find(',');
    DMRG_REQUIRE(comma != std::string::npos && parse(v.substr(0, comma), sh[0], true) &&
                     parse(v.substr(comma + 1), sh[1], false),
                 kErrInvalidArg, "DMRG_SU2_BF16_SHAPE must be \"s1,s2\", each 64x64, 128x64 or 64x128 "
                 "(stage 1 also 128x128)");
  }
  return {sh[0], sh[1]};
}

}  // namespace

double wigner_6j(int tj1, int tj2, int tj3, int tj4, int tj5, int tj6) {
  if (!(triangle(tj1, tj2, tj3) && triangle(tj1, tj5, tj6) && triangle(tj4, tj2, tj6) && triangle(tj4, tj5, tj3)))
    return 0.0;
  const double pre = delta(tj1, tj2, tj3) * delta(tj1, tj5, tj6) * delta(tj4, tj2, tj6) * delta(tj4, tj5, tj3);
  const int lo = std::max(std::max(tj1 + tj2 + tj3, tj1 + tj5 + tj6), std::max(tj4 + tj2 + tj6, tj4 + tj5 + tj3));
  const int hi = std::min(std::min(tj1 + tj2 + tj4 + tj5, tj2 + tj3 + tj5 + tj6), tj3 + tj1 + tj6 + tj4);
  double sum = 0.0;
  for (int t2 = lo; t2 <= hi; t2 += 2) {
    const double den = fact_half(t2 - tj1 - tj2 - tj3) * fact_half(t2 - tj1 - tj5 - tj6) *
                       fact_half(t2 - tj4 - tj2 - tj6) * fact_half(t2 - tj4 - tj5 - tj3) *
                       fact_half(tj1 + tj2 + tj4 + tj5 - t2) * fact_half(tj2 + tj3 + tj5 + tj6 - t2) *
                       fact_half(tj3 + tj1 + tj6 + tj4 - t2);
    sum += (((t2 / 2) & 1) ? -1.0 : 1.0) * fact_half(t2 + 2) / den;
  }
  return pre * sum;
}

int64_t su2_psi_size(const dmrg_su2_window& w) { return parse(w).size; }

namespace {

// The split-BF16x3 descriptors: operator blocks packed once into
// k-contiguous BF16 hi/lo planes (rows padded to 8), psi_b packed per call,
// stage 1 writing T(r, i)^T (d_b' x M_b, BF16 hi/lo) and stage 2 reading the
// d_a columns of block a from it; every product is NT on 16-byte aligned
// rows, as the BF16 kernel needs.
void build_bf16(Su2Plan& plan, const Window& W, const dmrg_su2_operator* left_ops,
                const dmrg_su2_operator* right_ops, const std::vector<std::vector<Prod>>& prods_of_r,
                const dmrg_su2_pair* pairs, const std::vector<std::map<int, S1>>& need,
                const std::vector<std::pair<int, int>>& chunks, const std::vector<int64_t>& mb,
                const std::vector<int64_t>& boff, const std::vector<int64_t>& rowoff, size_t seg_per_part,
                hipStream_t s) {
  const int nr = (int)W.rn.size();
  // packed operator blocks: (op, block) -> element offset of its hi plane
  std::vector<PackOp> ops;
  int64_t chunks8 = 0, total = 0;
  auto add = [&](const double* src, int rows, int k) {
    const int kp = (int)pad8(k);
    ops.push_back({src, total, chunks8, k, rows, k, kp, 0, 0});
    const int64_t at = total;
    total += 2 * (int64_t)rows * kp;
    chunks8 += (int64_t)rows * kp / 8;
    return at;
  };
  std::map<std::pair<int, int>, int64_t> lpos, rpos;  // (op, block) -> packed offset
  for (int r = 0; r < (int)prods_of_r.size(); ++r)
    for (const Prod& x : prods_of_r[r]) {
      const int l = pairs[x.p].left_op;
      const dmrg_su2_operator& A = left_ops[l];
      if (!lpos.count({l, x.j}))
        lpos[{l, x.j}] = add(A.data + A.offset[x.j], W.ld[A.out_sector[x.j]], W.ld[A.in_sector[x.j]]);
    }
  for (int r = 0; r < (int)need.size(); ++r)
    for (auto& kv : need[r]) {
      const dmrg_su2_operator& B = right_ops[r];
      rpos[{r, kv.first}] = add(B.data + B.offset[kv.first], W.rd[B.out_sector[kv.first]], W.rd[B.in_sector[kv.first]]);
    }
  plan.opk.alloc((size_t)std::max<int64_t>(total, 8) * sizeof(uint16_t));
  uint16_t* K = plan.opk.as<uint16_t>();
  {
    DevBuf d(std::max<size_t>(1, ops.size()) * sizeof(PackOp));
    if (!ops.empty()) {
      DMRG_HIP(hipMemcpy(d.p, ops.data(), ops.size() * sizeof(PackOp), hipMemcpyHostToDevice));
      launch_pack_bf16(d.as<PackOp>(), (int)ops.size(), chunks8, K, s);
    }
    DMRG_HIP(hipStreamSynchronize(s));
  }
  // psi_b packed per call: one pass over every right sector's M_b x d_b matrix
  std::vector<int64_t> poff(nr, 0);
  {
    std::vector<PackOp> pops;
    int64_t c8 = 0, at = 0;
    for (int b = 0; b < nr; ++b) {
      if (mb[b] == 0) continue;
      const int kp = (int)pad8(W.rd[b]);
      poff[b] = at;
      pops.push_back({plan.psi_b.as<double>() + boff[b], at, c8, W.rd[b], (int)mb[b], W.rd[b], kp, 0, 0});
      at += 2 * mb[b] * kp;
      c8 += mb[b] * kp / 8;
    }
    plan.psi_pack.alloc((size_t)std::max<int64_t>(at, 8) * sizeof(uint16_t));
    plan.psi_pack_ops.alloc(std::max<size_t>(1, pops.size()) * sizeof(PackOp));
    if (!pops.empty())
      DMRG_HIP(hipMemcpy(plan.psi_pack_ops.p, pops.data(), pops.size() * sizeof(PackOp), hipMemcpyHostToDevice));
    plan.n_psi_pack = (int)pops.size();
    plan.psi_pack_chunks = c8;
  }
  const uint16_t* Q = plan.psi_pack.as<uint16_t>();
  const auto shapes = su2_bf16_shapes();
  plan.wsk.alloc((size_t)std::max<int64_t>(2 * plan.ws_doubles, 8) * sizeof(uint16_t));
  uint16_t* T = plan.wsk.as<uint16_t>();
  const int64_t tlo = plan.ws_doubles;  // lo plane of the workspace
  double* Part = plan.part.as<double>();
  const int n_parts = plan.n_parts;
  for (size_t c = 0; c < chunks.size(); ++c) {
    // stage 1: columns [lo, pad8(hi)) of T(r, i)^T = B_r[i] psi_b^T (d_b' x M_b)
    GemmBatchB b1;
    b1.shape = shapes.first;
    for (int r = chunks[c].first; r < chunks[c].second; ++r) {
      const dmrg_su2_operator& B = right_ops[r];
      for (auto& kv : need.at(r)) {
        const int i = kv.first;
        const S1& e = kv.second;
        const int b2 = B.out_sector[i], b = B.in_sector[i];
        const int64_t kp = pad8(W.rd[b]);
        const size_t s0 = b1.segs.size();
        b1.segs.push_back({K + rpos.at({r, i}), Q + poff[b] + e.lo * kp, (int64_t)W.rd[b2] * kp,
                           mb[b] * kp, (int)kp, (int)kp, W.rd[b], kTransB, 1.0});
        b1.add_problem(T + e.off + e.lo, tlo, (int)mb[b], W.rd[b2], (int)(pad8(e.hi) - e.lo), s0, s0 + 1, 0);
      }
    }
    // stage 2: as the FP64 plan, on the packed operands
    std::map<std::pair<int, int>, std::vector<GemmSegB>> outs;
    for (int r = chunks[c].first; r < chunks[c].second; ++r)
      for (const Prod& x : prods_of_r[r]) {
        const int l = pairs[x.p].left_op;
        const dmrg_su2_operator& A = left_ops[l];
        const dmrg_su2_operator& B = right_ops[r];
        const int a2 = A.out_sector[x.j], a = A.in_sector[x.j], b2 = B.out_sector[x.i], b = B.in_sector[x.i];
        const int64_t kp = pad8(W.ld[a]);
        const S1& e = need[r].at(x.i);
        outs[{a2, b2}].push_back({K + lpos.at({l, x.j}), T + e.off + rowoff[(size_t)a * nr + b],
                                  (int64_t)W.ld[a2] * kp, tlo, (int)kp, (int)mb[b], W.ld[a], kTransB, x.scale});
      }
    GemmBatchB b2;
    b2.shape = shapes.second;
    for (auto& kv : outs) {
      const int a2 = kv.first.first, bb2 = kv.first.second;
      const std::vector<GemmSegB>& g = kv.second;
      const int parts = (int)std::min<size_t>(n_parts, (g.size() + seg_per_part - 1) / seg_per_part);
      for (int j = 0; j < parts; ++j) {
        const size_t lo = g.size() * j / parts, hi = g.size() * (j + 1) / parts;
        const size_t s0 = b2.segs.size();
        for (size_t q = lo; q < hi; ++q) b2.segs.push_back(g[q]);
        b2.add_problem(Part + (int64_t)j * W.size + W.at(a2, bb2), 0, W.rd[bb2], W.ld[a2], W.rd[bb2], s0,
                       b2.segs.size(), 1);
      }
    }
    plan.n_segments += (int64_t)(b1.segs.size() + b2.segs.size());
    plan.s1b.emplace_back();
    upload_gemm_bf16(b1, plan.s1b.back());
    plan.s2b.emplace_back();
    upload_gemm_bf16(b2, plan.s2b.back());
  }
}

}  // namespace

std::unique_ptr<Su2Plan> su2_plan(const dmrg_su2_window& w, int n_left_ops, const dmrg_su2_operator* left_ops,
                                  int n_right_ops, const dmrg_su2_operator* right_ops, int n_pairs,
                                  const dmrg_su2_pair* pairs, int precision, int64_t ws_budget, hipStream_t s) {
  DMRG_REQUIRE(precision == DMRG_FP64 || precision == DMRG_BF16X3, kErrInvalidArg,
               "su2: precision must be DMRG_FP64 or DMRG_BF16X3");
  const Window W = parse(w);
  const int nl = (int)W.ln.size(), nr = (int)W.rn.size();
  DMRG_REQUIRE(n_left_ops >= 0 && n_right_ops >= 0 && (n_left_ops == 0 || left_ops) &&
                   (n_right_ops == 0 || right_ops),
               kErrInvalidArg, "su2: NULL operator array");
  DMRG_REQUIRE(n_pairs >= 0 && (n_pairs == 0 || pairs), kErrInvalidArg, "su2: NULL pair array");
  auto check_op = [&](const dmrg_su2_operator& o, int ns) {
    DMRG_REQUIRE(o.n_blocks >= 0 && (o.n_blocks == 0 || (o.out_sector && o.in_sector && o.offset && o.data)),
                 kErrInvalidArg, "su2: NULL operator array");
    for (int i = 0; i < o.n_blocks; ++i)
      DMRG_REQUIRE(o.out_sector[i] >= 0 && o.out_sector[i] < ns && o.in_sector[i] >= 0 && o.in_sector[i] < ns &&
                       o.offset[i] >= 0,
                   kErrInvalidArg, "su2: operator block sector out of range");
  };
  for (int i = 0; i < n_left_ops; ++i) check_op(left_ops[i], nl);
  for (int i = 0; i < n_right_ops; ++i) check_op(right_ops[i], nr);
  for (int p = 0; p < n_pairs; ++p) {
    const dmrg_su2_pair& q = pairs[p];
    DMRG_REQUIRE(q.left_op >= 0 && q.left_op < n_left_ops && q.right_op >= 0 && q.right_op < n_right_ops,
                 kErrInvalidArg, "su2: pair operator index out of range");
    DMRG_REQUIRE(q.two_k >= 0 && (q.parity == 0 || q.parity == 1), kErrInvalidArg,
                 "su2: pair rank must be >= 0 and parity 0 or 1");
  }
  auto plan = std::make_unique<Su2Plan>();
  plan->precision = precision;
  plan->psi_size = W.size;
  plan->psi.alloc((size_t)std::max<int64_t>(W.size, 1) * sizeof(double));

  // The stage-2 products: for each pair, each ket block (a, b) of psi, each
  // block A[a', a] of its left operator and B[b', b] of its right operator
  // with (a', b') a coupled block and a non-zero recoupling factor.
  std::vector<std::vector<Prod>> prods_of_r(n_right_ops);  // grouped by right operator
  std::map<std::tuple<int, int, int, int, int>, double> wcache;
  std::vector<std::vector<std::vector<int>>> lin(n_left_ops), rin(n_right_ops);
  for (int p = 0; p < n_pairs; ++p) {
    const dmrg_su2_pair& q = pairs[p];
    if (lin[q.left_op].empty()) lin[q.left_op] = by_in_sector(left_ops[q.left_op], nl);
    if (rin[q.right_op].empty()) rin[q.right_op] = by_in_sector(right_ops[q.right_op], nr);
    const dmrg_su2_operator& A = left_ops[q.left_op];
    const dmrg_su2_operator& B = right_ops[q.right_op];
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nr; ++b) {
        if (W.at(a, b) < 0) continue;
        for (int j : lin[q.left_op][a])
          for (int i : rin[q.right_op][b]) {
            const int a2 = A.out_sector[j], b2 = B.out_sector[i];
            if (W.at(a2, b2) < 0) continue;
            const auto key = std::make_tuple(W.ls[a2], W.rs[b2], W.ls[a], W.rs[b], q.two_k);
            auto it = wcache.find(key);
            if (it == wcache.end())
              it = wcache.emplace(key, recoupling(W.ls[a2], W.rs[b2], W.ls[a], W.rs[b], W.ts, q.two_k)).first;
            if (it->second == 0.0) continue;
            const double sign = (q.parity && (W.ln[a] & 1)) ? -1.0 : 1.0;
            prods_of_r[q.right_op].push_back({p, i, j, q.coef * sign * it->second});
          }
      }
  }
  // psi regrouped by right sector inside the plan: for each b the coupled
  // blocks (a, b) stacked by a into one (M_b x d_b) matrix, block (a, b) at
  // row rowoff(a, b); stage 1 then multiplies every needed row of a right
  // sector by a block of B in one product.
  std::vector<int64_t> boff(nr + 1, 0), rowoff((size_t)nl * nr, -1), mb(nr, 0);
  // (each block's rows start at a multiple of 8, the rows between are zero:
  // the split-BF16 products read k-ranges of 16-byte aligned rows)
  for (int b = 0; b < nr; ++b) {
    for (int a = 0; a < nl; ++a)
      if (W.at(a, b) >= 0) {
        rowoff[(size_t)a * nr + b] = mb[b];
        mb[b] += pad8(W.ld[a]);
      }
    boff[b + 1] = boff[b] + mb[b] * W.rd[b];
  }
  // Stage-1 products per right operator: block i of B -> the row range of
  // psi_b it multiplies (from the first to the last needed left sector) and
  // the workspace offset of T(r, i) (M_b x d_b').
  std::vector<std::map<int, S1>> need(n_right_ops);
  std::vector<int64_t> rsize(n_right_ops, 0);
  for (int r = 0; r < n_right_ops; ++r) {
    for (const Prod& x : prods_of_r[r]) {
      const int a = left_ops[pairs[x.p].left_op].in_sector[x.j];
      const int b = right_ops[r].in_sector[x.i];
      const int64_t r0 = rowoff[(size_t)a * nr + b], r1 = r0 + W.ld[a];
      S1& e = need[r][x.i];
      e.lo = e.lo < 0 ? r0 : std::min(e.lo, r0);
      e.hi = std::max(e.hi, r1);
    }
    for (auto& kv : need[r]) rsize[r] += mb[right_ops[r].in_sector[kv.first]] * W.rd[right_ops[r].out_sector[kv.first]];
  }
  std::vector<std::pair<int, int>> chunks;
  {
    int r0 = 0;
    int64_t acc = 0;
    for (int r = 0; r < n_right_ops; ++r) {
      if (rsize[r] == 0) continue;
      if (acc > 0 && acc + rsize[r] > ws_budget) {
        chunks.push_back({r0, r});
        r0 = r;
        acc = 0;
      }
      acc += rsize[r];
      plan->ws_doubles = std::max(plan->ws_doubles, acc);
    }
    if (acc > 0) chunks.push_back({r0, n_right_ops});
  }
  const bool f64 = precision == DMRG_FP64;
  if (f64) plan->ws.alloc((size_t)std::max<int64_t>(plan->ws_doubles, 1) * sizeof(double));
  double* T = plan->ws.as<double>();
  plan->psi_b.alloc((size_t)std::max<int64_t>(boff[nr], 1) * sizeof(double));
  const double* P = plan->psi.as<double>();
  double* Pb = plan->psi_b.as<double>();
  launch_fill(Pb, 0.0, boff[nr], s);  // the rows between blocks stay zero
  {
    std::vector<CopyTask> tasks;
    for (int a = 0; a < nl; ++a)
      for (int b = 0; b < nr; ++b)
        if (W.at(a, b) >= 0)
          tasks.push_back({P + W.at(a, b), Pb + boff[b] + rowoff[(size_t)a * nr + b] * W.rd[b], W.ld[a], W.rd[b],
                           W.rd[b], W.rd[b]});
    plan->n_regroup = (int)tasks.size();
    plan->regroup.alloc(std::max<size_t>(1, tasks.size()) * sizeof(CopyTask));
    if (!tasks.empty())
      DMRG_HIP(hipMemcpy(plan->regroup.p, tasks.data(), tasks.size() * sizeof(CopyTask), hipMemcpyHostToDevice));
  }
  // stage-1 workspace offsets, and the stage-2 products of every output
  // block (a', b') per chunk: W c (-1)^(p N_a) A[a', a] T
  std::vector<std::map<std::pair<int, int>, std::vector<GemmSeg>>> outs(chunks.size());
  size_t max_segs = 0;
  for (size_t c = 0; c < chunks.size(); ++c) {
    int64_t off = 0;
    for (int r = chunks[c].first; r < chunks[c].second; ++r)
      for (auto& kv : need[r]) {
        const int b = right_ops[r].in_sector[kv.first], b2 = right_ops[r].out_sector[kv.first];
        kv.second.off = off;
        off += mb[b] * W.rd[b2];
        plan->flops1 += 2.0 * (kv.second.hi - kv.second.lo) * W.rd[b] * W.rd[b2];
      }
    size_t nseg = 0;
    for (int r = chunks[c].first; r < chunks[c].second; ++r)
      for (const Prod& x : prods_of_r[r]) {
        const dmrg_su2_operator& A = left_ops[pairs[x.p].left_op];
        const dmrg_su2_operator& B = right_ops[r];
        const int a2 = A.out_sector[x.j], a = A.in_sector[x.j], b2 = B.out_sector[x.i], b = B.in_sector[x.i];
        auto& list = outs[c][{a2, b2}];
        if (f64) {
          const int64_t to = need[r].at(x.i).off + rowoff[(size_t)a * nr + b] * W.rd[b2];
          list.push_back({A.data + A.offset[x.j], T + to, W.ld[a], W.rd[b2], W.ld[a], 0, x.scale});
        } else {
          list.emplace_back();  // counted only: the BF16 lists are built from the products
        }
        plan->flops2 += 2.0 * W.ld[a2] * W.ld[a] * W.rd[b2];
        ++nseg;
      }
    max_segs = std::max(max_segs, nseg);
  }
  // Few output blocks with long product lists would leave most compute
  // units idle: each output's list is split into up to n_parts pieces of
  // about seg_per_part products, piece j summed into partial sum j, and the
  // partial sums added in a fixed order at the end.
  size_t per_launch = kSu2PartsPerLaunch;
  if (const char* e = std::getenv("DMRG_SU2_PARTS")) per_launch = std::max<long long>(1, std::atoll(e));
  const size_t seg_per_part = std::max<size_t>(16, (max_segs + per_launch - 1) / per_launch);
  int n_parts = 1;
  for (auto& oc : outs)
    for (auto& kv : oc) n_parts = std::max<int>(n_parts, (int)((kv.second.size() + seg_per_part - 1) / seg_per_part));
  n_parts = (int)std::min<int64_t>(
      {(int64_t)n_parts, (int64_t)kSu2MaxParts, std::max<int64_t>(1, kSu2PartialBudget / std::max<int64_t>(1, W.size))});
  plan->n_parts = n_parts;
  plan->part.alloc((size_t)std::max<int64_t>(1, (int64_t)n_parts * W.size) * sizeof(double));
  {
    std::vector<double> ones(n_parts, 1.0);
    plan->ones.alloc(n_parts * sizeof(double));
    DMRG_HIP(hipMemcpy(plan->ones.p, ones.data(), n_parts * sizeof(double), hipMemcpyHostToDevice));
  }
  double* Part = plan->part.as<double>();
  const auto tiles = su2_tiles();
  if (precision == DMRG_BF16X3) {
    outs.clear();
    build_bf16(*plan, W, left_ops, right_ops, prods_of_r, pairs, need, chunks, mb, boff, rowoff, seg_per_part, s);
    return plan;
  }
  for (size_t c = 0; c < chunks.size(); ++c) {
    // stage 1: rows [lo, hi) of T(r, i) = psi_b B_r[i]^T (M_b x d_b'),
    // psi_b holding the blocks (a, b) stacked by a
    GemmBatch b1;
    b1.tile = tiles.first.first;
    b1.tile_n = tiles.first.second;
    for (int r = chunks[c].first; r < chunks[c].second; ++r) {
      const dmrg_su2_operator& B = right_ops[r];
      for (auto& kv : need[r]) {
        const int i = kv.first;
        const S1& e = kv.second;
        const int b2 = B.out_sector[i], b = B.in_sector[i];
        const size_t s0 = b1.segs.size();
        b1.segs.push_back({Pb + boff[b] + e.lo * W.rd[b], B.data + B.offset[i], W.rd[b], W.rd[b], W.rd[b],
                           kTransB, 1.0});
        b1.add_problem(T + e.off + e.lo * W.rd[b2], W.rd[b2], (int)(e.hi - e.lo), W.rd[b2], s0, s0 + 1, 0);
      }
    }
    // stage 2: each output's products in contiguous pieces, one per partial sum
    GemmBatch b2;
    b2.tile = tiles.second.first;
    b2.tile_n = tiles.second.second;
    for (auto& kv : outs[c]) {
      const int a2 = kv.first.first, bb2 = kv.first.second;
      const std::vector<GemmSeg>& g = kv.second;
      const int parts = (int)std::min<size_t>(n_parts, (g.size() + seg_per_part - 1) / seg_per_part);
      for (int j = 0; j < parts; ++j) {
        const size_t lo = g.size() * j / parts, hi = g.size() * (j + 1) / parts;
        const size_t s0 = b2.segs.size();
        for (size_t q = lo; q < hi; ++q) b2.segs.push_back(g[q]);
        b2.add_problem(Part + (int64_t)j * W.size + W.at(a2, bb2), W.rd[bb2], W.ld[a2], W.rd[bb2], s0,
                       b2.segs.size(), 1);
      }
    }
    plan->n_segments += (int64_t)(b1.segs.size() + b2.segs.size());
    plan->s1.emplace_back();
    upload_gemm(b1, plan->s1.back());
    plan->s2.emplace_back();
    upload_gemm(b2, plan->s2.back());
    outs[c].clear();
  }
  (void)s;
  return plan;
}

void su2_run(Su2Plan& p, const double* psi, double* sigma, hipStream_t s) {
  DMRG_REQUIRE(psi && sigma, kErrInvalidArg, "su2: NULL psi or sigma");
  if (p.psi_size == 0) return;
  // psi is copied into the plan first, so sigma may be the same buffer
  double* P = p.psi.as<double>();
  DMRG_HIP(hipMemcpyAsync(P, psi, (size_t)p.psi_size * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_copy_tasks(p.regroup.as<CopyTask>(), p.n_regroup, false, s);
  launch_fill(p.part.as<double>(), 0.0, (int64_t)p.n_parts * p.psi_size, s);
  if (p.precision == DMRG_BF16X3) {
    launch_pack_bf16(p.psi_pack_ops.as<PackOp>(), p.n_psi_pack, p.psi_pack_chunks, p.psi_pack.as<uint16_t>(), s);
    for (size_t c = 0; c < p.s1b.size(); ++c) {
      launch_gemm_bf16(p.s1b[c], true, kOutBf16, 1, s);
      launch_gemm_bf16(p.s2b[c], true, kOutF64, 2, s);
    }
  } else {
    for (size_t c = 0; c < p.s1.size(); ++c) {
      launch_gemm_f64(p.s1[c], s, 1);
      launch_gemm_f64(p.s2[c], s, 2);
    }
  }
  launch_lincomb(sigma, p.part.as<double>(), p.psi_size, p.n_parts, p.ones.as<double>(), p.psi_size, 0.0, s);
}

}  // namespace dmrg
