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
// of the U(1) sigma: stage 1 forms T = psi[a, b] B[b', b]^T once per right
// operator block and left sector (NT products), stage 2 accumulates
// W c (-1)^(p N_a) A[a', a] T into each output block (NN products), every
// output block one problem of the grouped GEMM with its segments.
#include "su2.h"

#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "common.h"
#include "gemm.h"

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
  std::map<std::pair<int, int>, int64_t> off;  // coupled block (a, b) -> element offset
  int64_t size = 0;
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
  for (int a = 0; a < w.n_left; ++a)
    for (int b = 0; b < w.n_right; ++b)
      if (W.ln[a] + W.rn[b] == W.n && triangle(W.ls[a], W.rs[b], W.ts)) {
        W.off[{a, b}] = W.size;
        W.size += (int64_t)W.ld[a] * W.rd[b];
      }
  return W;
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

void su2_sigma(hipStream_t s, const dmrg_su2_window& w, int n_left_ops, const dmrg_su2_operator* left_ops,
               int n_right_ops, const dmrg_su2_operator* right_ops, int n_pairs, const dmrg_su2_pair* pairs,
               const double* psi, double* sigma) {
  const Window W = parse(w);
  DMRG_REQUIRE(psi && sigma, kErrInvalidArg, "su2: NULL psi or sigma");
  DMRG_REQUIRE(n_pairs >= 0 && (n_pairs == 0 || pairs), kErrInvalidArg, "su2: NULL pair array");
  auto check_op = [&](const dmrg_su2_operator& o, int ns) {
    DMRG_REQUIRE(o.n_blocks >= 0 && (o.n_blocks == 0 || (o.out_sector && o.in_sector && o.offset && o.data)),
                 kErrInvalidArg, "su2: NULL operator array");
    for (int i = 0; i < o.n_blocks; ++i)
      DMRG_REQUIRE(o.out_sector[i] >= 0 && o.out_sector[i] < ns && o.in_sector[i] >= 0 && o.in_sector[i] < ns &&
                       o.offset[i] >= 0,
                   kErrInvalidArg, "su2: operator block sector out of range");
  };
  for (int i = 0; i < n_left_ops; ++i) check_op(left_ops[i], (int)W.ln.size());
  for (int i = 0; i < n_right_ops; ++i) check_op(right_ops[i], (int)W.rn.size());
  for (int p = 0; p < n_pairs; ++p) {
    const dmrg_su2_pair& q = pairs[p];
    DMRG_REQUIRE(q.left_op >= 0 && q.left_op < n_left_ops && q.right_op >= 0 && q.right_op < n_right_ops,
                 kErrInvalidArg, "su2: pair operator index out of range");
    DMRG_REQUIRE(q.two_k >= 0 && (q.parity == 0 || q.parity == 1), kErrInvalidArg,
                 "su2: pair rank must be >= 0 and parity 0 or 1");
  }
  launch_fill(sigma, 0.0, W.size, s);
  if (W.size == 0 || n_pairs == 0) {
    DMRG_HIP(hipStreamSynchronize(s));
    return;
  }
  // stage 1: T[r, block i of B_r, a] = psi[a, b] B_r[b', b]^T (d_a x d_b'), for
  // every right operator used by a pair, every block and left sector a whose
  // (a, b) and some (a', b') are coupled blocks
  std::vector<char> used_r(n_right_ops, 0);
  for (int p = 0; p < n_pairs; ++p) used_r[pairs[p].right_op] = 1;
  std::map<std::tuple<int, int, int>, int64_t> toff;  // (r, block, a) -> workspace offset
  int64_t wsize = 0;
  const int nl = (int)W.ln.size();
  for (int r = 0; r < n_right_ops; ++r) {
    if (!used_r[r]) continue;
    const dmrg_su2_operator& B = right_ops[r];
    for (int i = 0; i < B.n_blocks; ++i) {
      const int b2 = B.out_sector[i], b = B.in_sector[i];
      for (int a = 0; a < nl; ++a) {
        if (!W.off.count({a, b})) continue;
        toff[{r, i, a}] = wsize;
        wsize += (int64_t)W.ld[a] * W.rd[b2];
      }
    }
  }
  DevBuf ws((size_t)std::max<int64_t>(wsize, 1) * sizeof(double));
  double* T = ws.as<double>();
  {
    GemmBatch b1;
    for (auto& kv : toff) {
      const int r = std::get<0>(kv.first), i = std::get<1>(kv.first), a = std::get<2>(kv.first);
      const dmrg_su2_operator& B = right_ops[r];
      const int b2 = B.out_sector[i], b = B.in_sector[i];
      const size_t s0 = b1.segs.size();
      b1.segs.push_back({psi + W.off.at({a, b}), B.data + B.offset[i], W.rd[b], W.rd[b], W.rd[b], kTransB, 1.0});
      b1.add_problem(T + kv.second, W.rd[b2], W.ld[a], W.rd[b2], s0, s0 + 1, 0);
    }
    launch_gemm_f64(b1, s);
  }
  // stage 2: per output block (a', b'), the segments W c (-1)^(p N_a) A[a', a] T
  std::map<std::pair<int, int>, std::vector<GemmSeg>> outs;
  for (int p = 0; p < n_pairs; ++p) {
    const dmrg_su2_pair& q = pairs[p];
    const dmrg_su2_operator& A = left_ops[q.left_op];
    const dmrg_su2_operator& B = right_ops[q.right_op];
    for (int i = 0; i < B.n_blocks; ++i) {
      const int b2 = B.out_sector[i], b = B.in_sector[i];
      for (int j = 0; j < A.n_blocks; ++j) {
        const int a2 = A.out_sector[j], a = A.in_sector[j];
        if (!W.off.count({a, b}) || !W.off.count({a2, b2})) continue;
        const double wc = recoupling(W.ls[a2], W.rs[b2], W.ls[a], W.rs[b], W.ts, q.two_k);
        if (wc == 0.0) continue;
        const double sign = (q.parity && (W.ln[a] & 1)) ? -1.0 : 1.0;
        const int64_t to = toff.at({q.right_op, i, a});
        outs[{a2, b2}].push_back(
            {A.data + A.offset[j], T + to, W.ld[a], W.rd[b2], W.ld[a], 0, q.coef * sign * wc});
      }
    }
  }
  GemmBatch b2;
  for (auto& kv : outs) {
    const int a2 = kv.first.first, bb2 = kv.first.second;
    const size_t s0 = b2.segs.size();
    for (const GemmSeg& g : kv.second) b2.segs.push_back(g);
    b2.add_problem(sigma + W.off.at({a2, bb2}), W.rd[bb2], W.ld[a2], W.rd[bb2], s0, b2.segs.size(), 1);
  }
  launch_gemm_f64(b2, s);
  DMRG_HIP(hipStreamSynchronize(s));  // the workspace is released on return
}

}  // namespace dmrg
