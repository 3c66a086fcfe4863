// Two-site truncation and move of the window (standard two-site DMRG step:
// the reduced density matrix of the optimised window is diagonalised sector
// by sector, the D largest eigenvalues over all sectors are kept, the kept
// eigenvectors become the new site tensor, and the rest of the window is
// carried into the guess for the next window; White 1996).
//
// The window psi is reshaped, per middle-bond sector q = Q_l + Q_n1, into
// M_q[(l, n1), (n2, r)].  Moving right, rho = M M^T gives the new
// left-canonical A_i; moving left, rho = M^T M gives the new right-canonical
// B_{i+1}.  rho is formed by the FP64 MFMA GEMM, diagonalised by rocSOLVER
// dsyevd, and the discarded weight sum_{discarded} lambda / sum lambda is the
// truncation error of the Method section.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <map>
#include <numeric>
#include <tuple>

#include "truncate.h"

namespace dmrg {

namespace {

struct Sector {
  QN q;
  int nrow = 0, ncol = 0;
  std::map<std::pair<int, int>, int> row_off;  // (l, n1) -> row
  std::map<std::pair<int, int>, int> col_off;  // (n2, r) -> col
  DevBuf M, rho, evec, eval;
  std::vector<double> lam;  // ascending
  int kept = 0;
};

void check_rb(rocblas_status st, const char* what) {
  DMRG_REQUIRE(st == rocblas_status_success, kErrHip, std::string("rocSOLVER/rocBLAS failure in ") + what);
}

}  // namespace

struct SolverHandle {
  rocblas_handle h = nullptr;
  ~SolverHandle() {
    if (h) rocblas_destroy_handle(h);
  }
};

TruncResult truncate_and_move(Mps& m, int window, const double* psi, int dir, int max_d,
                              double cutoff, DevBuf& next_psi, DevBuf& scratch, hipStream_t s) {
  const int i = window, K = m.K;
  DMRG_REQUIRE(dir == 1 || dir == -1, kErrInvalidArg, "truncate: direction must be +1 or -1");
  DMRG_REQUIRE(!(dir == 1 && i + 1 > K - 2), kErrInvalidArg, "truncate: cannot move right from the last window");
  DMRG_REQUIRE(!(dir == -1 && i == 0), kErrInvalidArg, "truncate: cannot move left from the first window");
  DMRG_REQUIRE(max_d >= 1, kErrInvalidArg, "truncate: max bond dimension must be >= 1");
  const Bond& bl = m.bonds[i];
  const Bond& br = m.bonds[i + 2];
  PsiLayout ps;
  ps.build(bl, br);
  // ---- sectors of the middle bond ------------------------------------------
  std::map<QN, Sector> sec;
  for (size_t l = 0; l < bl.size(); ++l)
    for (int n1 = 0; n1 < 4; ++n1) {
      const QN q = bl.q[l] + kSiteQN[n1];
      bool any = false;
      for (int n2 = 0; n2 < 4 && !any; ++n2) any = br.find(q + kSiteQN[n2]) >= 0;
      if (!any) continue;
      Sector& S = sec[q];
      S.q = q;
      S.row_off[{(int)l, n1}] = S.nrow;
      S.nrow += bl.d[l];
    }
  for (auto& kv : sec) {
    Sector& S = kv.second;
    for (int n2 = 0; n2 < 4; ++n2) {
      const int r = br.find(S.q + kSiteQN[n2]);
      if (r < 0) continue;
      S.col_off[{n2, r}] = S.ncol;
      S.ncol += br.d[r];
    }
  }
  // gather M_q from psi
  std::vector<CopyTask> gather;
  for (auto& kv : sec) {
    Sector& S = kv.second;
    S.M.alloc((size_t)std::max(1, S.nrow * S.ncol) * sizeof(double));
    launch_fill(S.M.as<double>(), 0.0, (int64_t)S.nrow * S.ncol, s);
  }
  for (size_t r = 0; r < br.size(); ++r)
    for (auto& kv : ps.row_of[r]) {
      const int l = kv.first.first, n = kv.first.second, n1 = n >> 2, n2 = n & 3;
      Sector& S = sec.at(bl.q[l] + kSiteQN[n1]);
      const int ro = S.row_off.at({l, n1}), co = S.col_off.at({n2, (int)r});
      gather.push_back({psi + ps.off[r] + kv.second * br.d[r],
                        S.M.as<double>() + (int64_t)ro * S.ncol + co, bl.d[l], br.d[r], br.d[r], S.ncol});
    }
  DevBuf gt(std::max<size_t>(1, gather.size()) * sizeof(CopyTask));
  DMRG_HIP(hipMemcpyAsync(gt.p, gather.data(), gather.size() * sizeof(CopyTask), hipMemcpyHostToDevice, s));
  launch_copy_tasks(gt.as<CopyTask>(), (int)gather.size(), false, s);
  // ---- density matrices and eigen-decompositions ------------------------------
  SolverHandle sh;
  check_rb(rocblas_create_handle(&sh.h), "create_handle");
  check_rb(rocblas_set_stream(sh.h, s), "set_stream");
  DevBuf info(sizeof(rocblas_int) * 2);
  double total = 0;
  struct Cand {
    double lam;
    int sidx, j;
  };
  std::vector<Cand> cand;
  int sidx = 0;
  std::vector<Sector*> order;
  for (auto& kv : sec) order.push_back(&kv.second);
  for (Sector* Sp : order) {
    Sector& S = *Sp;
    const int n = dir > 0 ? S.nrow : S.ncol;
    S.rho.alloc((size_t)std::max(1, n * n) * sizeof(double));
    GemmBatch b;
    if (dir > 0)  // rho = M M^T
      b.segs.push_back({S.M.p, S.M.p, S.ncol, S.ncol, S.ncol, kTransB, 1.0});
    else  // rho = M^T M
      b.segs.push_back({S.M.p, S.M.p, S.ncol, S.ncol, S.nrow, kTransA, 1.0});
    b.add_problem(S.rho.p, n, n, n, 0, 1, 0);
    launch_gemm_f64(b, s);
    S.eval.alloc((size_t)std::max(1, n) * sizeof(double));
    DevBuf work((size_t)std::max(1, n) * sizeof(double));
    check_rb(rocsolver_dsyevd(sh.h, rocblas_evect_original, rocblas_fill_upper, n, S.rho.as<double>(), n,
                              S.eval.as<double>(), work.as<double>(), info.as<rocblas_int>()),
             "dsyevd");
    S.lam.resize(n);
    DMRG_HIP(hipMemcpyAsync(S.lam.data(), S.eval.p, n * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    rocblas_int inf = 0;
    DMRG_HIP(hipMemcpy(&inf, info.p, sizeof(inf), hipMemcpyDeviceToHost));
    DMRG_REQUIRE(inf == 0, kErrHip, "truncate: dsyevd did not converge");
    for (int j = 0; j < n; ++j) {
      const double lv = std::max(0.0, S.lam[j]);
      total += lv;
      cand.push_back({lv, sidx, j});
    }
    ++sidx;
  }
  // ---- global selection: largest weights; ties by (sector, index) -----------
  std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
    if (a.lam != b.lam) return a.lam > b.lam;
    if (a.sidx != b.sidx) return a.sidx < b.sidx;
    return a.j > b.j;
  });
  TruncResult res;
  const double lam_max = cand.empty() ? 0.0 : cand[0].lam;
  double kept_w = 0;
  for (size_t c = 0; c < cand.size(); ++c) {
    const bool keep = (int)c < max_d && cand[c].lam > std::max(cutoff, 1e-14) * std::max(lam_max, 1e-300);
    if (keep) {
      order[cand[c].sidx]->kept++;
      kept_w += cand[c].lam;
    }
  }
  DMRG_REQUIRE(kept_w > 0, kErrState, "truncate: nothing to keep (psi is zero)");
  res.trunc_err = total > 0 ? std::max(0.0, (total - kept_w) / total) : 0.0;
  // dsyevd returns ascending eigenvalues, so the kept ones are the last columns
  // of the (column-major) eigenvector matrix of each sector.
  // ---- new middle bond -----------------------------------------------------------
  Bond nb;
  for (Sector* Sp : order)
    if (Sp->kept > 0) {
      nb.q.push_back(Sp->q);
      nb.d.push_back(Sp->kept);
    }
  nb.finish();
  res.kept = (int)nb.total;
  // ---- new site tensor and next-window psi --------------------------------------
  if (dir > 0) {
    // A_i: blocks (l, n1) -> q, A[a][k] = evec[(j0 + k) * nrow + row(l, n1) + a]
    SiteTensor A;
    A.off.assign(4 * bl.size(), -1);
    int64_t tot = 0;
    for (size_t l = 0; l < bl.size(); ++l)
      for (int n1 = 0; n1 < 4; ++n1) {
        const int qi = nb.find(bl.q[l] + kSiteQN[n1]);
        if (qi < 0) continue;
        A.off[4 * l + n1] = tot;
        tot += (int64_t)bl.d[l] * nb.d[qi];
      }
    A.data.alloc((size_t)std::max<int64_t>(1, tot) * sizeof(double));
    std::vector<CopyTask> at;
    for (Sector* Sp : order) {
      Sector& S = *Sp;
      if (!S.kept) continue;
      const int j0 = S.nrow - S.kept;
      for (auto& ro : S.row_off) {
        const int l = ro.first.first, n1 = ro.first.second;
        at.push_back({S.rho.as<double>() + (int64_t)j0 * S.nrow + ro.second,
                      A.data.as<double>() + A.off[4 * l + n1], S.kept, bl.d[l], S.nrow, S.kept});
      }
    }
    DevBuf atd(std::max<size_t>(1, at.size()) * sizeof(CopyTask));
    DMRG_HIP(hipMemcpyAsync(atd.p, at.data(), at.size() * sizeof(CopyTask), hipMemcpyHostToDevice, s));
    launch_copy_tasks(atd.as<CopyTask>(), (int)at.size(), true, s);
    // C_q = U_kept^T M_q (kept x ncol), then psi'((q,k), n2, n3 -> r') = C[:, (n2, r)] B_{i+2}(r, n3)
    const Bond& b3 = m.bonds[i + 3];
    const SiteTensor& B2 = m.site[i + 2];
    DMRG_REQUIRE(!B2.off.empty(), kErrState, "truncate: site i+2 tensor missing");
    PsiLayout np;
    np.build(nb, b3);
    next_psi.alloc((size_t)std::max<int64_t>(1, np.size) * sizeof(double));
    launch_fill(next_psi.as<double>(), 0.0, np.size, s);
    std::map<QN, DevBuf> C;
    GemmBatch bc;
    for (Sector* Sp : order) {
      Sector& S = *Sp;
      if (!S.kept) continue;
      DevBuf& c = C[S.q];
      c.alloc((size_t)S.kept * S.ncol * sizeof(double));
      const int j0 = S.nrow - S.kept;
      const size_t s0 = bc.segs.size();
      bc.segs.push_back({S.rho.as<double>() + (int64_t)j0 * S.nrow, S.M.p, S.nrow, S.ncol, S.nrow, 0, 1.0});
      bc.add_problem(c.p, S.ncol, S.kept, S.ncol, s0, s0 + 1, 0);
    }
    launch_gemm_f64(bc, s);
    GemmBatch bp;
    for (size_t rp = 0; rp < b3.size(); ++rp)
      for (auto& kv : np.row_of[rp]) {
        const int q = kv.first.first, n = kv.first.second, n2 = n >> 2, n3 = n & 3;
        const QN qq = nb.q[q];
        const int r = br.find(qq + kSiteQN[n2]);
        if (r < 0) continue;
        Sector& S = sec.at(qq);
        auto co = S.col_off.find({n2, r});
        const int64_t ob = B2.off[4 * r + n3];
        if (co == S.col_off.end() || ob < 0) continue;
        const size_t s0 = bp.segs.size();
        bp.segs.push_back({C.at(qq).as<double>() + co->second, B2.data.as<double>() + ob, S.ncol, b3.d[rp],
                           br.d[r], 0, 1.0});
        bp.add_problem(next_psi.as<double>() + np.off[rp] + kv.second * b3.d[rp], b3.d[rp], nb.d[q], b3.d[rp],
                       s0, s0 + 1, 0);
      }
    launch_gemm_f64(bp, s);
    DMRG_HIP(hipStreamSynchronize(s));
    m.site[i] = std::move(A);
    m.bonds[i + 1] = nb;
    m.site[i + 1] = SiteTensor();
    m.site[i + 2] = SiteTensor();
    res.next_size = np.size;
  } else {
    // B_{i+1}: blocks (q, n2) -> r, B[k][b] = evec[(j0 + k) * ncol + col(n2, r) + b]
    SiteTensor B;
    B.off.assign(4 * nb.size(), -1);
    int64_t tot = 0;
    for (size_t q = 0; q < nb.size(); ++q)
      for (int n2 = 0; n2 < 4; ++n2) {
        const int r = br.find(nb.q[q] + kSiteQN[n2]);
        if (r < 0) continue;
        B.off[4 * q + n2] = tot;
        tot += (int64_t)nb.d[q] * br.d[r];
      }
    B.data.alloc((size_t)std::max<int64_t>(1, tot) * sizeof(double));
    std::vector<CopyTask> bt;
    for (size_t q = 0; q < nb.size(); ++q) {
      Sector& S = sec.at(nb.q[q]);
      const int j0 = S.ncol - S.kept;
      for (auto& co : S.col_off) {
        const int n2 = co.first.first, r = co.first.second;
        bt.push_back({S.rho.as<double>() + (int64_t)j0 * S.ncol + co.second,
                      B.data.as<double>() + B.off[4 * q + n2], S.kept, br.d[r], S.ncol, br.d[r]});
      }
    }
    DevBuf btd(std::max<size_t>(1, bt.size()) * sizeof(CopyTask));
    DMRG_HIP(hipMemcpyAsync(btd.p, bt.data(), bt.size() * sizeof(CopyTask), hipMemcpyHostToDevice, s));
    launch_copy_tasks(btd.as<CopyTask>(), (int)bt.size(), false, s);
    // C_q = M_q V_kept (nrow x kept); psi'((l', n0, n1) -> (q,k)) = A_{i-1}(l', n0 -> l) C[(l, n1), :]
    const Bond& b0 = m.bonds[i - 1];
    const SiteTensor& A1 = m.site[i - 1];
    DMRG_REQUIRE(!A1.off.empty(), kErrState, "truncate: site i-1 tensor missing");
    PsiLayout np;
    np.build(b0, nb);
    next_psi.alloc((size_t)std::max<int64_t>(1, np.size) * sizeof(double));
    launch_fill(next_psi.as<double>(), 0.0, np.size, s);
    std::map<QN, DevBuf> C;
    GemmBatch bc;
    for (size_t q = 0; q < nb.size(); ++q) {
      Sector& S = sec.at(nb.q[q]);
      DevBuf& c = C[S.q];
      c.alloc((size_t)S.nrow * S.kept * sizeof(double));
      const int j0 = S.ncol - S.kept;
      const size_t s0 = bc.segs.size();
      bc.segs.push_back({S.M.p, S.rho.as<double>() + (int64_t)j0 * S.ncol, S.ncol, S.ncol, S.ncol, kTransB, 1.0});
      bc.add_problem(c.p, S.kept, S.nrow, S.kept, s0, s0 + 1, 0);
    }
    launch_gemm_f64(bc, s);
    GemmBatch bp;
    for (size_t q = 0; q < nb.size(); ++q)
      for (auto& kv : np.row_of[q]) {
        const int lp = kv.first.first, n = kv.first.second, n0 = n >> 2, n1 = n & 3;
        const int l = bl.find(b0.q[lp] + kSiteQN[n0]);
        if (l < 0) continue;
        const int64_t oa = A1.off[4 * lp + n0];
        Sector& S = sec.at(nb.q[q]);
        auto ro = S.row_off.find({l, n1});
        if (oa < 0 || ro == S.row_off.end()) continue;
        const size_t s0 = bp.segs.size();
        bp.segs.push_back({A1.data.as<double>() + oa, C.at(S.q).as<double>() + (int64_t)ro->second * S.kept,
                           bl.d[l], S.kept, bl.d[l], 0, 1.0});
        bp.add_problem(next_psi.as<double>() + np.off[q] + kv.second * nb.d[q], nb.d[q], b0.d[lp], nb.d[q],
                       s0, s0 + 1, 0);
      }
    launch_gemm_f64(bp, s);
    DMRG_HIP(hipStreamSynchronize(s));
    m.site[i + 1] = std::move(B);
    m.bonds[i + 1] = nb;
    m.site[i - 1] = SiteTensor();
    m.site[i] = SiteTensor();
    res.next_size = np.size;
  }
  return res;
}

}  // namespace dmrg
