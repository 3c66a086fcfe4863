// Davidson eigensolver for the lowest eigenpair of H_eff (Davidson 1975) with
// the diagonal preconditioner and a precision ladder for the sigma products.
//
// Vectors live on the device in FP64; the subspace matrices (k <= 64) are
// diagonalised on the device in FP64 (rocSOLVER dsyevj), and their
// eigenvectors are copied to the host, which picks the Ritz pair and the
// restart combinations.  Each ladder stage
// uses one sigma precision until the residual norm drops below the stage
// threshold, reaches the floor that precision allows, or stalls; the
// subspace is then restarted from the current Ritz vector with sigma
// recomputed in the next precision.  The last stage is FP64, and the returned
// energy is the FP64 Rayleigh quotient.  With residual refinement, the FP64
// stage takes its correction vectors from inexact Jacobi-Davidson solves on
// the previous stage's precision (below).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include <rocsolver/rocsolver.h>

#include "davidson.h"

namespace dmrg {

namespace {
// Relative error of a sigma product per precision, as measured against the
// FP64 sigma (split-BF16x3 1.3e-6 .. 1.4e-6 at CAS(22,22) and CAS(54,36);
// BF16 products carry 2^-8 per operand), with margin.
double sigma_rel_error(int precision) {
  switch (precision) {
    case 1: return 4e-3;   // BF16
    case 2: return 3e-6;   // split-BF16x3
    case 3: return 1e-13;  // Ozaki, 47 bits
    default: return 0.0;   // FP64
  }
}
constexpr double kFloorFactor = 3.0;
constexpr int kStallWindow = 10;
// Residual refinement: relative reduction of the correction equation's
// residual that ends an inner solve, and the inner iterations allowed.
constexpr double kRefineEta = 1e-2;
constexpr int kRefineInner = 60;
}  // namespace

void launch_extract_diag(const DiagTask* tasks, int ntasks, hipStream_t s);
void launch_heff_diag(double* out, int64_t rows, int dr, const int64_t* rowinfo, int64_t offR,
                      int npairs, const double* yd, const double* Ld, int64_t DL,
                      const double* Zd, int64_t DR, hipStream_t s);
void launch_precondition(double* t, const double* r, const double* d, double theta, int64_t n,
                         hipStream_t s);

// ---- diagonal of H_eff (a sum over pairs with diagonal blocks) ------------
void build_diagonal(SigmaPlan& plan, const Bond& bl, const Bond& br, hipStream_t s) {
  const PsiLayout& ps = plan.psi;
  std::vector<int> use;
  for (size_t k = 0; k < plan.pairs.size(); ++k) {
    const SigmaPair& p = plan.pairs[k];
    if (!(p.L.lay->dq == QN{0, 0})) continue;
    if (p.z >= 0 && !(plan.zops[p.z].lay->dq == QN{0, 0})) continue;
    bool any = false;
    for (int n = 0; n < 16; ++n) any = any || p.y.m[n][n] != 0;
    if (any) use.push_back((int)k);
  }
  const int P = (int)use.size();
  const int64_t DL = bl.total, DR = br.total;
  DevBuf yd((size_t)std::max(1, P) * 16 * sizeof(double));
  DevBuf Ld((size_t)std::max<int64_t>(1, (int64_t)P * DL) * sizeof(double));
  DevBuf Zd((size_t)std::max<int64_t>(1, (int64_t)P * DR) * sizeof(double));
  launch_fill(Ld.as<double>(), 0.0, (int64_t)P * DL, s);
  launch_fill(Zd.as<double>(), 0.0, (int64_t)P * DR, s);
  std::vector<double> hy((size_t)P * 16);
  std::vector<DiagTask> tasks;
  for (int q = 0; q < P; ++q) {
    const SigmaPair& p = plan.pairs[use[q]];
    for (int n = 0; n < 16; ++n) hy[(size_t)q * 16 + n] = p.y.m[n][n];
    for (auto& b : p.L.lay->blk)
      if (b.r == b.c) tasks.push_back({p.L.data + b.off, Ld.as<double>() + (int64_t)q * DL + bl.off[b.c], b.dc, b.ld});
    if (p.z >= 0) {
      for (auto& b : plan.zops[p.z].lay->blk)
        if (b.r == b.c) tasks.push_back({plan.zops[p.z].data + b.off, Zd.as<double>() + (int64_t)q * DR + br.off[b.c], b.dc, b.ld});
    } else {
      launch_fill(Zd.as<double>() + (int64_t)q * DR, 1.0, DR, s);
    }
  }
  DMRG_HIP(hipMemcpy(yd.p, hy.data(), hy.size() * sizeof(double), hipMemcpyHostToDevice));
  DevBuf dt((size_t)std::max<size_t>(1, tasks.size()) * sizeof(DiagTask));
  DMRG_HIP(hipMemcpy(dt.p, tasks.data(), tasks.size() * sizeof(DiagTask), hipMemcpyHostToDevice));
  launch_extract_diag(dt.as<DiagTask>(), (int)tasks.size(), s);
  // row info: (global left state, site index n) of every psi row
  std::vector<int64_t> rowinfo;
  std::vector<int64_t> rowbase(br.size(), 0);
  for (size_t r = 0; r < br.size(); ++r) {
    rowbase[r] = (int64_t)rowinfo.size();
    std::vector<int64_t> rows(ps.rows_of[r] * 2, 0);
    for (auto& kv : ps.row_of[r]) {
      const int l = kv.first.first, n = kv.first.second;
      for (int a = 0; a < bl.d[l]; ++a) {
        rows[2 * (kv.second + a)] = bl.off[l] + a;
        rows[2 * (kv.second + a) + 1] = n;
      }
    }
    rowinfo.insert(rowinfo.end(), rows.begin(), rows.end());
  }
  DevBuf ri((size_t)std::max<size_t>(1, rowinfo.size()) * sizeof(int64_t));
  DMRG_HIP(hipMemcpy(ri.p, rowinfo.data(), rowinfo.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  plan.diag.alloc((size_t)std::max<int64_t>(1, ps.size) * sizeof(double));
  for (size_t r = 0; r < br.size(); ++r) {
    if (ps.rows_of[r] == 0) continue;
    launch_heff_diag(plan.diag.as<double>() + ps.off[r], ps.rows_of[r], br.d[r],
                     ri.as<int64_t>() + rowbase[r], br.off[r], P, yd.as<double>(),
                     Ld.as<double>(), DL, Zd.as<double>(), DR, s);
  }
  DMRG_HIP(hipStreamSynchronize(s));
}

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int davidson(SigmaPlan& plan, double* psi, const DavidsonOpts& o, DavidsonResult& res,
             hipStream_t s) {
  const int64_t n = plan.psi.size;
  DMRG_REQUIRE(n > 0, kErrShape, "davidson: empty window");
  const int kmax = std::max(3, std::min(o.max_subspace, 64));
  const double t_start = now_ms();
  res = DavidsonResult();
  DevBuf Vb((size_t)kmax * n * sizeof(double)), Wb((size_t)kmax * n * sizeof(double));
  DevBuf ub(n * sizeof(double)), wb(n * sizeof(double)), rb(n * sizeof(double)),
      tb(n * sizeof(double)), hb(64 * sizeof(double)), cb(128 * sizeof(double)),
      auxb(n * sizeof(double));
  double* aux = auxb.as<double>();
  double *V = Vb.as<double>(), *W = Wb.as<double>(), *u = ub.as<double>(), *w = wb.as<double>(),
         *r = rb.as<double>(), *t = tb.as<double>(), *h = hb.as<double>(), *cc = cb.as<double>();
  const double* d = plan.diag.as<double>();
  double dmin = 0;
  {
    std::vector<double> dh((size_t)n);
    DMRG_HIP(hipMemcpyAsync(dh.data(), d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    dmin = n > 0 ? *std::min_element(dh.begin(), dh.end()) : 0.0;
  }
  std::vector<double> G((size_t)kmax * kmax, 0.0), hh(64);
  // subspace eigenproblem on the device: G_k (k x k) -> eigenvalues ascending
  // in ev, eigenvector j in column j of Y (Y[i * k + j] = component i)
  struct Solver {
    rocblas_handle h = nullptr;
    ~Solver() {
      if (h) rocblas_destroy_handle(h);
    }
  } solver;
  DMRG_REQUIRE(rocblas_create_handle(&solver.h) == rocblas_status_success, kErrHip,
               "davidson: rocblas_create_handle failed");
  DMRG_REQUIRE(rocblas_set_stream(solver.h, s) == rocblas_status_success, kErrHip,
               "davidson: rocblas_set_stream failed");
  DevBuf eigA((size_t)kmax * kmax * sizeof(double)), eigD(kmax * sizeof(double)),
      eigRes(sizeof(double)), eigInfo(2 * sizeof(rocblas_int));
  std::vector<double> colmaj((size_t)kmax * kmax);
  auto subspace_eigh = [&](int k, const std::vector<double>& Gk, std::vector<double>& ev_,
                           std::vector<double>& Y_) {
    DMRG_HIP(hipMemcpyAsync(eigA.p, Gk.data(), (size_t)k * k * sizeof(double), hipMemcpyHostToDevice, s));
    // cyclic Jacobi (one small-matrix kernel); tolerance: machine precision
    DMRG_REQUIRE(rocsolver_dsyevj(solver.h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper,
                                  k, eigA.as<double>(), k, 0.0, eigRes.as<double>(), 100,
                                  eigInfo.as<rocblas_int>() + 1, eigD.as<double>(),
                                  eigInfo.as<rocblas_int>()) == rocblas_status_success,
                 kErrHip, "davidson: rocsolver_dsyevj failed");
    ev_.resize(k);
    rocblas_int info = 0;
    DMRG_HIP(hipMemcpyAsync(ev_.data(), eigD.p, (size_t)k * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipMemcpyAsync(colmaj.data(), eigA.p, (size_t)k * k * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipMemcpyAsync(&info, eigInfo.p, sizeof(info), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    DMRG_REQUIRE(info == 0, kErrHip, "davidson: subspace eigensolver did not converge");
    Y_.resize((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Y_[(size_t)i * k + j] = colmaj[(size_t)j * k + i];
  };
  DevBuf tmpV, tmpW;
  std::vector<double> ev, Y;
  auto dot = [&](const double* a, const double* b) {
    launch_multidot(h, a, 0, 1, b, n, s);
    double x;
    DMRG_HIP(hipMemcpyAsync(&x, h, sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    return x;
  };
  auto sigma = [&](const double* x, double* y, int prec) {
    const double t0 = now_ms();
    run_sigma(plan, x, y, prec, s);
    DMRG_HIP(hipStreamSynchronize(s));
    res.sigma_ms += now_ms() - t0;
    res.n_sigma[prec]++;
  };
  // column j of G against all previous basis vectors: G[i][j] = V_i . W_j
  auto fill_col = [&](int k) {
    launch_multidot(h, V, n, k + 1, W + (int64_t)k * n, n, s);
    DMRG_HIP(hipMemcpyAsync(hh.data(), h, (k + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    for (int i = 0; i <= k; ++i) G[(size_t)i * kmax + k] = G[(size_t)k * kmax + i] = hh[i];
  };
  // start: V0 = psi / |psi|
  const double nrm = std::sqrt(dot(psi, psi));
  DMRG_REQUIRE(nrm > 0 && std::isfinite(nrm), kErrInvalidArg, "davidson: psi has zero or non-finite norm");
  DMRG_HIP(hipMemcpyAsync(V, psi, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_scale(V, 1.0 / nrm, n, s);
  int stage = 0;
  const bool verbose = std::getenv("DMRG_VERBOSE") != nullptr;  // one progress line per iteration
  const int nst = std::max(1, o.n_ladder);
  auto prec_of = [&](int st) { return o.n_ladder > 0 ? o.ladder[st] : 0; };
  // Residual refinement after a reduced-precision stage (Jacobi-Davidson
  // with inexact inner solves): the FP64 stage keeps its Davidson subspace,
  // FP64 sigma products and Rayleigh-Ritz, but each correction vector t
  // solves the correction equation
  //   (1 - u u^T)(H - theta)(1 - u u^T) t = -r,  t orthogonal to u,
  // for the Ritz pair (theta, u) and FP64 residual r, by conjugate gradients
  // on the reduced-precision sigma with the diagonal preconditioner
  // (diag(H_eff) - theta, projected), to a relative residual of kRefineEta
  // (looser when |r| is within a few times tol).
  // The reduced-precision error limits how much each correction gains, not
  // the attainable residual, which the FP64 products set.
  DevBuf cgb;
  auto inner_cg = [&](double* x, int lp, double theta_, int& iters_) {
    if (!cgb.p) cgb.alloc((size_t)4 * n * sizeof(double));
    double* rs = cgb.as<double>();  // residual of the correction equation
    double* z = rs + n;             // preconditioned residual
    double* p = z + n;              // search direction
    double* q = p + n;              // projected (H - theta) p
    auto project = [&](double* v) { launch_axpy(v, -dot(u, v), u, n, s); };
    const bool below_ = theta_ < dmin;
    auto precond = [&]() {  // z = P (diag - theta)^-1 rs, or P rs
      if (o.precondition > 0 && below_) {
        launch_precondition(z, rs, d, theta_, n, s);
        launch_scale(z, -1.0, n, s);
      } else {
        DMRG_HIP(hipMemcpyAsync(z, rs, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      }
      project(z);
    };
    DMRG_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
    DMRG_HIP(hipMemcpyAsync(rs, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_scale(rs, -1.0, n, s);
    project(rs);
    precond();
    DMRG_HIP(hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double rz = dot(rs, z);
    const double r0 = std::sqrt(std::max(0.0, dot(rs, rs)));
    // near the target a looser solve suffices: the correction needs to cut
    // the residual only to a fraction of tol
    const double eta = std::max(kRefineEta, std::min(0.5, 0.3 * o.tol / std::max(r0, 1e-300)));
    for (int it = 0; it < kRefineInner && iters_ < o.max_iter; ++it) {
      ++iters_;
      sigma(p, q, lp);
      launch_axpy(q, -theta_, p, n, s);
      project(q);
      const double pq = dot(p, q);
      if (!(pq > 0) || !(rz > 0)) break;  // the projected operator is not positive here
      const double alpha = rz / pq;
      launch_axpy(x, alpha, p, n, s);
      launch_axpy(rs, -alpha, q, n, s);
      const double rsn = std::sqrt(std::max(0.0, dot(rs, rs)));
      if (verbose)
        fprintf(stderr, "[dmrg] refinement inner %d (precision %d): relative residual %.3e\n", it, lp,
                rsn / r0);
      if (rsn < eta * r0) break;
      precond();
      const double rz1 = dot(rs, z);
      launch_scale(p, rz1 / rz, n, s);
      launch_axpy(p, 1.0, z, n, s);
      rz = rz1;
    }
  };
  int refine_lp = -1;  // reduced precision of the inner solves, once refining
  sigma(V, W, prec_of(stage));
  int k = 1;
  fill_col(0);
  double theta = G[0], rnorm = 1e300;
  std::vector<double> hist;
  int iters = 0;
  bool converged = false;
  while (true) {
    std::vector<double> Gk((size_t)k * k);
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) Gk[(size_t)i * k + j] = G[(size_t)i * kmax + j];
    subspace_eigh(k, Gk, ev, Y);
    int imin = (int)(std::min_element(ev.begin(), ev.end()) - ev.begin());
    theta = ev[imin];
    std::vector<double> y(k);
    for (int i = 0; i < k; ++i) y[i] = Y[(size_t)i * k + imin];
    DMRG_HIP(hipMemcpyAsync(cc, y.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
    launch_lincomb(u, V, n, k, cc, n, 0.0, s);
    launch_lincomb(w, W, n, k, cc, n, 0.0, s);
    DMRG_HIP(hipMemcpyAsync(r, w, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_axpy(r, -theta, u, n, s);
    rnorm = std::sqrt(std::max(0.0, dot(r, r)));
    if (verbose)
      fprintf(stderr, "[dmrg] davidson iteration %d stage %d (precision %d): theta %.12f residual %.3e\n",
              iters, stage, prec_of(stage), theta, rnorm);
    hist.push_back(rnorm);
    res.residual_history.push_back(rnorm);
    res.stage_history.push_back(stage);
    const bool last = stage == nst - 1;
    const double thr = last ? o.tol : o.ladder_tol[stage];
    // A reduced-precision stage ends at its threshold, near the residual
    // floor its sigma error sets (kFloorFactor times the relative sigma
    // error times |theta|: an inexact sigma cannot give a smaller residual),
    // or when the residual has not dropped by 10% in kStallWindow iterations.
    // A short stall window ends stages early on the plateaus of slow
    // convergence (measured at CAS(54,36): with a 3-iteration window the FP64
    // stage did 224 of 236 iterations; floor factors 10, 3 and 1.5 gave
    // 178, 169 and 173 s to solution against 236 s for FP64 alone).
    bool stalled = false;
    if (!last) {
      const double floor_abs = kFloorFactor * sigma_rel_error(prec_of(stage)) * std::fabs(theta);
      stalled = rnorm < floor_abs;
      if (hist.size() > (size_t)kStallWindow)
        stalled = stalled || rnorm > 0.9 * hist[hist.size() - 1 - kStallWindow];
    }
    if (rnorm < thr || stalled) {
      if (last) { converged = rnorm < o.tol; break; }
      // next ladder stage: restart from the Ritz vector with a fresh sigma
      ++stage;
      hist.clear();
      if (o.refine && stage == nst - 1 && prec_of(stage - 1) != 0) refine_lp = prec_of(stage - 1);
      const double un = std::sqrt(dot(u, u));
      DMRG_HIP(hipMemcpyAsync(V, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_scale(V, 1.0 / un, n, s);
      sigma(V, W, prec_of(stage));
      k = 1;
      fill_col(0);
      continue;
    }
    if (iters >= o.max_iter) break;
    ++iters;
    // correction t = r / (theta - diag), orthogonalised twice against V.
    // (theta - diag)^-1 is a useful preconditioner only once theta is below
    // the whole diagonal: while theta lies inside its range some
    // denominators pass through zero and the correction is dominated by
    // the few components where diag ~ theta, so those steps take t = r.
    const bool below = theta < dmin;
    double tn0 = 0;
    if (refine_lp >= 0) {
      inner_cg(t, refine_lp, theta, iters);
      tn0 = std::sqrt(std::max(0.0, dot(t, t)));
    }
    if (refine_lp >= 0 && tn0 > 0) {
      // correction from the inner solve
    } else if (o.precondition == 2 && below) {
      // Olsen: t = M^-1 (r - eps u), eps = u.M^-1 r / u.M^-1 u, M = theta - diag;
      // removes the component of M^-1 r along the Ritz vector that makes the
      // plain correction degenerate when diag(H_eff) is a good approximation
      launch_precondition(t, r, d, theta, n, s);
      launch_precondition(aux, u, d, theta, n, s);
      const double num = dot(u, t), den = dot(u, aux);
      if (std::abs(den) > 1e-300) launch_axpy(t, -num / den, aux, n, s);
    } else if (o.precondition == 1 && below) {
      launch_precondition(t, r, d, theta, n, s);
    } else {
      DMRG_HIP(hipMemcpyAsync(t, r, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    for (int pass = 0; pass < 2; ++pass) {
      launch_multidot(h, V, n, k, t, n, s);
      DMRG_HIP(hipMemcpyAsync(hh.data(), h, k * sizeof(double), hipMemcpyDeviceToHost, s));
      DMRG_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < k; ++i) hh[i] = -hh[i];
      DMRG_HIP(hipMemcpyAsync(cc, hh.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
      launch_lincomb(t, V, n, k, cc, n, 1.0, s);
    }
    double tn = std::sqrt(dot(t, t));
    if (k == kmax || !(tn > 1e-14)) {
      // thick restart: keep the m lowest Ritz vectors (V Y_m, W Y_m)
      const int m = std::min(k, std::max(1, std::min(o.restart, kmax - 1)));
      std::vector<int> order(k);
      for (int i = 0; i < k; ++i) order[i] = i;
      std::sort(order.begin(), order.end(), [&](int a, int b) { return ev[a] < ev[b]; });
      if (tmpV.bytes < (size_t)m * n * sizeof(double)) {
        tmpV.alloc((size_t)m * n * sizeof(double));
        tmpW.alloc((size_t)m * n * sizeof(double));
      }
      for (int j = 0; j < m; ++j) {
        std::vector<double> yj(k);
        for (int i = 0; i < k; ++i) yj[i] = Y[(size_t)i * k + order[j]];
        DMRG_HIP(hipMemcpyAsync(cc, yj.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        launch_lincomb(tmpV.as<double>() + (int64_t)j * n, V, n, k, cc, n, 0.0, s);
        launch_lincomb(tmpW.as<double>() + (int64_t)j * n, W, n, k, cc, n, 0.0, s);
        DMRG_HIP(hipStreamSynchronize(s));
      }
      DMRG_HIP(hipMemcpyAsync(V, tmpV.p, (size_t)m * n * sizeof(double), hipMemcpyDeviceToDevice, s));
      DMRG_HIP(hipMemcpyAsync(W, tmpW.p, (size_t)m * n * sizeof(double), hipMemcpyDeviceToDevice, s));
      k = m;
      for (int j = 0; j < m; ++j) fill_col(j);
      // re-orthogonalise t against the restarted basis
      for (int pass = 0; pass < 2; ++pass) {
        launch_multidot(h, V, n, k, t, n, s);
        DMRG_HIP(hipMemcpyAsync(hh.data(), h, k * sizeof(double), hipMemcpyDeviceToHost, s));
        DMRG_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < k; ++i) hh[i] = -hh[i];
        DMRG_HIP(hipMemcpyAsync(cc, hh.data(), k * sizeof(double), hipMemcpyHostToDevice, s));
        launch_lincomb(t, V, n, k, cc, n, 1.0, s);
      }
      tn = std::sqrt(dot(t, t));
      if (!(tn > 1e-14)) continue;
    }
    DMRG_HIP(hipMemcpyAsync(V + (int64_t)k * n, t, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_scale(V + (int64_t)k * n, 1.0 / tn, n, s);
    sigma(V + (int64_t)k * n, W + (int64_t)k * n, prec_of(stage));
    fill_col(k);
    ++k;
  }
  // final FP64 Rayleigh quotient of the normalised Ritz vector
  const double un = std::sqrt(dot(u, u));
  launch_scale(u, 1.0 / un, n, s);
  sigma(u, w, 0);
  res.energy = dot(u, w);
  DMRG_HIP(hipMemcpyAsync(r, w, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  launch_axpy(r, -res.energy, u, n, s);
  res.residual = std::sqrt(std::max(0.0, dot(r, r)));
  DMRG_HIP(hipMemcpyAsync(psi, u, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  DMRG_HIP(hipStreamSynchronize(s));
  res.iterations = iters;
  res.converged = converged || res.residual < o.tol;
  res.time_ms = now_ms() - t_start;
  return res.converged ? kOk : kWarnNotConverged;
}

}  // namespace dmrg
