// C ABI of the library (see include/dmrg.h).  Arguments are validated on the
// host before any device work; exceptions never cross the ABI.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>

#include "../../include/dmrg.h"
#include "backward.h"
#include "davidson.h"
#include "engine.h"
#include "su2.h"
#include "su2_product.h"
#include "noalloc.h"
#include "truncate.h"

using namespace dmrg;

struct dmrg_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool have_problem = false, have_mps = false;
  Problem P;
  Mps m;
  int window = -1;
  std::map<int, std::unique_ptr<Env>> left, right;  // by bond
  std::unique_ptr<SigmaPlan> plan;
  DevBuf desc;
  int64_t ws_budget = (int64_t)1 << 30;  // doubles of sigma intermediates (8 GiB)
  bool use_graphs = false;               // sigma replayed from HIP graphs
  DevBuf next_psi;                       // guess for the window left by dmrg_truncate
  int64_t next_size = -1;
  std::map<dmrg_su2_plan, std::unique_ptr<Su2Plan>> su2_plans;  // live spin-adapted plans
};

// A plan handle is an identity token; the context owns the plan it names.
struct dmrg_su2_plan_s {};

// Blocks kept while growing along the chain (for sweeps); larger ones are
// rebuilt on demand.
static const size_t kCacheBytes = (size_t)1 << 30;

static thread_local std::string g_err;

// DMRG_VERBOSE=1 prints one line per renormalisation step to stderr.
static bool verbose() {
  static int v = -1;
  if (v < 0) v = std::getenv("DMRG_VERBOSE") ? std::atoi(std::getenv("DMRG_VERBOSE")) : 0;
  return v > 0;
}
static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static dmrg_status fail(dmrg_ctx c, int code, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return code;
}

template <class F>
static dmrg_status guarded(dmrg_ctx c, F&& f) {
  try {
    if (c) DMRG_HIP(hipSetDevice(c->device));
    return f();
  } catch (const Error& e) {
    return fail(c, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(c, kErrOom, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, kErrState, e.what());
  }
}

extern "C" {

dmrg_status dmrg_create(dmrg_ctx* out, int32_t device, void* stream) {
  if (!out) return fail(nullptr, kErrInvalidArg, "out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
    return fail(nullptr, kErrNoDevice, "no HIP device");
  if (device < 0 || device >= n) return fail(nullptr, kErrNoDevice, "device index out of range");
  auto c = new (std::nothrow) dmrg_ctx_s;
  if (!c) return fail(nullptr, kErrOom, "host allocation failed");
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  // device address of the no-allocation scratch, looked up with the device current
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return fail(nullptr, kErrHip, "hipSetDevice failed");
  }
  try {
    noalloc_scratch_init(device);
  } catch (const Error& e) {
    delete c;
    return fail(nullptr, e.code, e.what());
  }
  if (const char* b = std::getenv("DMRG_WS_BUDGET_MB")) c->ws_budget = std::atoll(b) * (1 << 17);
  *out = c;
  return kOk;
}

dmrg_status dmrg_destroy(dmrg_ctx c) {
  if (!c) return kOk;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& kv : c->su2_plans) delete kv.first;
  delete c;
  return kOk;
}

const char* dmrg_last_error(dmrg_ctx c) { return c ? c->err.c_str() : g_err.c_str(); }

// Host-side checks of the active space and the integrals: ranges, parity,
// and the symmetries the operator algebra relies on (h symmetric, (pq|rs)
// with the 8-fold permutational symmetry of real orbitals), each to
// 1e-10 of the largest entry.
static void validate_problem(const dmrg_problem* p) {
  DMRG_REQUIRE(p, kErrInvalidArg, "problem is NULL");
  DMRG_REQUIRE(p->h && p->eri, kErrInvalidArg, "problem: h and eri must be non-NULL");
  const int K = p->n_orb, N = p->n_elec, t = p->two_sz;
  DMRG_REQUIRE(K >= 2 && K <= 127, kErrInvalidArg, "problem: need 2 <= n_orb <= 127");
  DMRG_REQUIRE(N >= 0 && N <= 2 * K, kErrInvalidArg, "problem: need 0 <= n_elec <= 2*n_orb");
  DMRG_REQUIRE(((N - t) % 2) == 0, kErrInvalidArg, "problem: n_elec and two_sz must have equal parity");
  DMRG_REQUIRE(std::abs(t) <= std::min(N, 2 * K - N), kErrInvalidArg, "problem: |two_sz| too large");
  DMRG_REQUIRE(std::isfinite(p->e_core), kErrInvalidArg, "problem: e_core is not finite");
  const size_t K2 = (size_t)K * K;
  double hmax = 0, gmax = 0;
  for (size_t a = 0; a < K2; ++a) {
    DMRG_REQUIRE(std::isfinite(p->h[a]), kErrInvalidArg, "problem: h has a non-finite entry");
    hmax = std::max(hmax, std::fabs(p->h[a]));
  }
  for (size_t a = 0; a < K2 * K2; ++a) {
    DMRG_REQUIRE(std::isfinite(p->eri[a]), kErrInvalidArg, "problem: eri has a non-finite entry");
    gmax = std::max(gmax, std::fabs(p->eri[a]));
  }
  const double th = 1e-10 * std::max(1.0, hmax), tg = 1e-10 * std::max(1.0, gmax);
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < a; ++b)
      DMRG_REQUIRE(std::fabs(p->h[(size_t)a * K + b] - p->h[(size_t)b * K + a]) <= th, kErrInvalidArg,
                   "problem: h is not symmetric");
  auto g = [&](int a, int b, int c, int d) { return p->eri[(((size_t)a * K + b) * K + c) * K + d]; };
  for (int a = 0; a < K; ++a)
    for (int b = 0; b < K; ++b)
      for (int c = 0; c < K; ++c)
        for (int d = 0; d < K; ++d) {
          const double x = g(a, b, c, d);
          DMRG_REQUIRE(std::fabs(x - g(b, a, c, d)) <= tg && std::fabs(x - g(a, b, d, c)) <= tg &&
                           std::fabs(x - g(c, d, a, b)) <= tg,
                       kErrInvalidArg, "problem: eri lacks the 8-fold symmetry (pq|rs) = (qp|rs) = (pq|sr) = (rs|pq)");
        }
}

static void load_problem(dmrg_ctx c, const dmrg_problem* p) {
  validate_problem(p);
  const int K = p->n_orb;
  c->P.K = K;
  c->P.N = p->n_elec;
  c->P.tsz = p->two_sz;
  c->P.e_core = p->e_core;
  c->P.h.assign(p->h, p->h + (size_t)K * K);
  c->P.eri.assign(p->eri, p->eri + (size_t)K * K * K * K);
  c->have_problem = true;
}

// Host-side checks of the MPS layout against the active space (K sites,
// sorted unique sectors, boundary bonds (0,0) and (N, 2Sz), positive
// dimensions, a tensor for every site outside the window); returns the bonds
// and, per site outside the window, the number of doubles of its tensor.
static Mps parse_mps(int K, int N, int tsz, const dmrg_mps* q, std::vector<int64_t>& site_size) {
  DMRG_REQUIRE(q, kErrInvalidArg, "mps is NULL");
  DMRG_REQUIRE(q->n_sites == K, kErrShape, "mps: n_sites differs from n_orb");
  DMRG_REQUIRE(q->bond_offsets && q->sector_n && q->sector_2sz && q->sector_dim && q->site_data,
               kErrInvalidArg, "mps: NULL array");
  DMRG_REQUIRE(q->window >= 0 && q->window <= K - 2, kErrInvalidArg, "mps: window out of range");
  Mps m;
  m.K = K;
  m.N = N;
  m.tsz = tsz;
  m.bonds.resize(K + 1);
  DMRG_REQUIRE(q->bond_offsets[0] == 0, kErrShape, "mps: bond_offsets[0] must be 0");
  for (int b = 0; b <= K; ++b) {
    const int s0 = q->bond_offsets[b], s1 = q->bond_offsets[b + 1];
    DMRG_REQUIRE(s0 >= 0 && s1 >= s0, kErrShape, "mps: bond offsets must be non-decreasing");
    DMRG_REQUIRE(s1 > s0, kErrShape, "mps: every bond needs at least one sector");
    Bond& B = m.bonds[b];
    for (int s = s0; s < s1; ++s) {
      QN x{q->sector_n[s], q->sector_2sz[s]};
      DMRG_REQUIRE(q->sector_dim[s] > 0, kErrShape, "mps: sector dims must be positive");
      DMRG_REQUIRE(B.q.empty() || B.q.back() < x, kErrShape, "mps: sectors must be sorted and unique");
      B.q.push_back(x);
      B.d.push_back(q->sector_dim[s]);
    }
    B.finish();
  }
  DMRG_REQUIRE(m.bonds[0].size() == 1 && m.bonds[0].q[0] == (QN{0, 0}) && m.bonds[0].d[0] == 1,
               kErrShape, "mps: bond 0 must be (0,0) of dim 1");
  DMRG_REQUIRE(m.bonds[K].size() == 1 && m.bonds[K].q[0] == (QN{N, tsz}) && m.bonds[K].d[0] == 1,
               kErrShape, "mps: bond K must be (N, 2Sz) of dim 1");
  site_size.assign(K, 0);
  for (int b = 0; b < K; ++b) {
    if (b == q->window || b == q->window + 1) continue;
    DMRG_REQUIRE(q->site_data[b], kErrInvalidArg, "mps: site tensor pointer is NULL");
    const Bond &L = m.bonds[b], &R = m.bonds[b + 1];
    int64_t off = 0;
    for (size_t l = 0; l < L.size(); ++l)
      for (int n = 0; n < 4; ++n) {
        const int r = R.find(L.q[l] + kSiteQN[n]);
        if (r >= 0) off += (int64_t)L.d[l] * R.d[r];
      }
    DMRG_REQUIRE(off > 0, kErrShape, "mps: a site tensor outside the window has no allowed block");
    site_size[b] = off;
  }
  return m;
}

static void load_mps(dmrg_ctx c, const dmrg_mps* q) {
  DMRG_REQUIRE(c->have_problem, kErrState, "mps: load a problem first");
  std::vector<int64_t> sz;
  Mps m = parse_mps(c->P.K, c->P.N, c->P.tsz, q, sz);
  m.site.resize(m.K);
  for (int b = 0; b < m.K; ++b) {
    if (b == q->window || b == q->window + 1) continue;
    const Bond &L = m.bonds[b], &R = m.bonds[b + 1];
    SiteTensor& st = m.site[b];
    st.off.assign(4 * L.size(), -1);
    int64_t off = 0;
    for (size_t l = 0; l < L.size(); ++l)
      for (int n = 0; n < 4; ++n) {
        int r = R.find(L.q[l] + kSiteQN[n]);
        if (r < 0) continue;
        st.off[4 * l + n] = off;
        off += (int64_t)L.d[l] * R.d[r];
      }
    st.data.alloc((size_t)std::max<int64_t>(off, 1) * sizeof(double));
    DMRG_HIP(hipMemcpy(st.data.p, q->site_data[b], off * sizeof(double), hipMemcpyHostToDevice));
  }
  c->m = std::move(m);
  c->window = q->window;
  c->have_mps = true;
  c->left.clear();
  c->right.clear();
  c->plan.reset();
}

dmrg_status dmrg_build_ops(dmrg_ctx c, const dmrg_problem* problem, const dmrg_mps* mps,
                           int32_t site, int32_t direction, uint32_t precision_mask) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    if (problem) {
      load_problem(c, problem);
      c->have_mps = false;
      c->left.clear();
      c->right.clear();
      c->plan.reset();
    }
    DMRG_REQUIRE(c->have_problem, kErrState, "build_ops: no problem loaded");
    DMRG_REQUIRE(mps || c->have_mps, kErrState, "build_ops: no MPS loaded");
    const int K = c->P.K;
    DMRG_REQUIRE(site >= 0 && site <= K - 2, kErrInvalidArg, "build_ops: site out of range");
    DMRG_REQUIRE(direction >= -1 && direction <= 1, kErrInvalidArg, "build_ops: direction must be -1, 0 or +1");
    DMRG_REQUIRE((precision_mask & ~7u) == 0, kErrInvalidArg, "build_ops: unknown precision bits");
    if (mps) {
      DMRG_REQUIRE(mps->window == site, kErrInvalidArg, "build_ops: mps.window must equal site");
      load_mps(c, mps);
    }
    DMRG_REQUIRE(c->window == site, kErrState, "build_ops: the loaded MPS has a different window");
    hipStream_t s = c->stream;
    // left block at bond `site`
    // (older blocks are released as soon as the next one exists)
    c->plan.reset();
    if (!c->left.count(site)) {
      int b = site;
      while (b > 0 && !c->left.count(b)) --b;
      std::unique_ptr<Env> cur = c->left.count(b) ? std::move(c->left[b]) : left_start(c->m, s);
      c->left.erase(b);
      for (; b < site; ++b) {
        const double t0 = now_s();
        auto nxt = grow_left(c->P, c->m, *cur, c->desc, s);
        if (cur->bytes() < kCacheBytes) c->left[b] = std::move(cur);
        cur = std::move(nxt);
        if (verbose())
          fprintf(stderr, "[dmrg] left block -> bond %d: %.2f s, %.2f GB\n", b + 1, now_s() - t0,
                  cur->bytes() / 1e9), fflush(stderr);
      }
      c->left[site] = std::move(cur);
    }
    if (!c->right.count(site + 2)) {
      int b = site + 2;
      while (b < K && !c->right.count(b)) ++b;
      std::unique_ptr<Env> cur = c->right.count(b) ? std::move(c->right[b]) : right_start(c->m, s);
      c->right.erase(b);
      for (; b > site + 2; --b) {
        const double t0 = now_s();
        auto nxt = grow_right(c->P, c->m, *cur, c->desc, s);
        if (cur->bytes() < kCacheBytes) c->right[b] = std::move(cur);
        cur = std::move(nxt);
        if (verbose())
          fprintf(stderr, "[dmrg] right block -> bond %d: %.2f s, %.2f GB\n", b - 1, now_s() - t0,
                  cur->bytes() / 1e9), fflush(stderr);
      }
      c->right[site + 2] = std::move(cur);
    }
    // large blocks away from this window are not kept
    for (auto it = c->left.begin(); it != c->left.end();)
      it = (it->first != site && it->second->bytes() >= kCacheBytes) ? c->left.erase(it) : std::next(it);
    for (auto it = c->right.begin(); it != c->right.end();)
      it = (it->first != site + 2 && it->second->bytes() >= kCacheBytes) ? c->right.erase(it) : std::next(it);
    const double t0 = now_s();
    c->plan = plan_sigma(c->P, c->m, *c->left[site], *c->right[site + 2], c->ws_budget, s);
    c->plan->use_graphs = c->use_graphs;
    plan_fixed_workspace(*c->plan, noalloc_scratch(c->device), kNoAllocScratchDoubles);
    DMRG_HIP(hipStreamSynchronize(s));
    if (verbose())
      fprintf(stderr, "[dmrg] sigma plan: %.2f s, %zu pairs, %zu right ops, %.3e flops\n",
              now_s() - t0, c->plan->pairs.size(), c->plan->zops.size(), c->plan->flops),
          fflush(stderr);
    (void)precision_mask;
    return kOk;
  });
}

dmrg_status dmrg_psi_size(dmrg_ctx c, int64_t* n) {
  if (!c || !n) return fail(c, kErrInvalidArg, "NULL argument");
  if (!c->plan) return fail(c, kErrState, "psi_size: call dmrg_build_ops first");
  *n = c->plan->psi.size;
  return kOk;
}

dmrg_status dmrg_sigma(dmrg_ctx c, const double* psi, double* sigma, int32_t precision) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "sigma: call dmrg_build_ops first");
    DMRG_REQUIRE(psi && sigma, kErrInvalidArg, "sigma: NULL buffer");
    DMRG_REQUIRE(precision >= 0 && precision <= 3, kErrInvalidArg, "sigma: unknown precision");
    run_sigma(*c->plan, psi, sigma, precision, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_sigma_noalloc(dmrg_ctx c, const double* psi, double* sigma) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "sigma_noalloc: call dmrg_build_ops first");
    DMRG_REQUIRE(psi && sigma, kErrInvalidArg, "sigma_noalloc: NULL buffer");
    DMRG_REQUIRE(c->plan->fx_ready, kErrShape,
                 "sigma_noalloc: the window's stage-1 workspace (" +
                     std::to_string((c->plan->ws_doubles * 8) >> 20) +
                     " MiB per chunk) exceeds the fixed scratch (" +
                     std::to_string((kNoAllocScratchDoubles * 8) >> 20) +
                     " MiB); create the context with DMRG_WS_BUDGET_MB at most that size");
    run_sigma_fixed_workspace(*c->plan, psi, sigma, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_sigma_backward(dmrg_ctx c, const double* psi, const double* sigma_bar, double* dh,
                                double* deri, int32_t precision) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "sigma_backward: call dmrg_build_ops first");
    DMRG_REQUIRE(psi && dh && deri, kErrInvalidArg, "sigma_backward: NULL buffer");
    DMRG_REQUIRE(precision == DMRG_FP64 || precision == DMRG_BF16 || precision == DMRG_BF16X3,
                 kErrInvalidArg, "sigma_backward: unknown precision");
    const int K = c->P.K;
    const size_t n1 = (size_t)K * K, n2 = n1 * n1;
    std::vector<double> g(n1 + n2);
    const double t0 = now_s();
    BackwardStats st = sigma_backward(c->P, c->m, c->window, psi, sigma_bar ? sigma_bar : psi, g.data(),
                                      c->ws_budget, c->stream, precision);
    DMRG_HIP(hipMemcpyAsync(dh, g.data(), n1 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    DMRG_HIP(hipMemcpyAsync(deri, g.data() + n1, n2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    DMRG_HIP(hipStreamSynchronize(c->stream));
    if (verbose())
      fprintf(stderr, "[dmrg] backward window %d (precision %d): rebuild %.1f ms, window %.1f ms, chains %.1f ms, %lld groups (%.1f ms)\n",
              c->window, precision, st.ms_chain, st.ms_window, st.ms_adjoint, (long long)st.n_groups,
              1e3 * (now_s() - t0));
    return kOk;
  });
}

dmrg_status dmrg_orbital_gradient(dmrg_ctx c, const double* dh, const double* deri, double* fock,
                                  double* grad) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->have_problem, kErrState, "orbital_gradient: no integrals loaded");
    DMRG_REQUIRE(dh && deri && grad, kErrInvalidArg, "orbital_gradient: NULL buffer");
    orbital_gradient(c->P, dh, deri, fock, grad, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_davidson(dmrg_ctx c, double* psi, const dmrg_davidson_opts* opts,
                          double* energy_out, dmrg_davidson_stats* stats) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "davidson: call dmrg_build_ops first");
    DMRG_REQUIRE(psi && opts && energy_out, kErrInvalidArg, "davidson: NULL argument");
    DavidsonOpts o;
    o.max_iter = opts->max_iter;
    o.max_subspace = opts->max_subspace;
    o.tol = opts->tol;
    o.n_ladder = opts->n_ladder;
    o.precondition = opts->precondition;
    if (opts->restart > 0) o.restart = opts->restart;
    o.refine = opts->refine != 0;
    DMRG_REQUIRE(o.max_iter >= 0 && o.max_subspace >= 3 && o.max_subspace <= 64, kErrInvalidArg,
                 "davidson: need max_iter >= 0 and 3 <= max_subspace <= 64");
    DMRG_REQUIRE(o.tol > 0, kErrInvalidArg, "davidson: tol must be positive");
    DMRG_REQUIRE(o.n_ladder >= 1 && o.n_ladder <= 4, kErrInvalidArg, "davidson: 1 <= n_ladder <= 4");
    for (int k = 0; k < o.n_ladder; ++k) {
      DMRG_REQUIRE(opts->ladder[k] >= 0 && opts->ladder[k] <= 3, kErrInvalidArg, "davidson: bad ladder precision");
      o.ladder[k] = opts->ladder[k];
      o.ladder_tol[k] = opts->ladder_tol[k];
    }
    DMRG_REQUIRE(o.ladder[o.n_ladder - 1] == DMRG_FP64, kErrInvalidArg, "davidson: the last ladder stage must be DMRG_FP64");
    SigmaPlan& p = *c->plan;
    if (!p.diag_ready) {
      build_diagonal(p, c->m.bonds[c->window], c->m.bonds[c->window + 2], c->stream);
      p.diag_ready = true;
    }
    DavidsonResult r;
    const int st = davidson(p, psi, o, r, c->stream);
    *energy_out = r.energy + c->P.e_core;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->energy = r.energy + c->P.e_core;
      stats->residual = r.residual;
      stats->time_ms = r.time_ms;
      stats->sigma_ms = r.sigma_ms;
      stats->iterations = r.iterations;
      stats->converged = r.converged;
      for (int k = 0; k < 4; ++k) stats->n_sigma[k] = r.n_sigma[k];
      const int nh = (int)std::min<size_t>(256, r.residual_history.size());
      stats->n_history = nh;
      for (int k = 0; k < nh; ++k) {
        stats->residual_history[k] = r.residual_history[k];
        stats->stage_history[k] = r.stage_history[k];
      }
    }
    return st;
  });
}

dmrg_status dmrg_truncate(dmrg_ctx c, const double* psi, int32_t direction, int32_t max_d,
                          double cutoff, double* trunc_err, int32_t* kept) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan && c->have_mps, kErrState, "truncate: call dmrg_build_ops first");
    DMRG_REQUIRE(psi, kErrInvalidArg, "truncate: NULL psi");
    DMRG_REQUIRE(direction == 1 || direction == -1, kErrInvalidArg, "truncate: direction must be +1 or -1");
    DMRG_REQUIRE(max_d >= 1 && cutoff >= 0, kErrInvalidArg, "truncate: need max_bond_dim >= 1, cutoff >= 0");
    const int i = c->window, K = c->P.K;
    DMRG_REQUIRE(!(direction > 0 && i + 1 > K - 2) && !(direction < 0 && i == 0), kErrInvalidArg,
                 "truncate: the window cannot move further in this direction");
    c->plan.reset();
    TruncResult r = truncate_and_move(c->m, i, psi, direction, max_d, cutoff, c->next_psi, c->desc, c->stream);
    // blocks that contain a changed tensor
    if (direction > 0) {
      for (auto it = c->left.begin(); it != c->left.end();) it = it->first >= i + 1 ? c->left.erase(it) : std::next(it);
      for (auto it = c->right.begin(); it != c->right.end();) it = it->first <= i + 2 ? c->right.erase(it) : std::next(it);
    } else {
      for (auto it = c->right.begin(); it != c->right.end();) it = it->first <= i + 1 ? c->right.erase(it) : std::next(it);
      for (auto it = c->left.begin(); it != c->left.end();) it = it->first >= i ? c->left.erase(it) : std::next(it);
    }
    c->window = i + direction;
    c->next_size = r.next_size;
    if (trunc_err) *trunc_err = r.trunc_err;
    if (kept) *kept = r.kept;
    return kOk;
  });
}

dmrg_status dmrg_get_psi(dmrg_ctx c, double* out) {
  if (!c || !out) return fail(c, kErrInvalidArg, "NULL argument");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->next_size >= 0, kErrState, "get_psi: no guess (call dmrg_truncate first)");
    DMRG_REQUIRE(c->plan && c->plan->psi.size == c->next_size, kErrState,
                 "get_psi: call dmrg_build_ops for the new window first");
    DMRG_HIP(hipMemcpyAsync(out, c->next_psi.p, c->next_size * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return kOk;
  });
}

dmrg_status dmrg_debug_diag(dmrg_ctx c, double* out) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "debug_diag: call dmrg_build_ops first");
    DMRG_REQUIRE(out, kErrInvalidArg, "debug_diag: NULL buffer");
    SigmaPlan& p = *c->plan;
    if (!p.diag_ready) {
      build_diagonal(p, c->m.bonds[c->window], c->m.bonds[c->window + 2], c->stream);
      p.diag_ready = true;
    }
    DMRG_HIP(hipMemcpyAsync(out, p.diag.p, p.psi.size * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return kOk;
  });
}

dmrg_status dmrg_sigma_get_info(dmrg_ctx c, int32_t precision, dmrg_sigma_info* out) {
  if (!c || !out) return fail(c, kErrInvalidArg, "NULL argument");
  return guarded(c, [&]() -> dmrg_status {
  DMRG_REQUIRE(c->plan, kErrState, "sigma_get_info: call dmrg_build_ops first");
  DMRG_REQUIRE(precision >= 0 && precision <= 3, kErrInvalidArg, "sigma_get_info: unknown precision");
  std::memset(out, 0, sizeof(*out));
  const SigmaPlan& p = *c->plan;
  out->flops = p.flops;
  out->flops_stage1 = p.flops_stage1;
  out->flops_stage2 = p.flops_stage2;
  const int kap = precision == DMRG_OZAKI ? ozaki_kappa() : 0;
  out->hw_flops = precision == DMRG_BF16X3 ? 3 * p.flops
                  : precision == DMRG_OZAKI ? 0.5 * kap * (kap + 1) * p.flops
                                            : p.flops;
  out->n_pairs = (int64_t)p.pairs.size();
  out->n_right_ops = (int64_t)p.zops.size();
  for (auto& g : p.f64_s1) out->n_stage1_tiles += (int64_t)g.ntiles;
  for (auto& g : p.f64_s2) {
    out->n_stage2_tiles += (int64_t)g.ntiles;
    out->n_stage2_segments += (int64_t)g.nsegs;
  }
  out->workspace_bytes = p.ws_doubles * 8;
  auto code = [](const BfChoice& c) { return c.shape + 16 * c.order + 256 * c.sort_a; };
  out->bf_config_stage1 = code(p.bf_choice[0]);
  out->bf_config_stage2 = code(p.bf_choice[1]);
  out->tune_ms = p.tune_ms;
  out->flops_terms = p.flops_terms;
  out->flops_stage1_used = p.flops_s1_used;
  out->n_chunks = (int32_t)p.s1.size();
  for (auto& kv : c->left) out->operator_bytes += (int64_t)kv.second->bytes();
  for (auto& kv : c->right) out->operator_bytes += (int64_t)kv.second->bytes();
  if (p.psums) out->operator_bytes += (int64_t)p.psums->bytes();
  return kOk;
  });
}

dmrg_status dmrg_sigma_graphs(dmrg_ctx c, int32_t enable) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(enable == 0 || enable == 1, kErrInvalidArg, "sigma_graphs: enable must be 0 or 1");
    c->use_graphs = enable == 1;
    if (c->plan) {
      DMRG_HIP(hipStreamSynchronize(c->stream));
      c->plan->use_graphs = c->use_graphs;
    }
    return kOk;
  });
}

dmrg_status dmrg_sigma_timing(dmrg_ctx c, int32_t mode, dmrg_sigma_times* out) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "sigma_timing: call dmrg_build_ops first");
    DMRG_REQUIRE(mode >= -1 && mode <= 1, kErrInvalidArg, "sigma_timing: mode must be -1, 0 or 1");
    SigmaPlan& p = *c->plan;
    SigmaTiming& t = p.timing;
    t.collect(c->stream);
    if (mode == 1) t.reset();
    if (mode >= 0) t.on = mode == 1;
    if (out) {
      std::memset(out, 0, sizeof(*out));
      out->calls = t.calls;
      out->launches_stage1 = t.launches[1];
      out->launches_stage2 = t.launches[2];
      out->launches_pinned = t.launches[3];
      out->ms_stage1 = t.ms[1];
      out->ms_stage2 = t.ms[2];
      out->ms_pinned = t.ms[3];
      out->launches_convert = t.launches[0];
      out->ms_convert = t.ms[0];
      for (auto& a : p.s1) out->flops_stage1 += a.flops;
      for (auto& a : p.s2) out->flops_stage2 += a.flops;
      out->flops_pinned = p.p1.flops + p.p2.flops;
    }
    return kOk;
  });
}

dmrg_status dmrg_su2_psi_size(const dmrg_su2_window* window, int64_t* n) {
  return guarded(nullptr, [&]() -> dmrg_status {
    DMRG_REQUIRE(window && n, kErrInvalidArg, "su2_psi_size: NULL pointer");
    *n = su2_psi_size(*window);
    return kOk;
  });
}

dmrg_status dmrg_su2_sigma(dmrg_ctx c, const dmrg_su2_window* window, int32_t n_left_ops,
                           const dmrg_su2_operator* left_ops, int32_t n_right_ops,
                           const dmrg_su2_operator* right_ops, int32_t n_pairs, const dmrg_su2_pair* pairs,
                           const double* psi, double* sigma) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(window, kErrInvalidArg, "su2_sigma: NULL window");
    auto plan = su2_plan(*window, n_left_ops, left_ops, n_right_ops, right_ops, n_pairs, pairs, DMRG_FP64,
                         c->ws_budget, c->stream);
    su2_run(*plan, psi, sigma, c->stream);
    DMRG_HIP(hipStreamSynchronize(c->stream));  // the plan's buffers are released on return
    return kOk;
  });
}

dmrg_status dmrg_su2_plan_create(dmrg_ctx c, const dmrg_su2_window* window, int32_t n_left_ops,
                                 const dmrg_su2_operator* left_ops, int32_t n_right_ops,
                                 const dmrg_su2_operator* right_ops, int32_t n_pairs,
                                 const dmrg_su2_pair* pairs, int32_t precision, dmrg_su2_plan* out) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(window && out, kErrInvalidArg, "su2_plan_create: NULL pointer");
    *out = nullptr;
    auto plan = su2_plan(*window, n_left_ops, left_ops, n_right_ops, right_ops, n_pairs, pairs, precision,
                         c->ws_budget, c->stream);
    dmrg_su2_plan h = new dmrg_su2_plan_s;
    c->su2_plans[h] = std::move(plan);
    *out = h;
    return kOk;
  });
}

static Su2Plan& su2_of(dmrg_ctx c, dmrg_su2_plan h) {
  auto it = c->su2_plans.find(h);
  DMRG_REQUIRE(h && it != c->su2_plans.end(), kErrInvalidArg, "su2: not a plan of this context");
  return *it->second;
}

dmrg_status dmrg_su2_plan_sigma(dmrg_ctx c, dmrg_su2_plan h, const double* psi, double* sigma) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    su2_run(su2_of(c, h), psi, sigma, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_su2_plan_info(dmrg_ctx c, dmrg_su2_plan h, dmrg_su2_info* out) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(out, kErrInvalidArg, "su2_plan_info: NULL output");
    const Su2Plan& p = su2_of(c, h);
    *out = dmrg_su2_info{};
    out->psi_size = p.psi_size;
    const bool x3 = p.precision == DMRG_BF16X3;
    out->n_chunks = (int32_t)(x3 ? p.s1b.size() : p.s1.size());
    out->n_segments = p.n_segments;
    out->workspace_bytes = p.ws_doubles * (int64_t)(x3 ? 2 * sizeof(uint16_t) : sizeof(double));
    out->flops_stage1 = p.flops1;
    out->flops_stage2 = p.flops2;
    return kOk;
  });
}

dmrg_status dmrg_su2_plan_destroy(dmrg_ctx c, dmrg_su2_plan h) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  if (!h) return kOk;
  return guarded(c, [&]() -> dmrg_status {
    su2_of(c, h);
    DMRG_HIP(hipStreamSynchronize(c->stream));
    c->su2_plans.erase(h);
    delete h;
    return kOk;
  });
}

dmrg_status dmrg_su2_product_size(const dmrg_su2_window* sectors, const dmrg_su2_operator* a,
                                  const dmrg_su2_operator* b, int32_t two_k1, int32_t two_k2, int32_t two_k,
                                  int32_t* n_blocks, int64_t* n_elems) {
  return guarded(nullptr, [&]() -> dmrg_status {
    DMRG_REQUIRE(sectors && a && b && n_blocks && n_elems, kErrInvalidArg, "su2_product_size: NULL pointer");
    const Su2Product p = su2_product_plan(*sectors, *a, *b, two_k1, two_k2, two_k, 0);
    *n_blocks = (int32_t)p.blocks.size();
    *n_elems = p.size;
    return kOk;
  });
}

dmrg_status dmrg_su2_product(dmrg_ctx c, const dmrg_su2_window* sectors, const dmrg_su2_operator* a,
                             const dmrg_su2_operator* b, int32_t two_k1, int32_t two_k2, int32_t two_k,
                             int32_t parity_b, int32_t* out_sector, int32_t* in_sector, int64_t* offset,
                             double* data) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(sectors && a && b, kErrInvalidArg, "su2_product: NULL pointer");
    const Su2Product p = su2_product_plan(*sectors, *a, *b, two_k1, two_k2, two_k, parity_b);
    DMRG_REQUIRE(p.blocks.empty() || (out_sector && in_sector && offset), kErrInvalidArg,
                 "su2_product: NULL output array");
    for (size_t i = 0; i < p.blocks.size(); ++i) {
      out_sector[i] = p.blocks[i].out;
      in_sector[i] = p.blocks[i].in;
      offset[i] = p.blocks[i].offset;
    }
    su2_product_run(p, *a, *b, data, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_su2_rotate_size(const dmrg_su2_basis* basis, int32_t n_blocks, const int32_t* out_sector,
                                 const int32_t* in_sector, int32_t* n_out, int64_t* n_elems) {
  return guarded(nullptr, [&]() -> dmrg_status {
    DMRG_REQUIRE(basis && n_out && n_elems, kErrInvalidArg, "su2_rotate_size: NULL pointer");
    const Su2Rotation r = su2_rotation_plan(*basis, n_blocks, out_sector, in_sector);
    *n_out = (int32_t)r.outs.size();
    *n_elems = r.size;
    return kOk;
  });
}

dmrg_status dmrg_su2_rotate(dmrg_ctx c, const dmrg_su2_basis* basis, int32_t n_blocks, const int32_t* out_sector,
                            const int32_t* in_sector, const int64_t* offset, const double* data,
                            int32_t* out_group, int32_t* in_group, int64_t* out_offset, double* out_data) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(basis, kErrInvalidArg, "su2_rotate: NULL basis");
    const Su2Rotation r = su2_rotation_plan(*basis, n_blocks, out_sector, in_sector);
    DMRG_REQUIRE(r.outs.empty() || (out_group && in_group && out_offset), kErrInvalidArg,
                 "su2_rotate: NULL output array");
    for (size_t i = 0; i < r.outs.size(); ++i) {
      out_group[i] = r.outs[i].g2;
      in_group[i] = r.outs[i].g;
      out_offset[i] = r.outs[i].offset;
    }
    su2_rotation_run(r, *basis, out_sector, in_sector, offset, data, out_data, c->stream);
    return kOk;
  });
}

dmrg_status dmrg_debug_gemm(dmrg_ctx c, int32_t m, int32_t n, int32_t k, const double* a,
                            int32_t lda, int32_t trans_a, const double* b, int32_t ldb,
                            int32_t trans_b, double* cc, int32_t ldc, double alpha, int32_t beta,
                            int32_t precision) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(a && b && cc, kErrInvalidArg, "debug_gemm: NULL pointer");
    DMRG_REQUIRE(m > 0 && n > 0 && k > 0, kErrInvalidArg, "debug_gemm: sizes must be positive");
    DMRG_REQUIRE(beta == 0 || beta == 1, kErrInvalidArg, "debug_gemm: beta must be 0 or 1");
    DMRG_REQUIRE(lda >= (trans_a ? m : k) && ldb >= (trans_b ? k : n) && ldc >= n, kErrInvalidArg,
                 "debug_gemm: leading dimension too small");
    DMRG_REQUIRE(precision >= 0 && precision <= 3, kErrInvalidArg, "debug_gemm: unknown precision");
    const int flags = (trans_a ? kTransA : 0) | (trans_b ? kTransB : 0);
    if (precision == DMRG_FP64) {
      GemmBatch bt;
      bt.segs.push_back({a, b, lda, ldb, k, flags, alpha});
      bt.add_problem(cc, ldc, m, n, 0, 1, beta);
      launch_gemm_f64(bt, c->stream);
      return kOk;
    }
    if (precision == DMRG_OZAKI) {
      // digit planes of A (m rows) and of B's n x k storage (n rows)
      const int kappa = ozaki_kappa(), kp = oz_kp(k);
      const int64_t pa = (int64_t)m * kp, pb = (int64_t)n * kp;
      SliceOp ops[2] = {};
      ops[0] = {a, 0, pa, 0, 0, lda, m, k, kp, trans_a ? 1 : 0, 0};
      ops[1] = {b, kappa * pa, pb, m, m, ldb, n, k, kp, trans_b ? 0 : 1, 0};
      DevBuf arena((size_t)(kappa * (pa + pb))), exps((size_t)(m + n) * sizeof(int32_t)), dops(sizeof(ops));
      DMRG_HIP(hipMemcpyAsync(dops.p, ops, sizeof(ops), hipMemcpyHostToDevice, c->stream));
      launch_slice_oz(dops.as<SliceOp>(), 2, m + n, arena.as<int8_t>(), exps.as<int32_t>(), kappa, c->stream);
      GemmBatchO bt;
      GemmSegO g{};
      g.a = arena.as<int8_t>();
      g.b = arena.as<int8_t>() + kappa * pa;
      g.ea = exps.as<int32_t>();
      g.eb = exps.as<int32_t>() + m;
      g.a_plane = pa;
      g.b_plane = pb;
      g.lda = g.ldb = kp;
      g.k = k;
      g.alpha = alpha;
      bt.segs.push_back(g);
      bt.add_problem(cc, ldc, m, n, 0, 1, beta);
      DevGemmO d;
      upload_gemm_oz(bt, kappa, d);
      launch_gemm_oz(d, kappa, c->stream);
      DMRG_HIP(hipStreamSynchronize(c->stream));
      return kOk;
    }
    // padded NT copies: A as m x pad8(k) rows, B as n x pad8(k) rows, then BF16 hi/lo
    const int kp = (k + 7) & ~7;
    std::vector<double> ha((size_t)(trans_a ? k : m) * lda), hb((size_t)(trans_b ? n : k) * ldb);
    DMRG_HIP(hipStreamSynchronize(c->stream));
    DMRG_HIP(hipMemcpy(ha.data(), a, ha.size() * sizeof(double), hipMemcpyDeviceToHost));
    DMRG_HIP(hipMemcpy(hb.data(), b, hb.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> pa((size_t)m * kp, 0.0), pb((size_t)n * kp, 0.0);
    for (int i = 0; i < m; ++i)
      for (int q = 0; q < k; ++q)
        pa[(size_t)i * kp + q] = trans_a ? ha[(size_t)q * lda + i] : ha[(size_t)i * lda + q];
    for (int j = 0; j < n; ++j)
      for (int q = 0; q < k; ++q)
        pb[(size_t)j * kp + q] = trans_b ? hb[(size_t)j * ldb + q] : hb[(size_t)q * ldb + j];
    const int64_t na = (int64_t)pa.size(), nb = (int64_t)pb.size();
    DevBuf da(na * sizeof(double)), db(nb * sizeof(double));
    DMRG_HIP(hipMemcpy(da.p, pa.data(), na * sizeof(double), hipMemcpyHostToDevice));
    DMRG_HIP(hipMemcpy(db.p, pb.data(), nb * sizeof(double), hipMemcpyHostToDevice));
    DevBuf abf((size_t)2 * na * sizeof(uint16_t)), bbf((size_t)2 * nb * sizeof(uint16_t));
    launch_split_bf16(abf.as<uint16_t>(), da.as<double>(), na, c->stream);
    launch_split_bf16(bbf.as<uint16_t>(), db.as<double>(), nb, c->stream);
    GemmBatchB bt;
    if (const char* sh = std::getenv("DMRG_BF16_SHAPE")) bt.shape = std::max(0, std::min(kNumShapes - 1, std::atoi(sh)));
    bt.segs.push_back({abf.as<uint16_t>(), bbf.as<uint16_t>(), na, nb, kp, kp, k, kTransB, alpha});
    bt.add_problem(cc, 0, ldc, m, n, 0, 1, beta);
    DevGemmB d;
    upload_gemm_bf16(bt, d);
    launch_gemm_bf16(d, precision == DMRG_BF16X3, kOutF64, 0, c->stream);
    DMRG_HIP(hipStreamSynchronize(c->stream));
    return kOk;
  });
}

dmrg_status dmrg_validate(const dmrg_problem* problem, const dmrg_mps* mps) {
  return guarded(nullptr, [&]() -> dmrg_status {
    validate_problem(problem);
    if (mps) {
      std::vector<int64_t> sz;
      (void)parse_mps(problem->n_orb, problem->n_elec, problem->two_sz, mps, sz);
    }
    return kOk;
  });
}

dmrg_status dmrg_get_bond(dmrg_ctx c, int32_t bond, int32_t capacity, int32_t* n_sectors,
                          int32_t* sector_n, int32_t* sector_2sz, int32_t* sector_dim) {
  if (!c || !n_sectors) return fail(c, kErrInvalidArg, "NULL argument");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->have_mps, kErrState, "get_bond: no MPS loaded");
    DMRG_REQUIRE(bond >= 0 && bond <= c->P.K, kErrInvalidArg, "get_bond: bond out of range");
    const Bond& B = c->m.bonds[bond];
    const int n = (int)B.size();
    if (sector_n || sector_2sz || sector_dim) {
      DMRG_REQUIRE(sector_n && sector_2sz && sector_dim, kErrInvalidArg,
                   "get_bond: give all three sector arrays or none");
      DMRG_REQUIRE(capacity >= n, kErrShape, "get_bond: capacity below the number of sectors");
      for (int k = 0; k < n; ++k) {
        sector_n[k] = B.q[k].n;
        sector_2sz[k] = B.q[k].s;
        sector_dim[k] = B.d[k];
      }
    }
    *n_sectors = n;
    return kOk;
  });
}

dmrg_status dmrg_get_site(dmrg_ctx c, int32_t site, int64_t capacity, double* out, int64_t* size) {
  if (!c || !size) return fail(c, kErrInvalidArg, "NULL argument");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->have_mps, kErrState, "get_site: no MPS loaded");
    DMRG_REQUIRE(site >= 0 && site < c->P.K, kErrInvalidArg, "get_site: site out of range");
    DMRG_REQUIRE(site != c->window && site != c->window + 1, kErrState,
                 "get_site: the window's sites are held in psi, not as site tensors");
    const SiteTensor& st = c->m.site[site];
    DMRG_REQUIRE(!st.off.empty(), kErrState, "get_site: the site tensor is not held");
    const Bond &L = c->m.bonds[site], &R = c->m.bonds[site + 1];
    // packed size in the dmrg_mps layout (blocks (l, n) -> r, ascending l then n)
    int64_t n = 0;
    for (size_t l = 0; l < L.size(); ++l)
      for (int k = 0; k < 4; ++k) {
        const int r = R.find(L.q[l] + kSiteQN[k]);
        if (r >= 0) {
          DMRG_REQUIRE(st.off[4 * l + k] == n, kErrState, "get_site: internal layout differs from the packed layout");
          n += (int64_t)L.d[l] * R.d[r];
        }
      }
    if (out) {
      DMRG_REQUIRE(capacity >= n, kErrShape, "get_site: capacity below the tensor size");
      DMRG_HIP(hipStreamSynchronize(c->stream));
      DMRG_HIP(hipMemcpy(out, st.data.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
    }
    *size = n;
    return kOk;
  });
}

dmrg_status dmrg_energy(dmrg_ctx c, const double* h, const double* eri, const double* psi,
                        int32_t precision, double* sigma_out, double* grad_psi, double* energy_out,
                        double* norm2_out) {
  if (!c) return fail(c, kErrInvalidArg, "ctx is NULL");
  return guarded(c, [&]() -> dmrg_status {
    DMRG_REQUIRE(c->plan, kErrState, "energy: call dmrg_build_ops first");
    DMRG_REQUIRE(psi && energy_out, kErrInvalidArg, "energy: NULL psi or energy_out");
    DMRG_REQUIRE(precision >= 0 && precision <= 3, kErrInvalidArg, "energy: unknown precision");
    DMRG_REQUIRE((h == nullptr) == (eri == nullptr), kErrInvalidArg, "energy: give both h and eri or neither");
    if (h) {
      const int K = c->P.K;
      const size_t n1 = (size_t)K * K, n2 = n1 * n1;
      double dmax = 0, xmax = 0;
      for (size_t a = 0; a < n1; ++a) {
        dmax = std::max(dmax, std::fabs(h[a] - c->P.h[a]));
        xmax = std::max(xmax, std::fabs(c->P.h[a]));
      }
      for (size_t a = 0; a < n2; ++a) {
        dmax = std::max(dmax, std::fabs(eri[a] - c->P.eri[a]));
        xmax = std::max(xmax, std::fabs(c->P.eri[a]));
      }
      DMRG_REQUIRE(dmax <= 1e-13 * std::max(1.0, xmax), kErrInvalidArg,
                   "energy: h / eri differ from the integrals the operators were built from (max |diff| " +
                       std::to_string(dmax) + ")");
    }
    const int64_t n = c->plan->psi.size;
    hipStream_t s = c->stream;
    DevBuf own;
    double* sig = sigma_out;
    if (!sig) {
      own.alloc((size_t)std::max<int64_t>(1, n) * sizeof(double));
      sig = own.as<double>();
    }
    run_sigma(*c->plan, psi, sig, precision, s);
    DevBuf dots(2 * sizeof(double));
    launch_multidot(dots.as<double>(), sig, 0, 1, psi, n, s);
    launch_multidot(dots.as<double>() + 1, psi, 0, 1, psi, n, s);
    if (grad_psi) launch_axpby(grad_psi, 2.0, sig, 2.0 * c->P.e_core, psi, n, s);
    double hd[2];
    DMRG_HIP(hipMemcpyAsync(hd, dots.p, sizeof(hd), hipMemcpyDeviceToHost, s));
    DMRG_HIP(hipStreamSynchronize(s));
    *energy_out = hd[0] + c->P.e_core * hd[1];
    if (norm2_out) *norm2_out = hd[1];
    return kOk;
  });
}

}  // extern "C"
