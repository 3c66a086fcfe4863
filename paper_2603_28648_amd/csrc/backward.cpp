// Reverse mode of the two-site sigma with respect to the integrals.
//
// For fixed window vectors psi, lam and a fixed MPS, f = <lam, H_eff psi> is
// linear in (h, (pq|rs)); its gradient is the transition 1- and 2-RDM of the
// two full-space states the window vectors stand for (with lam = psi, the
// RDMs that orbital optimisation needs: dE/dh_pq = gamma_pq and
// dE/d(pq|rs) = Gamma_pqrs / 2).
//
// Every integral enters the sigma through exactly one component coefficient:
// of a block Hamiltonian, of a complementary operator, or of a window partial
// sum.  The operator such a coefficient multiplies is always an identity or a
// normal string, which does not depend on the integrals.  So, in reverse:
//   1. window: adjoints of the integral-dependent operators of the pairs,
//        L_bar[l',l] += y s * lam(l',n')[r'] . (Z psi^T)[r'](l,n)   (left)
//        U_bar = y s * L^T lam,  Z_bar[r',r] += a * U_bar^T psi(r)   (right)
//      and the partial sums' coefficient gradients <W_bar, x_L>;
//   2. along each chain, from the window outwards, the adjoint of
//      X -> Proj(X (x) y):
//        left  X_bar[l',l] += y s * A(l',n') N_bar[r',r] A(l,n)^T
//        right X_bar[r',r] += y s * B(l',n')^T N_bar[l',l] B(l,n)
//      carries the adjoints of block Hamiltonians and complementary
//      operators to the operators they were built from, and every
//      coefficient with integral dependence receives <N_bar_t, Proj(x (x) y)>.
// All contractions are grouped GEMMs of the forward's kernels: FP64, or the
// BF16 kernel (BF16 or split-BF16x3 products, FP32 accumulation flushed into
// FP64) for the mixed variant; the blocks are rebuilt in FP64 either way.
#include "backward.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <set>
#include <tuple>

namespace dmrg {
namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

using Kinds = std::vector<std::vector<uint8_t>>;
Kinds kinds_of(const Env& e) {
  Kinds k(e.classes.size());
  for (size_t c = 0; c < e.classes.size(); ++c) k[c].assign((size_t)e.classes[c]->nops, 255);
  for (auto& kv : e.ops) k[kv.second.cls][kv.second.idx] = kv.first.kind;
  return k;
}
// Operators whose entries depend on the integrals.
bool dependent(uint8_t kind) { return kind == kHam || kind == kComp || kind == kPsum; }

// Adjoints of the operators of one block: one zeroed array per class.
struct Adj {
  std::vector<DevBuf> cls;
  double* op(const Env& e, int c, int i) const {
    return cls[c].as<double>() + (int64_t)i * e.classes[c]->L.nnz;
  }
};
void alloc_adj(const Env& e, Adj& a, hipStream_t s) {
  a.cls.clear();
  a.cls.resize(e.classes.size());
  for (size_t c = 0; c < e.classes.size(); ++c) {
    const int64_t n = std::max<int64_t>(1, (int64_t)e.classes[c]->nops * e.classes[c]->L.nnz);
    a.cls[c].alloc((size_t)n * sizeof(double));
    launch_fill(a.cls[c].as<double>(), 0.0, n, s);
  }
}

void grow(DevBuf& b, size_t bytes, hipStream_t s) {
  if (b.bytes >= bytes) return;
  DMRG_HIP(hipStreamSynchronize(s));
  b.alloc(bytes);
}

// dst (old-bond operator, layout dl) += alpha * Proj^T(src, y), the adjoint
// of X -> Proj(X (x) y) applied to the new-bond operator src (layout sl).
// Same chunked two-stage scheme as the forward projections.
void run_adjoint_projections(int side, const Mps& m, int site, const std::vector<Projection>& projs,
                             DevBuf& desc, DevBuf& uws, int64_t budget, hipStream_t s) {
  const SiteTensor& st = m.site[site];
  const double* S = st.data.as<double>();
  const Bond& oldb = side > 0 ? m.bonds[site] : m.bonds[site + 1];
  const Bond& newb = side > 0 ? m.bonds[site + 1] : m.bonds[site];
  // visits every (dst block, n', n) term; f(tb, n', n, yv, idx...) with the
  // sector indices on both bonds
  struct Term {
    const Layout::Blk* tb;
    const Layout::Blk* xb;
    int n, np;
    double yv;
    int o0, o1;        // old-bond sectors (ket, bra)
    int w0, w1;        // new-bond sectors (ket, bra)
    int64_t s0, s1;    // site blocks (ket, bra)
  };
  auto visit = [&](const Projection& pr, auto&& f) {
    for (auto& tb : pr.dl->blk) {
      f.begin(tb);
      for (int n = 0; n < 4; ++n)
        for (int np = 0; np < 4; ++np) {
          const double yv = pr.y.m[np][n];
          if (yv == 0) continue;
          const int o0 = tb.c, o1 = tb.r;
          int w0, w1;
          if (side > 0) {
            w0 = newb.find(oldb.q[o0] + kSiteQN[n]);
            w1 = newb.find(oldb.q[o1] + kSiteQN[np]);
          } else {
            w0 = newb.find(oldb.q[o0] - kSiteQN[n]);
            w1 = newb.find(oldb.q[o1] - kSiteQN[np]);
          }
          if (w0 < 0 || w1 < 0) continue;
          const Layout::Blk* xb = pr.sl->col(w0);
          if (!xb || xb->r != w1) continue;
          const int64_t s0 = side > 0 ? st.off[4 * o0 + n] : st.off[4 * w0 + n];
          const int64_t s1 = side > 0 ? st.off[4 * o1 + np] : st.off[4 * w1 + np];
          if (s0 < 0 || s1 < 0) continue;
          f.term(Term{&tb, xb, n, np, yv, o0, o1, w0, w1, s0, s1});
        }
      f.end(tb);
    }
  };
  size_t p = 0;
  while (p < projs.size()) {
    int64_t need = 0;
    size_t q = p;
    for (; q < projs.size(); ++q) {
      struct {
        int64_t u = 0;
        const Bond *ob, *nb;
        void begin(const Layout::Blk&) {}
        void end(const Layout::Blk&) {}
        void term(const Term& t) {
          u += (int64_t)nb->d[t.w1] * ob->d[t.o0];
        }
      } sz;
      sz.ob = &oldb;
      sz.nb = &newb;
      visit(projs[q], sz);
      if (q > p && need + sz.u > budget) break;
      need += sz.u;
    }
    grow(uws, (size_t)std::max<int64_t>(need, 1) * sizeof(double), s);
    double* U = uws.as<double>();
    int64_t uoff = 0;
    GemmBatch b1, b2;
    for (size_t k = p; k < q; ++k) {
      const Projection& pr = projs[k];
      const int xpar = pr.dl->dq.n & 1;
      struct {
        GemmBatch *b1, *b2;
        const Projection* pr;
        const Bond *ob, *nb;
        const double* S;
        double* U;
        int64_t* uoff;
        int side, xpar;
        size_t s0 = 0;
        void begin(const Layout::Blk&) { s0 = b2->segs.size(); }
        void term(const Term& t) {
          double* u = U + *uoff;
          const size_t t0 = b1->segs.size();
          if (side > 0) {
            // old sectors l = o0, l' = o1; new sectors r = w0, r' = w1
            const int dl = ob->d[t.o0], dlp = ob->d[t.o1], dr = nb->d[t.w0], drp = nb->d[t.w1];
            *uoff += (int64_t)drp * dl;
            // u (r' x l) = N[r', r] A(l, n)^T
            b1->segs.push_back({pr->src + t.xb->off, S + t.s0, t.xb->ld, dr, dr, kTransB, 1.0});
            b1->add_problem(u, dl, drp, dl, t0, t0 + 1, 0);
            const double sg = ((pr->ypar & 1) && (ob->q[t.o0].n & 1)) ? -1.0 : 1.0;
            // X[l', l] += A(l', n') u
            b2->segs.push_back({S + t.s1, u, drp, dl, drp, 0, pr->alpha * t.yv * sg});
          } else {
            // old sectors r = o0, r' = o1; new sectors l = w0, l' = w1
            const int dr = ob->d[t.o0], drp = ob->d[t.o1], dl = nb->d[t.w0], dlp = nb->d[t.w1];
            *uoff += (int64_t)dlp * dr;
            // u (l' x r) = N[l', l] B(l, n)
            b1->segs.push_back({pr->src + t.xb->off, S + t.s0, t.xb->ld, dr, dl, 0, 1.0});
            b1->add_problem(u, dr, dlp, dr, t0, t0 + 1, 0);
            const double sg = (xpar && (kSiteN[t.n] & 1)) ? -1.0 : 1.0;
            // X[r', r] += B(l', n')^T u
            b2->segs.push_back({S + t.s1, u, drp, dr, dlp, kTransA, pr->alpha * t.yv * sg});
          }
        }
        void end(const Layout::Blk& tb) {
          b2->add_problem(pr->dst + tb.off, tb.ld, tb.dr, tb.dc, s0, b2->segs.size(), 1);
        }
      } em;
      em.b1 = &b1;
      em.b2 = &b2;
      em.pr = &pr;
      em.ob = &oldb;
      em.nb = &newb;
      em.S = S;
      em.U = U;
      em.uoff = &uoff;
      em.side = side;
      em.xpar = xpar;
      visit(pr, em);
    }
    launch_gemm(b1, desc, s);
    launch_gemm(b2, desc, s);
    p = q;
  }
}

const int64_t kProjBudget = (int64_t)1 << 27;  // doubles of projection intermediates per chunk


struct Work {
  DevBuf desc, uws, tmp, tmp2, coef, gout;
  std::vector<double> host;
};

// Downloads G (rows x cols) after the stream drains.
const std::vector<double>& fetch(Work& w, int64_t n, hipStream_t s) {
  w.host.resize((size_t)n);
  DMRG_HIP(hipStreamSynchronize(s));
  DMRG_HIP(hipMemcpy(w.host.data(), w.gout.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
  return w.host;
}

void upload(DevBuf& d, const std::vector<double>& h, hipStream_t s) {
  grow(d, std::max<size_t>(1, h.size()) * sizeof(double), s);
  DMRG_HIP(hipStreamSynchronize(s));
  DMRG_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
}

// C (m x n, ldc) = or += alpha * op(A) op(B) as one problem.  An empty
// contraction (k = 0, e.g. an operator class without blocks) still sets C = 0
// when beta = 0.
void gemm(void* c, int ldc, int m, int n, const void* a, int lda, const void* b, int ldb, int k,
          int flags, double alpha, int beta, DevBuf& desc, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  if (k <= 0) {
    if (!beta) {
      DMRG_REQUIRE(ldc == n, kErrState, "gemm: empty product into a strided output");
      launch_fill(static_cast<double*>(c), 0.0, (int64_t)m * n, s);
    }
    return;
  }
  GemmBatch g;
  g.segs.push_back({a, b, lda, ldb, k, flags, alpha});
  g.add_problem(c, ldc, m, n, 0, 1, beta);
  launch_gemm(g, desc, s);
}

// One renormalisation step backwards: the adjoints an of the new block's
// operators give the gradient of the step's coefficients and the adjoints
// (added to ao) of the old block's integral-dependent operators.
void step_back(const Mps& m, const Env& old, const Env& neu, const CompProv& rec, const Adj& an,
               Adj& ao, std::vector<double>& grad, Work& w, hipStream_t s, BackwardStats& stats) {
  const int side = neu.side;
  const int site = side > 0 ? old.bond : neu.bond;
  const Kinds ko = kinds_of(old), kn = kinds_of(neu);
  struct Group {
    std::map<int, std::vector<std::pair<int, const CompKey*>>> by_t;  // target -> (source, key)
    std::set<int> srcs;
  };
  std::map<std::tuple<int, uint64_t, int>, Group> groups;
  for (auto& kv : rec.coef) {
    int tc, ti, sc, si;
    uint64_t yk;
    std::tie(tc, ti, sc, si, yk) = kv.first;
    if (!dependent(kn[tc][ti])) continue;
    const bool dep = dependent(ko[sc][si]);
    if (!dep && !rec.prov.count(kv.first)) continue;
    if (dep && kv.second == 0.0) continue;
    Group& g = groups[std::make_tuple(tc, yk, sc)];
    g.by_t[ti].push_back({si, &kv.first});
    g.srcs.insert(si);
  }
  for (auto& gk : groups) {
    ++stats.n_groups;
    const int tc = std::get<0>(gk.first), sc = std::get<2>(gk.first);
    const Str ys = Str::from_key(std::get<1>(gk.first));
    const Mat4 y = site_matrix(ys);
    const int ypar = ys.parity();
    const Group& g = gk.second;
    const OpClass& T = *neu.classes[tc];
    const OpClass& S = *old.classes[sc];
    const int64_t nnzS = S.L.nnz, nnzT = T.L.nnz;
    std::vector<int> tids;
    for (auto& t : g.by_t) tids.push_back(t.first);
    const int nt = (int)tids.size();
    std::vector<int> prov_src, dep_src;
    for (int si : g.srcs) (dependent(ko[sc][si]) ? dep_src : prov_src).push_back(si);
    const int ns = (int)g.srcs.size();
    auto add_grad = [&](int ti, int si, double gval) {
      for (auto& e : g.by_t.at(ti))
        if (e.first == si) {
          auto it = rec.prov.find(*e.second);
          if (it == rec.prov.end()) continue;
          for (auto& pe : it->second) grad[(size_t)pe.first] += pe.second * gval;
        }
    };
    if (nt <= ns) {
      // adjoint first: M[k] = Proj^T(N_bar[t_k], y) on the old bond
      grow(w.tmp, (size_t)std::max<int64_t>(1, (int64_t)nt * nnzS) * sizeof(double), s);
      double* M = w.tmp.as<double>();
      launch_fill(M, 0.0, (int64_t)nt * nnzS, s);
      std::vector<Projection> pj;
      for (int k = 0; k < nt; ++k)
        pj.push_back({an.op(neu, tc, tids[k]), &T.L, y, ypar, M + (int64_t)k * nnzS, &S.L, 1.0});
      run_adjoint_projections(side, m, site, pj, w.desc, w.uws, kProjBudget, s);
      if (!prov_src.empty()) {
        // G (nt x nops_S) = M S^T
        grow(w.gout, (size_t)std::max(1, nt * S.nops) * sizeof(double), s);
        gemm(w.gout.p, S.nops, nt, S.nops, M, (int)nnzS, S.data.p, (int)nnzS, (int)nnzS, kTransB, 1.0,
             0, w.desc, s);
        const auto& G = fetch(w, (int64_t)nt * S.nops, s);
        for (int k = 0; k < nt; ++k)
          for (int si : prov_src) add_grad(tids[k], si, G[(size_t)k * S.nops + si]);
      }
      if (!dep_src.empty()) {
        // ao[sc] (nops_S x nnz) += C^T M, C[k][s] = coefficient of (t_k, s)
        std::vector<double> Ct((size_t)S.nops * nt, 0.0);
        for (int k = 0; k < nt; ++k)
          for (auto& e : g.by_t.at(tids[k]))
            if (dependent(ko[sc][e.first])) Ct[(size_t)e.first * nt + k] += rec.coef.at(*e.second);
        upload(w.coef, Ct, s);
        gemm(ao.cls[sc].p, (int)nnzS, S.nops, (int)nnzS, w.coef.p, nt, M, (int)nnzS, nt, 0, 1.0, 1,
             w.desc, s);
      }
    } else {
      // project first
      if (!prov_src.empty()) {
        const int np = (int)prov_src.size();
        grow(w.tmp, (size_t)std::max<int64_t>(1, (int64_t)np * nnzT) * sizeof(double), s);
        double* Pj = w.tmp.as<double>();
        launch_fill(Pj, 0.0, (int64_t)np * nnzT, s);
        std::vector<Projection> pj;
        for (int k = 0; k < np; ++k)
          pj.push_back({S.op(prov_src[k]), &S.L, y, ypar, Pj + (int64_t)k * nnzT, &T.L, 1.0});
        run_projections(side, m, site, pj, w.desc, w.uws, kProjBudget, s);
        // G (nops_T x np) = N_bar_T P^T
        grow(w.gout, (size_t)std::max(1, T.nops * np) * sizeof(double), s);
        gemm(w.gout.p, np, T.nops, np, an.cls[tc].p, (int)nnzT, Pj, (int)nnzT, (int)nnzT, kTransB, 1.0,
             0, w.desc, s);
        const auto& G = fetch(w, (int64_t)T.nops * np, s);
        for (int ti : tids)
          for (int k = 0; k < np; ++k) add_grad(ti, prov_src[k], G[(size_t)ti * np + k]);
      }
      if (!dep_src.empty()) {
        // X (nd x nnz_T) = C^T N_bar_T, then ao[s] += Proj^T(X_s, y)
        const int nd = (int)dep_src.size();
        std::map<int, int> dpos;
        for (int k = 0; k < nd; ++k) dpos[dep_src[k]] = k;
        std::vector<double> Ct((size_t)nd * T.nops, 0.0);
        for (int ti : tids)
          for (auto& e : g.by_t.at(ti))
            if (dpos.count(e.first)) Ct[(size_t)dpos[e.first] * T.nops + ti] += rec.coef.at(*e.second);
        upload(w.coef, Ct, s);
        grow(w.tmp2, (size_t)std::max<int64_t>(1, (int64_t)nd * nnzT) * sizeof(double), s);
        gemm(w.tmp2.p, (int)nnzT, nd, (int)nnzT, w.coef.p, T.nops, an.cls[tc].p, (int)nnzT, T.nops, 0,
             1.0, 0, w.desc, s);
        std::vector<Projection> pj;
        for (int k = 0; k < nd; ++k)
          pj.push_back({w.tmp2.as<double>() + (int64_t)k * nnzT, &T.L, y, ypar, ao.op(old, sc, dep_src[k]),
                        &S.L, 1.0});
        run_adjoint_projections(side, m, site, pj, w.desc, w.uws, kProjBudget, s);
      }
    }
    DMRG_HIP(hipStreamSynchronize(s));
  }
}

// Window adjoints of the pairs' integral-dependent operators.
void window_back(const Mps& m, const SigmaPlan& plan, const Env& L, const Env& R, const double* lam_pad,
                 Adj& aL, Adj& aW, Adj& aR, int64_t budget, Work& w, hipStream_t s) {
  const int i = plan.window;
  const Bond& bl = m.bonds[i];
  const Bond& br = m.bonds[i + 2];
  const PsiLayout& ps = plan.psi;
  const Env& W = *plan.psums;
  const Kinds kL = kinds_of(L), kR = kinds_of(R);
  const double* Ppad = plan.bufs[plan.buf_psi].f64;
  const double* PT = plan.bufs[plan.buf_psit].f64;
  auto ldep = [&](const SigmaPair& p) {
    return p.lsrc == 1 || dependent(kL[p.lref.cls][p.lref.idx]);
  };
  auto zdep = [&](const SigmaPair& p) {
    return p.z >= 0 && dependent(kR[plan.zrefs[p.z].cls][plan.zrefs[p.z].idx]);
  };
  std::set<int> zl, zz;
  for (auto& p : plan.pairs) {
    if (ldep(p) && p.z >= 0) zl.insert(p.z);
    if (zdep(p)) zz.insert(p.z);
  }
  const int nz = (int)plan.zops.size();
  auto zsize = [&](int z) {
    int64_t n = 0;
    for (auto& blk : plan.zops[z].lay->blk)
      if (ps.rows_of[blk.c] > 0 && ps.rows_of[blk.r] > 0) n += ps.rows_pad[blk.c] * br.d[blk.r];
    return n;
  };
  // chunks over z (each z needs T (left-dependent pairs) and/or U_bar)
  std::vector<std::pair<int, int>> chunks;
  {
    int z0 = 0;
    int64_t acc = 0;
    for (int z = 0; z < nz; ++z) {
      const int64_t need = (zl.count(z) + zz.count(z)) * zsize(z);
      if (z > z0 && acc + need > budget) {
        chunks.push_back({z0, z});
        z0 = z;
        acc = 0;
      }
      acc += need;
    }
    chunks.push_back({z0, std::max(nz, z0 + 1)});
  }
  for (size_t ci = 0; ci < chunks.size(); ++ci) {
    const int z0 = chunks[ci].first, z1 = chunks[ci].second;
    std::map<std::pair<int, int>, int64_t> tloc, uloc;  // (z, r) -> ws offset (d_r' x rows_pad_r)
    int64_t off = 0;
    for (int z = z0; z < std::min(z1, nz); ++z)
      for (auto& blk : plan.zops[z].lay->blk) {
        const int r = blk.c, rp = blk.r;
        if (ps.rows_of[r] == 0 || ps.rows_of[rp] == 0) continue;
        const int64_t n = ps.rows_pad[r] * br.d[rp];
        if (zl.count(z)) { tloc[{z, r}] = off; off += n; }
        if (zz.count(z)) { uloc[{z, r}] = off; off += n; }
      }
    grow(w.tmp, (size_t)std::max<int64_t>(1, off) * sizeof(double), s);
    double* ws = w.tmp.as<double>();
    launch_fill(ws, 0.0, std::max<int64_t>(1, off), s);
    // B1: T^T[z, r] = a Z(r', r) psi_r^T   (as the forward's first stage)
    GemmBatch b1;
    for (auto& t : tloc) {
      const int z = t.first.first, r = t.first.second;
      const OpView& Z = plan.zops[z];
      const Layout::Blk* blk = Z.lay->col(r);
      const double alpha = (plan.zpar[z] && (br.q[r].n & 1)) ? -1.0 : 1.0;
      const size_t s0 = b1.segs.size();
      b1.segs.push_back({Z.data + blk->off, Ppad + ps.off_pad[r], blk->ld, ps.ld[r], br.d[r], kTransB, alpha});
      b1.add_problem(ws + t.second, (int)ps.rows_pad[r], br.d[blk->r], (int)ps.rows_pad[r], s0, s0 + 1, 0);
    }
    launch_gemm(b1, w.desc, s);
    // B2 (left adjoints) and B3 (U_bar), output-stationary
    std::map<double*, std::vector<GemmSeg>> outL, outU;
    std::map<double*, std::array<int, 3>> shapeL, shapeU;  // m, n, ldc
    for (auto& pr : plan.pairs) {
      const bool dl = ldep(pr) && (pr.z < 0 ? ci == 0 : (pr.z >= z0 && pr.z < z1));
      const bool dz = zdep(pr) && pr.z >= z0 && pr.z < z1;
      if (!dl && !dz) continue;
      const Layout& Ll = *pr.L.lay;
      const Env& LE = pr.lsrc ? W : L;
      const Adj& LA = pr.lsrc ? aW : aL;
      for (int np = 0; np < 16; ++np)
        for (int n = 0; n < 16; ++n) {
          const double yv = pr.y.m[np][n];
          if (yv == 0) continue;
          const QN qn = kSiteQN[n >> 2] + kSiteQN[n & 3];
          const QN qnp = kSiteQN[np >> 2] + kSiteQN[np & 3];
          for (auto& lb : Ll.blk) {
            const int l = lb.c, lp = lb.r;
            const int r = br.find(bl.q[l] + qn);
            const int rp = br.find(bl.q[lp] + qnp);
            if (r < 0 || rp < 0) continue;
            auto kr = ps.row_pad_of[r].find({l, n});
            auto krp = ps.row_pad_of[rp].find({lp, np});
            if (kr == ps.row_pad_of[r].end() || krp == ps.row_pad_of[rp].end()) continue;
            if (pr.z >= 0) {
              const Layout::Blk* zb = plan.zops[pr.z].lay->col(r);
              if (!zb || zb->r != rp) continue;
            } else if (r != rp) {
              continue;
            }
            const double sg = ((pr.ypar & 1) && (bl.q[l].n & 1)) ? -1.0 : 1.0;
            const double* lamb = lam_pad + ps.off_pad[rp] + krp->second * ps.ld[rp];
            if (dl) {
              // L_bar[l', l] += lam(l', n') (d_l' x d_r') . T^T[z, r](:, (l, n)) (d_r' x d_l)
              const double* B = pr.z < 0 ? PT + ps.offT[r] + kr->second
                                         : ws + tloc.at({pr.z, r}) + kr->second;
              double* out = LA.op(LE, pr.lref.cls, pr.lref.idx) + lb.off;
              outL[out].push_back({lamb, B, ps.ld[rp], (int)ps.rows_pad[r], br.d[rp], 0, yv * sg});
              shapeL[out] = {lb.dr, lb.dc, lb.ld};
            }
            if (dz) {
              // U_bar^T[z, r](:, (l, n)) += lam(l', n')^T (d_r' x d_l') . L[l', l]
              double* out = ws + uloc.at({pr.z, r}) + kr->second;
              outU[out].push_back({lamb, pr.L.data + lb.off, ps.ld[rp], lb.ld, lb.dr, kTransA, yv * sg});
              shapeU[out] = {br.d[rp], lb.dc, (int)ps.rows_pad[r]};
            }
          }
        }
    }
    GemmBatch b2;
    for (auto* o : {&outL, &outU}) {
      auto& shp = o == &outL ? shapeL : shapeU;
      for (auto& kv : *o) {
        const size_t s0 = b2.segs.size();
        for (auto& g : kv.second) b2.segs.push_back(g);
        const auto& sh = shp[kv.first];
        b2.add_problem(kv.first, sh[2], sh[0], sh[1], s0, b2.segs.size(), 1);
      }
    }
    launch_gemm(b2, w.desc, s);
    // B4: Z_bar[r', r] += a U_bar^T[z, r] psi_r
    GemmBatch b4;
    for (auto& u : uloc) {
      const int z = u.first.first, r = u.first.second;
      const OpRef& zr = plan.zrefs[z];
      const Layout::Blk* blk = plan.zops[z].lay->col(r);
      const double alpha = (plan.zpar[z] && (br.q[r].n & 1)) ? -1.0 : 1.0;
      const size_t s0 = b4.segs.size();
      b4.segs.push_back({ws + u.second, Ppad + ps.off_pad[r], (int)ps.rows_pad[r], ps.ld[r],
                         (int)ps.rows_pad[r], 0, alpha});
      b4.add_problem(aR.op(R, zr.cls, zr.idx) + blk->off, blk->ld, blk->dr, blk->dc, s0, s0 + 1, 1);
    }
    launch_gemm(b4, w.desc, s);
    DMRG_HIP(hipStreamSynchronize(s));
  }
}

}  // namespace

BackwardStats sigma_backward(const Problem& P0, const Mps& m, int window, const double* psi,
                             const double* lam, double* grad_out, int64_t ws_budget, hipStream_t s,
                             int precision) {
  BackwardStats st;
  const int K = P0.K, i = window;
  DMRG_REQUIRE(i >= 0 && i + 1 < K, kErrInvalidArg, "sigma_backward: bad window");
  Problem P = P0;
  P.all_terms = true;  // every integral entry is an input, zero or not
  std::vector<double> grad((size_t)K * K + (size_t)K * K * K * K, 0.0);
  Work w;
  // ---- rebuild both blocks, recording the components ----------------------
  double t0 = now_ms();
  std::vector<std::unique_ptr<Env>> Ls(i + 1), Rs(K + 1);
  std::vector<CompProv> recL(i + 1), recR(K + 1);
  Ls[0] = left_start(m, s);
  for (int b = 0; b < i; ++b) Ls[b + 1] = grow_left(P, m, *Ls[b], w.desc, s, &recL[b + 1]);
  Rs[K] = right_start(m, s);
  for (int b = K; b > i + 2; --b) Rs[b - 1] = grow_right(P, m, *Rs[b], w.desc, s, &recR[b - 1]);
  auto plan = plan_sigma(P, m, *Ls[i], *Rs[i + 2], ws_budget, s, true);
  DMRG_HIP(hipStreamSynchronize(s));
  st.ms_chain = now_ms() - t0;
  // ---- window ---------------------------------------------------------------
  // Every contraction from here on runs in the requested precision; the
  // gradient itself is accumulated in FP64 on the host.
  GemmPrecisionScope scope(precision);
  t0 = now_ms();
  const int64_t npad = plan->psi.size_pad;
  DevBuf lam_pad((size_t)std::max<int64_t>(1, npad) * sizeof(double));
  plan_load_psi(*plan, lam, s);
  DMRG_HIP(hipMemcpyAsync(lam_pad.p, plan->bufs[plan->buf_psi].f64, (size_t)npad * sizeof(double),
                          hipMemcpyDeviceToDevice, s));
  plan_load_psi(*plan, psi, s);
  std::vector<Adj> aL(i + 1), aR(K + 1);
  Adj aW;
  alloc_adj(*Ls[i], aL[i], s);
  alloc_adj(*Rs[i + 2], aR[i + 2], s);
  alloc_adj(*plan->psums, aW, s);
  window_back(m, *plan, *Ls[i], *Rs[i + 2], lam_pad.as<double>(), aL[i], aW, aR[i + 2], ws_budget, w, s);
  // partial sums: W = C x_L, so dC = W_bar x_L^T
  const Env& W = *plan->psums;
  for (auto& wc : plan->w_src_cls) {
    const OpClass& Wc = *W.classes[wc.first];
    const OpClass& Sc = *Ls[i]->classes[wc.second];
    const int64_t nnz = Wc.L.nnz;
    grow(w.gout, (size_t)std::max(1, Wc.nops * Sc.nops) * sizeof(double), s);
    gemm(w.gout.p, Sc.nops, Wc.nops, Sc.nops, aW.cls[wc.first].p, (int)nnz, Sc.data.p, (int)nnz, (int)nnz,
         kTransB, 1.0, 0, w.desc, s);
    const auto& G = fetch(w, (int64_t)Wc.nops * Sc.nops, s);
    for (auto& wk : plan->wkeys) {
      if (wk.second.cls != wc.first) continue;
      auto it = plan->psum_prov.find(wk.first);
      if (it == plan->psum_prov.end()) continue;
      for (auto& src : it->second)
        for (auto& pe : src.second)
          grad[(size_t)pe.first] += pe.second * G[(size_t)wk.second.idx * Sc.nops + src.first.second];
    }
  }
  DMRG_HIP(hipStreamSynchronize(s));
  plan.reset();
  st.ms_window = now_ms() - t0;
  // ---- adjoint renormalisation along both chains -------------------------------
  t0 = now_ms();
  for (int b = i; b >= 1; --b) {
    alloc_adj(*Ls[b - 1], aL[b - 1], s);
    step_back(m, *Ls[b - 1], *Ls[b], recL[b], aL[b], aL[b - 1], grad, w, s, st);
    aL[b].cls.clear();
    Ls[b].reset();
  }
  for (int b = i + 2; b <= K - 1; ++b) {
    alloc_adj(*Rs[b + 1], aR[b + 1], s);
    step_back(m, *Rs[b + 1], *Rs[b], recR[b], aR[b], aR[b + 1], grad, w, s, st);
    aR[b].cls.clear();
    Rs[b].reset();
  }
  DMRG_HIP(hipStreamSynchronize(s));
  st.ms_adjoint = now_ms() - t0;
  std::copy(grad.begin(), grad.end(), grad_out);
  return st;
}

}  // namespace dmrg

namespace dmrg {

void orbital_gradient(const Problem& P, const double* dh, const double* deri, double* fock,
                      double* grad, hipStream_t s) {
  const int K = P.K;
  const int64_t K2 = (int64_t)K * K, K3 = K2 * K;
  DMRG_REQUIRE(K3 < ((int64_t)1 << 31), kErrShape, "orbital_gradient: K^3 exceeds the GEMM index range");
  std::vector<double> eye((size_t)K2, 0.0);
  for (int p = 0; p < K; ++p) eye[(size_t)p * K + p] = 1.0;
  DevBuf dH((size_t)K2 * sizeof(double)), dE((size_t)(K3 * K) * sizeof(double)),
      dI((size_t)K2 * sizeof(double)), dF((size_t)K2 * sizeof(double)), desc;
  DMRG_HIP(hipMemcpyAsync(dH.p, P.h.data(), (size_t)K2 * sizeof(double), hipMemcpyHostToDevice, s));
  DMRG_HIP(hipMemcpyAsync(dE.p, P.eri.data(), (size_t)(K3 * K) * sizeof(double), hipMemcpyHostToDevice, s));
  DMRG_HIP(hipMemcpyAsync(dI.p, eye.data(), (size_t)K2 * sizeof(double), hipMemcpyHostToDevice, s));
  double* F = fock ? fock : dF.as<double>();
  // F = gamma h^T + (2 deri)(K x K^3) eri(K x K^3)^T
  GemmBatch f;
  f.segs.push_back({dh, dH.p, K, K, K, kTransB, 1.0});
  f.segs.push_back({deri, dE.p, (int)K3, (int)K3, (int)K3, kTransB, 2.0});
  f.add_problem(F, K, K, K, 0, 2, 0);
  launch_gemm_f64(f, s);
  // g = 2 F^T I - 2 F I
  GemmBatch g;
  g.segs.push_back({F, dI.p, K, K, K, kTransA, 2.0});
  g.segs.push_back({F, dI.p, K, K, K, 0, -2.0});
  g.add_problem(grad, K, K, K, 0, 2, 0);
  launch_gemm_f64(g, s);
  DMRG_HIP(hipStreamSynchronize(s));
}

}  // namespace dmrg
