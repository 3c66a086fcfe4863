// Construction of renormalised block operators and the two-site sigma plan.
//
// Every operator of a block is either a normal-ordered string of at most two
// creation/annihilation operators, the block Hamiltonian, the identity, or a
// "complementary" sum of Hamiltonian terms (standard ab initio DMRG: White and
// Martin 1999; Chan and Head-Gordon 2002).  All of them are derived from one
// rule: split every term of H by the regions of its spin-orbitals (block,
// site, rest) with the Jordan-Wigner exchange sign, and route the block part
// either to a stored operator or to a linear combination of stored operators.
//
//   left block  (sites [0, b)): identity, H, strings of length 1 and 2,
//               T(w) = sum over three-operator block parts x of coef(x w) x,
//               for every one-operator string w outside the block;
//   right block (sites [b, K)): identity, H, strings of length 1,
//               S(w) = sum over one- and three-operator parts (w outside),
//               Q(w) = sum over two-operator parts (w a two-operator string).
//
// A new block operator is sum_c coef_c * Proj(X_c (x) y_c) with X_c an old
// block operator and y_c a 4x4 site matrix; Proj is the projection with the
// site tensor (A^T (X (x) y) A on the left, B (y (x) X) B^T on the right).
// Linear combinations are dense GEMMs over operator classes (operators with
// the same quantum-number change share one block layout); projections are
// two-stage grouped GEMMs.
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <map>
#include <set>
#include <tuple>
#include <unordered_set>

namespace dmrg {

// ---------------------------------------------------------------------------
void Env::allocate(hipStream_t s) {
  for (auto& c : classes) {
    c->data.alloc((size_t)std::max<int64_t>(1, c->nops * c->L.nnz) * sizeof(double));
    launch_fill(c->data.as<double>(), 0.0, c->nops * c->L.nnz, s);
  }
}

// Writes the exact identity into the registered identity operator.
static void set_identity(Env& e, hipStream_t s) {
  const OpRef* r = e.get({kIdent, 0});
  if (!r) return;
  OpClass& c = *e.classes[r->cls];
  std::vector<double> h((size_t)c.L.nnz, 0.0);
  for (auto& b : c.L.blk)
    for (int i = 0; i < b.dr; ++i) h[(size_t)b.off + (size_t)i * b.ld + i] = 1.0;
  DMRG_HIP(hipStreamSynchronize(s));
  DMRG_HIP(hipMemcpy(c.op(r->idx), h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
}

// All canonical strings with n operators over the spin-orbitals `so`.
static void strings_over(const std::vector<int>& so, int n, std::vector<Str>& out) {
  const int m = (int)so.size();
  for (int nc = 0; nc <= n; ++nc) {
    int na = n - nc;
    if (nc > m || na > m) continue;
    std::vector<int> ci(nc), ai(na);
    // enumerate combinations
    std::function<void(int, int, std::vector<int>&, std::vector<std::vector<int>>&)> comb;
    comb = [&](int start, int k, std::vector<int>& cur, std::vector<std::vector<int>>& res) {
      if ((int)cur.size() == k) { res.push_back(cur); return; }
      for (int x = start; x < m; ++x) { cur.push_back(x); comb(x + 1, k, cur, res); cur.pop_back(); }
    };
    std::vector<std::vector<int>> cs, as;
    std::vector<int> cur;
    comb(0, nc, cur, cs);
    comb(0, na, cur, as);
    for (auto& c : cs)
      for (auto& a : as) {
        Str s;
        for (int x : c) s.push(so[x], 1);
        for (int x : a) s.push(so[x], 0);
        out.push_back(s);
      }
  }
}

static std::unique_ptr<Env> start_env(const Mps& m, int side, hipStream_t s) {
  auto e = std::make_unique<Env>();
  e->side = side;
  e->bond = side > 0 ? 0 : m.K;
  e->basis = m.bonds[e->bond];
  e->add({kIdent, 0}, QN{0, 0});
  e->allocate(s);
  set_identity(*e, s);
  return e;
}
std::unique_ptr<Env> left_start(const Mps& m, hipStream_t s) { return start_env(m, +1, s); }
std::unique_ptr<Env> right_start(const Mps& m, hipStream_t s) { return start_env(m, -1, s); }

// ---------------------------------------------------------------------------
// Components and their execution.
namespace {

struct Target {
  OpRef ref;
};

using CompMap = std::map<CompKey, double>;
// key: (target cls, target idx, source cls, source idx, site-string key)

thread_local CompProv* g_rec = nullptr;  // set while a backward rebuild records provenance

void add_comp(CompMap& cm, const OpRef& t, const OpRef* src, const Str& y, double c,
              int64_t entry = -1, double factor = 0.0) {
  if (!src || (c == 0.0 && !(g_rec && entry >= 0))) return;
  const CompKey k = std::make_tuple(t.cls, t.idx, src->cls, src->idx, y.key());
  cm[k] += c;
  if (g_rec && entry >= 0) g_rec->prov[k].push_back({entry, factor});
}

}  // namespace

// Emits the two-stage GEMMs of a list of projections, in chunks bounded by the
// intermediate workspace, and runs them.
void run_projections(int side, const Mps& m, int site, const std::vector<Projection>& projs,
                     DevBuf& desc, DevBuf& uws, int64_t budget, hipStream_t s) {
  const SiteTensor& st = m.site[site];
  const double* S = st.data.as<double>();
  const Bond& oldb = side > 0 ? m.bonds[site] : m.bonds[site + 1];
  const Bond& newb = side > 0 ? m.bonds[site + 1] : m.bonds[site];
  size_t p = 0;
  while (p < projs.size()) {
    // size the chunk
    int64_t need = 0;
    size_t q = p;
    for (; q < projs.size(); ++q) {
      int64_t u = 0;
      const Projection& pr = projs[q];
      for (auto& tb : pr.dl->blk)
        for (int n = 0; n < 4; ++n)
          for (int np = 0; np < 4; ++np) {
            if (pr.y.m[np][n] == 0) continue;
            if (side > 0) {
              int lp = oldb.find(newb.q[tb.r] - kSiteQN[np]);
              if (lp >= 0) u += (int64_t)oldb.d[lp] * newb.d[tb.c];
            } else {
              int rp = oldb.find(newb.q[tb.r] + kSiteQN[np]);
              if (rp >= 0) u += (int64_t)oldb.d[rp] * newb.d[tb.c];
            }
          }
      if (q > p && need + u > budget) break;
      need += u;
    }
    if ((int64_t)(uws.bytes / sizeof(double)) < need) {
      DMRG_HIP(hipStreamSynchronize(s));
      uws.alloc((size_t)std::max<int64_t>(need, 1) * sizeof(double));
    }
    double* U = uws.as<double>();
    int64_t uoff = 0;
    GemmBatch b1, b2;
    for (size_t k = p; k < q; ++k) {
      const Projection& pr = projs[k];
      const int xpar = pr.sl->dq.n & 1;
      for (auto& tb : pr.dl->blk) {
        const size_t s0 = b2.segs.size();
        for (int n = 0; n < 4; ++n)
          for (int np = 0; np < 4; ++np) {
            const double yv = pr.y.m[np][n];
            if (yv == 0) continue;
            if (side > 0) {
              // target (r', r) = (tb.r, tb.c) on the new bond
              const int r = tb.c, rp = tb.r;
              const int l = oldb.find(newb.q[r] - kSiteQN[n]);
              const int lp = oldb.find(newb.q[rp] - kSiteQN[np]);
              if (l < 0 || lp < 0) continue;
              const Layout::Blk* xb = pr.sl->col(l);
              if (!xb || xb->r != lp) continue;
              const int64_t oa = st.off[4 * l + n], oap = st.off[4 * lp + np];
              if (oa < 0 || oap < 0) continue;
              const int dl = oldb.d[l], dlp = oldb.d[lp], dr = newb.d[r], drp = newb.d[rp];
              double* u = U + uoff;
              uoff += (int64_t)dlp * dr;
              const size_t t0 = b1.segs.size();
              b1.segs.push_back({pr.src + xb->off, S + oa, xb->ld, dr, dl, 0, 1.0});
              b1.add_problem(u, dr, dlp, dr, t0, t0 + 1, 0);
              double sg = ((pr.ypar & 1) && (oldb.q[l].n & 1)) ? -1.0 : 1.0;
              b2.segs.push_back({S + oap, u, drp, dr, dlp, kTransA, pr.alpha * yv * sg});
            } else {
              // target (l', l) = (tb.r, tb.c) on the new bond
              const int l = tb.c, lp = tb.r;
              const int r = oldb.find(newb.q[l] + kSiteQN[n]);
              const int rp = oldb.find(newb.q[lp] + kSiteQN[np]);
              if (r < 0 || rp < 0) continue;
              const Layout::Blk* xb = pr.sl->col(r);
              if (!xb || xb->r != rp) continue;
              const int64_t ob = st.off[4 * l + n], obp = st.off[4 * lp + np];
              if (ob < 0 || obp < 0) continue;
              const int dr = oldb.d[r], drp = oldb.d[rp], dl = newb.d[l], dlp = newb.d[lp];
              double* u = U + uoff;
              uoff += (int64_t)drp * dl;
              const size_t t0 = b1.segs.size();
              b1.segs.push_back({pr.src + xb->off, S + ob, xb->ld, dr, dr, kTransB, 1.0});
              b1.add_problem(u, dl, drp, dl, t0, t0 + 1, 0);
              double sg = (xpar && (kSiteN[n] & 1)) ? -1.0 : 1.0;
              b2.segs.push_back({S + obp, u, drp, dl, drp, 0, pr.alpha * yv * sg});
            }
          }
        const size_t s1 = b2.segs.size();
        b2.add_problem(pr.dst + tb.off, tb.ld, tb.dr, tb.dc, s0, s1, 1);
      }
    }
    launch_gemm(b1, desc, s);
    launch_gemm(b2, desc, s);
    p = q;
  }
}

namespace {

// Runs a list of projections whose targets may repeat: rounds in which every
// target appears once (tiles of one launch must not overlap), each round as
// few launches as the intermediate budget allows.
void run_projection_rounds(int side, const Mps& m, int site, std::vector<Projection> projs,
                           DevBuf& desc, DevBuf& uws, int64_t budget, hipStream_t s) {
  std::stable_sort(projs.begin(), projs.end(),
                   [](const Projection& a, const Projection& b) { return a.dst < b.dst; });
  std::vector<std::vector<Projection>> rounds;
  for (size_t k = 0; k < projs.size();) {
    size_t e = k;
    while (e < projs.size() && projs[e].dst == projs[k].dst) ++e;
    for (size_t j = k; j < e; ++j) {
      if (rounds.size() <= j - k) rounds.emplace_back();
      rounds[j - k].push_back(projs[j]);
    }
    k = e;
  }
  for (auto& r : rounds) run_projections(side, m, site, r, desc, uws, budget, s);
}

// Executes all components: new = sum coef * Proj(old (x) y).
//
// Components are grouped by (target class, site string, source class).  A
// group with one source per target is a plain projection; otherwise the
// cheaper order is taken: with fewer targets than sources the sources are
// combined first (X = Coef S, one dense GEMM, then X projected), else every
// source is projected first into a temporary and the temporaries combined
// into the targets (T += Coef P).  All groups of a step run together: the
// combinations of every group are one grouped launch, every projection goes
// into one list (rounds with distinct targets), and the final combinations
// are grouped launches in rounds with disjoint target rows.  Temporaries are
// bounded by a budget; groups beyond it run in further batches.
void execute(const Env& old, Env& neu, const CompMap& cm, const Mps& m, int site,
             DevBuf& desc, hipStream_t s) {
  const int64_t kBudget = (int64_t)1 << 28;     // doubles of projection intermediates (2 GiB)
  const int64_t kTmpBudget = (int64_t)1 << 28;  // doubles of group temporaries per batch (2 GiB)
  struct Group {
    std::map<int, std::vector<std::pair<int, double>>> by_t;  // target idx -> (src idx, c)
    std::set<int> srcs;
  };
  std::map<std::tuple<int, uint64_t, int>, Group> groups;
  for (auto& kv : cm) {
    int tc, ti, sc, si;
    uint64_t yk;
    std::tie(tc, ti, sc, si, yk) = kv.first;
    if (kv.second == 0.0) continue;
    Group& g = groups[std::make_tuple(tc, yk, sc)];
    g.by_t[ti].push_back({si, kv.second});
    g.srcs.insert(si);
  }
  DevBuf uws;
  std::vector<Projection> direct;
  struct Multi {
    const Group* g;
    int tc, sc, ypar;
    Mat4 y;
    bool sum_first;
    int64_t tmp_doubles;
  };
  std::vector<Multi> multi;
  for (auto& gk : groups) {
    const int tc = std::get<0>(gk.first), sc = std::get<2>(gk.first);
    const Str ys = Str::from_key(std::get<1>(gk.first));
    const Mat4 y = site_matrix(ys);
    const int ypar = ys.parity();
    const Group& g = gk.second;
    const OpClass& T = *neu.classes[tc];
    const OpClass& S = *old.classes[sc];
    bool single = true;
    for (auto& t : g.by_t) single = single && t.second.size() == 1;
    const int nt = (int)g.by_t.size(), ns = (int)g.srcs.size();
    if (single) {
      for (auto& t : g.by_t)
        direct.push_back({S.op(t.second[0].first), &S.L, y, ypar, T.op(t.first), &T.L,
                          t.second[0].second});
      continue;
    }
    const bool sf = nt <= ns;
    multi.push_back({&g, tc, sc, ypar, y, sf, sf ? (int64_t)nt * S.L.nnz : (int64_t)ns * T.L.nnz});
  }
  DevBuf tmp, coef;
  std::vector<std::vector<double>> host_coef;  // kept until the stream is synchronised
  size_t g0 = 0;
  bool first = true;
  while (g0 < multi.size() || first) {
    // one batch of groups within the temporary budget
    size_t g1 = g0;
    int64_t need = 0;
    while (g1 < multi.size() && (g1 == g0 || need + multi[g1].tmp_doubles <= kTmpBudget))
      need += multi[g1++].tmp_doubles;
    if (need > 0 && (int64_t)(tmp.bytes / sizeof(double)) < need) {
      DMRG_HIP(hipStreamSynchronize(s));
      tmp.alloc((size_t)need * sizeof(double));
    }
    // coefficient matrices of the batch in one upload
    std::vector<double> C;
    std::vector<int64_t> coff(g1 - g0), toff(g1 - g0);
    int64_t to = 0;
    for (size_t q = g0; q < g1; ++q) {
      const Multi& u = multi[q];
      const Group& g = *u.g;
      coff[q - g0] = (int64_t)C.size();
      toff[q - g0] = to;
      to += u.tmp_doubles;
      if (u.sum_first) {
        const OpClass& S = *old.classes[u.sc];
        const size_t base = C.size();
        C.resize(base + g.by_t.size() * (size_t)S.nops, 0.0);
        int row = 0;
        for (auto& t : g.by_t) {
          for (auto& sc2 : t.second) C[base + (size_t)row * S.nops + sc2.first] += sc2.second;
          ++row;
        }
      } else {
        const int ns = (int)g.srcs.size();
        std::map<int, int> spos;
        for (int sid : g.srcs) spos.emplace(sid, (int)spos.size());
        const int t0 = g.by_t.begin()->first, t1 = g.by_t.rbegin()->first + 1;
        const size_t base = C.size();
        C.resize(base + (size_t)(t1 - t0) * ns, 0.0);
        for (auto& t : g.by_t)
          for (auto& sc2 : t.second) C[base + (size_t)(t.first - t0) * ns + spos[sc2.first]] += sc2.second;
      }
    }
    if (!C.empty()) {
      if (coef.bytes < C.size() * sizeof(double)) {
        DMRG_HIP(hipStreamSynchronize(s));
        coef.alloc(C.size() * sizeof(double));
      }
      DMRG_HIP(hipMemcpyAsync(coef.p, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
    }
    double* cbase = coef.as<double>();
    double* tbase = tmp.as<double>();
    // sum first: X = Coef * S for every such group (one launch)
    GemmBatch comb;
    std::vector<Projection> projs;
    if (first) projs = direct;
    for (size_t q = g0; q < g1; ++q) {
      const Multi& u = multi[q];
      const Group& g = *u.g;
      const OpClass& S = *old.classes[u.sc];
      const OpClass& T = *neu.classes[u.tc];
      double* X = tbase + toff[q - g0];
      if (u.sum_first) {
        const int nt = (int)g.by_t.size();
        const size_t s0 = comb.segs.size();
        comb.segs.push_back({cbase + coff[q - g0], S.data.p, S.nops, (int)S.L.nnz, S.nops, 0, 1.0});
        comb.add_problem(X, (int)S.L.nnz, nt, (int)S.L.nnz, s0, s0 + 1, 0);
        int k = 0;
        for (auto& t : g.by_t)
          projs.push_back({X + (int64_t)(k++) * S.L.nnz, &S.L, u.y, u.ypar, T.op(t.first), &T.L, 1.0});
      } else {
        // project first into zeroed temporaries
        launch_fill(X, 0.0, u.tmp_doubles, s);
        int k = 0;
        for (int sid : g.srcs)
          projs.push_back({S.op(sid), &S.L, u.y, u.ypar, X + (int64_t)(k++) * T.L.nnz, &T.L, 1.0});
      }
    }
    launch_gemm_f64(comb, s);
    run_projection_rounds(neu.side, m, site, std::move(projs), desc, uws, kBudget, s);
    // project first: T += Coef * P, rounds of disjoint target rows
    struct Acc {
      int tc, t0, t1;
      size_t q;
    };
    std::vector<Acc> acc;
    for (size_t q = g0; q < g1; ++q)
      if (!multi[q].sum_first)
        acc.push_back({multi[q].tc, multi[q].g->by_t.begin()->first, multi[q].g->by_t.rbegin()->first + 1, q});
    while (!acc.empty()) {
      GemmBatch b;
      std::vector<Acc> rest;
      std::map<int, std::vector<std::pair<int, int>>> taken;  // class -> row ranges in this launch
      for (const Acc& a : acc) {
        bool clash = false;
        for (auto& r : taken[a.tc]) clash = clash || (a.t0 < r.second && r.first < a.t1);
        if (clash) {
          rest.push_back(a);
          continue;
        }
        taken[a.tc].push_back({a.t0, a.t1});
        const Multi& u = multi[a.q];
        const OpClass& T = *neu.classes[u.tc];
        const int ns = (int)u.g->srcs.size();
        const size_t s0 = b.segs.size();
        b.segs.push_back({cbase + coff[a.q - g0], tbase + toff[a.q - g0], ns, (int)T.L.nnz, ns, 0, 1.0});
        b.add_problem(T.op(a.t0), (int)T.L.nnz, a.t1 - a.t0, (int)T.L.nnz, s0, s0 + 1, 1);
      }
      launch_gemm_f64(b, s);
      acc.swap(rest);
    }
    host_coef.push_back(std::move(C));
    // the next batch reuses tmp and coef
    DMRG_HIP(hipStreamSynchronize(s));
    host_coef.clear();
    g0 = g1;
    first = false;
  }
}

std::vector<int> site_so(int b) { return {2 * b, 2 * b + 1}; }

}  // namespace

// ---------------------------------------------------------------------------
std::unique_ptr<Env> grow_left(const Problem& P, const Mps& m, const Env& old, DevBuf& desc,
                               hipStream_t s, CompProv* rec) {
  g_rec = rec;
  const int b = old.bond;
  DMRG_REQUIRE(old.side > 0 && b < m.K, kErrState, "grow_left: bad block");
  DMRG_REQUIRE(!m.site[b].off.empty(), kErrState, "grow_left: site tensor missing");
  auto e = std::make_unique<Env>();
  e->side = +1;
  e->bond = b + 1;
  e->basis = m.bonds[b + 1];
  const int M = 2 * (b + 1), Mall = 2 * P.K;
  auto region = [&](int p) { return p < 2 * b ? 0 : (p < M ? 1 : 2); };
  CompMap cm;
  const OpRef* oldI = old.get({kIdent, 0});
  // identity
  OpRef tI = e->add({kIdent, 0}, QN{0, 0});
  // normal strings of length 1 and 2
  std::vector<int> inner(M);
  for (int p = 0; p < M; ++p) inner[p] = p;
  std::vector<Str> normals;
  strings_over(inner, 1, normals);
  strings_over(inner, 2, normals);
  for (const Str& x : normals) {
    OpRef t = e->add({kNormal, x.key()}, x.qn());
    Str parts[3];
    int sg = split_regions(x, region, 3, parts);
    if (sg == 0) continue;
    const OpRef* src = parts[0].n ? old.get({kNormal, parts[0].key()}) : oldI;
    add_comp(cm, t, src, parts[1], (double)sg);
  }
  // complementary T(w) for one-operator strings w outside
  for (int p = M; p < Mall; ++p)
    for (int dag = 0; dag < 2; ++dag) {
      Str w;
      w.push(p, dag);
      e->add({kComp, w.key()}, -w.qn());
    }
  OpRef tH = e->add({kHam, 0}, QN{0, 0});
  // Hamiltonian terms with at most one spatial index outside [0, b]
  for_each_term(
      P, [&](const int* ix, int n) {
        int out = 0;
        for (int k = 0; k < n; ++k) out += ix[k] > b;
        return out <= 1;
      },
      [&](double c, const Str& term, int64_t ent, double fac) {
        Str parts[3];
        int sg = split_regions(term, region, 3, parts);
        if (sg == 0) return;
        const Str &x = parts[0], &y = parts[1], &z = parts[2];
        OpRef t;
        if (z.n == 0) t = tH;
        else if (z.n == 1 && x.n + y.n == 3) t = *e->get({kComp, z.key()});
        else return;
        if (x.n == 0) add_comp(cm, t, oldI, y, c * sg, ent, fac * sg);
        else if (x.n == 3) return;                       // inside T of the old block
        else if (y.n == 0 && z.n == 0) return;           // inside H of the old block
        else add_comp(cm, t, old.get({kNormal, x.key()}), y, c * sg, ent, fac * sg);
      });
  // pass-through of the old complementary operators and H
  Str none;
  add_comp(cm, tH, old.get({kHam, 0}), none, 1.0);
  std::vector<Str> y1;
  strings_over(site_so(b), 1, y1);
  for (const Str& y : y1) add_comp(cm, tH, old.get({kComp, y.key()}), y, 1.0);
  for (int p = M; p < Mall; ++p)
    for (int dag = 0; dag < 2; ++dag) {
      Str w;
      w.push(p, dag);
      add_comp(cm, *e->get({kComp, w.key()}), old.get({kComp, w.key()}), none, 1.0);
    }
  e->allocate(s);
  // the identity is exact by construction, not projected
  CompMap cm2;
  for (auto& kv : cm)
    if (!(std::get<0>(kv.first) == tI.cls && std::get<1>(kv.first) == tI.idx)) cm2.insert(kv);
  if (rec) rec->coef = cm2;
  g_rec = nullptr;
  execute(old, *e, cm2, m, b, desc, s);
  set_identity(*e, s);
  return e;
}

std::unique_ptr<Env> grow_right(const Problem& P, const Mps& m, const Env& old, DevBuf& desc,
                                hipStream_t s, CompProv* rec) {
  g_rec = rec;
  const int b = old.bond - 1;  // the new site
  DMRG_REQUIRE(old.side < 0 && b >= 0, kErrState, "grow_right: bad block");
  DMRG_REQUIRE(!m.site[b].off.empty(), kErrState, "grow_right: site tensor missing");
  auto e = std::make_unique<Env>();
  e->side = -1;
  e->bond = b;
  e->basis = m.bonds[b];
  const int M0 = 2 * b, Mall = 2 * P.K;
  auto region = [&](int p) { return p < M0 ? 0 : (p < M0 + 2 ? 1 : 2); };
  CompMap cm;
  const OpRef* oldI = old.get({kIdent, 0});
  OpRef tI = e->add({kIdent, 0}, QN{0, 0});
  // normal strings of length 1 on [2b, 2K)
  for (int p = M0; p < Mall; ++p)
    for (int dag = 0; dag < 2; ++dag) {
      Str x;
      x.push(p, dag);
      OpRef t = e->add({kNormal, x.key()}, x.qn());
      if (p < M0 + 2) add_comp(cm, t, oldI, x, 1.0);
      else add_comp(cm, t, old.get({kNormal, x.key()}), Str(), 1.0);
    }
  std::vector<int> outer(M0);
  for (int p = 0; p < M0; ++p) outer[p] = p;
  std::vector<Str> w1, w2;
  strings_over(outer, 1, w1);
  strings_over(outer, 2, w2);
  for (const Str& w : w1) e->add({kComp, w.key()}, -w.qn());
  for (const Str& w : w2) e->add({kComp, w.key()}, -w.qn());
  OpRef tH = e->add({kHam, 0}, QN{0, 0});
  for_each_term(
      P, [&](const int* ix, int n) {
        int out = 0;
        for (int k = 0; k < n; ++k) out += ix[k] < b;
        return out <= 2;
      },
      [&](double c, const Str& term, int64_t ent, double fac) {
        Str parts[3];
        int sg = split_regions(term, region, 3, parts);
        if (sg == 0) return;
        const Str &z = parts[0], &y = parts[1], &x = parts[2];
        OpRef t;
        const int inside = y.n + x.n;
        if (z.n == 0) t = tH;
        else if (z.n == 1 && (inside == 1 || inside == 3)) t = *e->get({kComp, z.key()});
        else if (z.n == 2 && inside == 2) t = *e->get({kComp, z.key()});
        else return;
        if (x.n == 0) add_comp(cm, t, oldI, y, c * sg, ent, fac * sg);
        else if (z.n + y.n <= 2) return;                 // inside H, S or Q of the old block
        else add_comp(cm, t, old.get({kNormal, x.key()}), y, c * sg, ent, fac * sg);
      });
  Str none;
  add_comp(cm, tH, old.get({kHam, 0}), none, 1.0);
  std::vector<Str> y1, y2;
  strings_over(site_so(b), 1, y1);
  strings_over(site_so(b), 2, y2);
  for (const Str& y : y1) add_comp(cm, tH, old.get({kComp, y.key()}), y, 1.0);
  for (const Str& y : y2) add_comp(cm, tH, old.get({kComp, y.key()}), y, 1.0);
  for (const Str& z : w1) {
    OpRef t = *e->get({kComp, z.key()});
    add_comp(cm, t, old.get({kComp, z.key()}), none, 1.0);
    for (const Str& y : y1) {
      Str w;
      int eps = concat_canonical(z, y, w);
      if (eps == 0) continue;
      add_comp(cm, t, old.get({kComp, w.key()}), y, (double)eps);
    }
  }
  for (const Str& z : w2) add_comp(cm, *e->get({kComp, z.key()}), old.get({kComp, z.key()}), none, 1.0);
  e->allocate(s);
  CompMap cm2;
  for (auto& kv : cm)
    if (!(std::get<0>(kv.first) == tI.cls && std::get<1>(kv.first) == tI.idx)) cm2.insert(kv);
  if (rec) rec->coef = cm2;
  g_rec = nullptr;
  execute(old, *e, cm2, m, b, desc, s);
  set_identity(*e, s);
  return e;
}

// ---------------------------------------------------------------------------
void PsiLayout::build(const Bond& bl, const Bond& br) {
  const size_t nr = br.size();
  rows_of.assign(nr, 0);
  off.assign(nr, 0);
  row_of.assign(nr, {});
  rows_pad.assign(nr, 0);
  off_pad.assign(nr, 0);
  offT.assign(nr, 0);
  ld.assign(nr, 0);
  row_pad_of.assign(nr, {});
  size = size_pad = sizeT = 0;
  for (size_t r = 0; r < nr; ++r) {
    for (size_t l = 0; l < bl.size(); ++l)
      for (int n1 = 0; n1 < 4; ++n1)
        for (int n2 = 0; n2 < 4; ++n2)
          if (bl.q[l] + kSiteQN[n1] + kSiteQN[n2] == br.q[r]) {
            row_of[r][{(int)l, 4 * n1 + n2}] = rows_of[r];
            row_pad_of[r][{(int)l, 4 * n1 + n2}] = rows_pad[r];
            rows_of[r] += bl.d[l];
            rows_pad[r] += pad8(bl.d[l]);
          }
    ld[r] = pad8(br.d[r]);
    off[r] = size;
    size += rows_of[r] * br.d[r];
    off_pad[r] = size_pad;
    size_pad += rows_pad[r] * ld[r];
    offT[r] = sizeT;
    sizeT += (int64_t)br.d[r] * rows_pad[r];
  }
}

// Problem indices of a stage ordered by locality key (stable).
static std::vector<size_t> by_key(const AStage& A) {
  std::vector<size_t> idx(A.probs.size());
  for (size_t q = 0; q < idx.size(); ++q) idx[q] = q;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](size_t x, size_t y) { return A.probs[x].key < A.probs[y].key; });
  return idx;
}

// FP64 descriptors of one stage (XCD-aware tile order).  Buffer `swap`
// (if >= 0) is addressed at swap_ptr instead of its own storage.
// Output tile (rows, cols) of the FP64 sigma stages (stage 1, stage 2),
// measured at CAS(54,36) D=4096 (ms per sigma, stage 1 / stage 2):
// 128 x 128 for stage 1 (309 against 355 with 64 x 64); 128 x 64 with eight
// waves for stage 2 (565, against 599 with 64 x 64, 586 with 64 x 128 and
// 611 with 128 x 128, whose padding of narrow output blocks costs more than
// its operand reuse gains).  DMRG_F64_TILE="t1,t2" overrides, each of 64,
// 128 (square), 128x64 or 64x128.
static std::pair<int, int> f64_sigma_tile(int stage) {
  std::pair<int, int> t[2] = {{128, 128}, {128, 64}};
  if (const char* e = std::getenv("DMRG_F64_TILE")) {
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
                 kErrInvalidArg, "DMRG_F64_TILE must be \"t1,t2\", each 64, 128, 128x64 or 64x128");
  }
  return t[stage - 1];
}

static void materialize_f64(const std::vector<PlanBuf>& bufs, const AStage& A, DevGemm& out,
                            int swap = -1, double* swap_ptr = nullptr,
                            std::pair<int, int> tile = {kTileM, kTileN}) {
  auto base = [&](int k) { return k == swap ? swap_ptr : bufs[k].f64; };
  GemmBatch b;
  b.tile = tile.first;
  b.tile_n = tile.second;
  b.segs.reserve(A.segs.size());
  for (auto& g : A.segs)
    b.segs.push_back({base(g.a.buf) + g.a.off, base(g.b.buf) + g.b.off, g.lda, g.ldb, g.k, g.flags, g.alpha});
  std::vector<int> keys;
  for (size_t q : by_key(A)) {
    const AProb& pb = A.probs[q];
    b.add_problem(base(pb.c.buf) + pb.c.off, pb.ldc, pb.m, pb.n, (size_t)pb.s0, (size_t)pb.s1, pb.beta);
    keys.resize(b.tiles.size(), pb.key);
  }
  xcd_order(b.tiles, keys, [&](const GemmTile& t) {
    double c = 0;
    for (int k = t.seg_begin; k < t.seg_end; ++k) c += b.segs[k].k + 32;
    return c;
  });
  upload_gemm(b, out);
}

std::unique_ptr<SigmaPlan> plan_sigma(const Problem& P, const Mps& m, const Env& L, const Env& R,
                                      int64_t ws_budget, hipStream_t s, bool record) {
  const int i = L.bond;
  DMRG_REQUIRE(L.side > 0 && R.side < 0 && R.bond == i + 2, kErrState, "plan_sigma: blocks do not bracket a window");
  auto plan = std::make_unique<SigmaPlan>();
  plan->window = i;
  plan->record = record;
  const Bond& bl = m.bonds[i];
  const Bond& br = m.bonds[i + 2];
  plan->psi.build(bl, br);
  const int ML = 2 * i, MS = 2 * i + 4;
  auto region = [&](int p) { return p < ML ? 0 : (p < MS ? 1 : 2); };
  const OpRef* LI = L.get({kIdent, 0});

  // ---- pairs -------------------------------------------------------------
  struct PKey {
    int lsrc;      // 0 stored L op, 1 partial sum
    int lcls, lidx;
    int z;         // R op index or -1
    bool operator<(const PKey& o) const {
      return std::tie(lsrc, lcls, lidx, z) < std::tie(o.lsrc, o.lcls, o.lidx, o.z);
    }
  };
  std::map<OpKey, int, bool (*)(const OpKey&, const OpKey&)> zindex(
      [](const OpKey& a, const OpKey& b) { return std::tie(a.kind, a.s) < std::tie(b.kind, b.s); });
  std::vector<OpRef> zrefs;
  auto zid = [&](OpKey k) -> int {
    const OpRef* r = R.get(k);
    if (!r) return -2;
    auto it = zindex.find(k);
    if (it != zindex.end()) return it->second;
    int id = (int)zrefs.size();
    zrefs.push_back(*r);
    zindex[k] = id;
    return id;
  };
  struct PVal {
    Mat16 y;
    int ypar;
    bool any;
  };
  std::map<PKey, PVal> pmap;
  auto add_pair = [&](int lsrc, OpRef lref, int z, const Str& y, double c) {
    if (z == -2 || c == 0.0) return;
    Mat16 Y = two_site_matrix(y, i);
    PKey k{lsrc, lref.cls, lref.idx, z};
    auto it = pmap.find(k);
    if (it == pmap.end()) {
      PVal v;
      v.y = Mat16::zero();
      v.ypar = y.parity();
      v.any = true;
      it = pmap.emplace(k, v).first;
    }
    DMRG_REQUIRE(it->second.ypar == y.parity(), kErrState, "plan_sigma: parity mix");
    for (int a = 0; a < 16; ++a)
      for (int b = 0; b < 16; ++b) it->second.y.m[a][b] += c * Y.m[a][b];
  };
  // partial sums W(y, xR) = sum_xL c xL
  std::map<std::pair<uint64_t, uint64_t>, std::map<std::pair<int, int>, double>> psum;
  std::map<std::pair<uint64_t, uint64_t>, QN> psum_dq;
  for_each_term(
      P, [](const int*, int) { return true; },
      [&](double c, const Str& term, int64_t ent, double fac) {
        Str parts[3];
        int sg = split_regions(term, region, 3, parts);
        if (sg == 0) return;
        const Str &xl = parts[0], &y = parts[1], &xr = parts[2];
        if (xr.n > 0 && xl.n + y.n <= 2) return;       // right complementary pass-through
        if (xl.n == 3) return;                          // left T pass-through
        if (xl.n > 0 && y.n == 0 && xr.n == 0) return;  // left H
        const OpRef* src = xl.n ? L.get({kNormal, xl.key()}) : LI;
        DMRG_REQUIRE(src, kErrState, "plan_sigma: missing left operator");
        auto key = std::make_pair(y.key(), xr.key());
        psum[key][{src->cls, src->idx}] += c * sg;
        psum_dq[key] = -(y.qn() + xr.qn());
        if (plan->record) plan->psum_prov[key][{src->cls, src->idx}].push_back({ent, fac * sg});
      });
  Str none;
  // stored pass-through pairs
  if (const OpRef* h = L.get({kHam, 0})) add_pair(0, *h, -1, none, 1.0);
  if (LI) add_pair(0, *LI, zid({kHam, 0}), none, 1.0);
  std::vector<int> sso = {2 * i, 2 * i + 1, 2 * i + 2, 2 * i + 3};
  std::vector<Str> ys1, ys2, lstr1, lstr2;
  strings_over(sso, 1, ys1);
  strings_over(sso, 2, ys2);
  for (const Str& y : ys1)
    if (const OpRef* t = L.get({kComp, y.key()})) add_pair(0, *t, -1, y, 1.0);
  for (int p = MS; p < 2 * P.K; ++p)
    for (int dag = 0; dag < 2; ++dag) {
      Str xr;
      xr.push(p, dag);
      if (const OpRef* t = L.get({kComp, xr.key()})) add_pair(0, *t, zid({kNormal, xr.key()}), none, 1.0);
    }
  std::vector<int> lso(ML);
  for (int p = 0; p < ML; ++p) lso[p] = p;
  strings_over(lso, 1, lstr1);
  strings_over(lso, 2, lstr2);
  auto rpass = [&](const Str& xl, const Str& y) {
    Str w;
    int eps = concat_canonical(xl, y, w);
    if (eps == 0 || w.n == 0) return;
    const OpRef* lr = xl.n ? L.get({kNormal, xl.key()}) : LI;
    if (!lr) return;
    add_pair(0, *lr, zid({kComp, w.key()}), y, (double)eps);
  };
  for (const Str& xl : lstr2) rpass(xl, none);
  for (const Str& xl : lstr1) {
    rpass(xl, none);
    for (const Str& y : ys1) rpass(xl, y);
  }
  for (const Str& y : ys1) rpass(none, y);
  for (const Str& y : ys2) rpass(none, y);
  // partial sums
  plan->psums = std::make_unique<Env>();
  Env& W = *plan->psums;
  W.side = +1;
  W.bond = i;
  W.basis = bl;
  std::vector<std::pair<std::pair<uint64_t, uint64_t>, OpRef>> wlist;
  uint64_t wid = 0;
  for (auto& kv : psum) {
    OpRef r = W.add({kPsum, wid++}, psum_dq[kv.first]);
    wlist.push_back({kv.first, r});
  }
  plan->wkeys = wlist;
  W.allocate(s);
  {
    // per W class: Coef (nW x nops of the source class) * source class
    std::map<int, std::vector<std::pair<const std::map<std::pair<int, int>, double>*, int>>> by_cls;
    for (size_t k = 0; k < wlist.size(); ++k) by_cls[wlist[k].second.cls].push_back({&psum[wlist[k].first], wlist[k].second.idx});
    DevBuf desc, coef;
    for (auto& kv : by_cls) {
      OpClass& Wc = *W.classes[kv.first];
      // all sources of a W class share one L class (same dq)
      int scls = -1;
      for (auto& e : kv.second)
        for (auto& t : *e.first) {
          DMRG_REQUIRE(scls < 0 || scls == t.first.first, kErrState, "plan_sigma: mixed source classes");
          scls = t.first.first;
        }
      if (scls < 0) continue;
      plan->w_src_cls[kv.first] = scls;
      const OpClass& Sc = *L.classes[scls];
      DMRG_REQUIRE(Sc.L.nnz == Wc.L.nnz, kErrState, "plan_sigma: layout mismatch");
      std::vector<double> C((size_t)Wc.nops * Sc.nops, 0.0);
      for (auto& e : kv.second)
        for (auto& t : *e.first) C[(size_t)e.second * Sc.nops + t.first.second] += t.second;
      coef.alloc(C.size() * sizeof(double));
      DMRG_HIP(hipStreamSynchronize(s));
      DMRG_HIP(hipMemcpy(coef.p, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice));
      GemmBatch b;
      b.segs.push_back({coef.p, Sc.data.p, Sc.nops, (int)Sc.L.nnz, Sc.nops, 0, 1.0});
      b.add_problem(Wc.data.p, (int)Wc.L.nnz, Wc.nops, (int)Wc.L.nnz, 0, 1, 0);
      launch_gemm_f64(b, s);
    }
    DMRG_HIP(hipStreamSynchronize(s));
  }
  for (auto& w : wlist) {
    const Str y = Str::from_key(w.first.first), xr = Str::from_key(w.first.second);
    int z = xr.n ? zid({kNormal, xr.key()}) : -1;
    add_pair(1, w.second, z, y, 1.0);
  }
  // ---- finalise pairs ------------------------------------------------------
  const OpRef* hL = L.get({kHam, 0});
  int zH = -1;
  {
    auto it = zindex.find(OpKey{kHam, 0});
    if (it != zindex.end()) zH = it->second;
  }
  plan->zrefs = zrefs;
  for (auto& r : zrefs) {
    const OpClass& c = *R.classes[r.cls];
    plan->zops.push_back({c.op(r.idx), &c.L});
    plan->zpar.push_back(c.L.dq.n & 1);
  }
  for (auto& kv : pmap) {
    const PKey& k = kv.first;
    const Env& src = k.lsrc ? W : L;
    const OpClass& c = *src.classes[k.lcls];
    bool nz = false;
    for (int a = 0; a < 16 && !nz; ++a)
      for (int b = 0; b < 16; ++b)
        if (kv.second.y.m[a][b] != 0) { nz = true; break; }
    if (!nz) continue;
    SigmaPair sp{{c.op(k.lidx), &c.L}, k.z, kv.second.y, kv.second.ypar};
    sp.pinned = (k.lsrc == 0 && hL && k.lcls == hL->cls && k.lidx == hL->idx) ||
                (k.z >= 0 && k.z == zH);
    sp.lsrc = k.lsrc;
    sp.lref = OpRef{k.lcls, k.lidx};
    plan->pairs.push_back(sp);
  }

  // ---- execution schedule ----------------------------------------------------
  // Every product is "NT": A row-major with k contiguous, B stored (n x k).
  //   stage 1: T_{z,r}^T (d_r' x rows_pad_r) = Z(r', r) * Psi_r^T
  //   stage 2: sigma_pad rows (l', n') of r' += L(l', l) * [T_{z,r}^T or Psi_r^T]
  //            columns of the row group (l, n)
  const PsiLayout& ps = plan->psi;
  std::map<const double*, int> buf_of_class;
  auto reg_env = [&](const Env& e) {
    for (auto& c : e.classes) {
      PlanBuf b;
      b.f64 = c->data.as<double>();
      b.n = (int64_t)c->nops * c->L.nnz;
      b.is_operator = true;
      buf_of_class[b.f64] = (int)plan->bufs.size();
      plan->bufs.push_back(std::move(b));
    }
  };
  reg_env(L);
  reg_env(W);
  reg_env(R);
  auto own = [&](int64_t n) {
    PlanBuf b;
    b.n = n;
    b.own.alloc((size_t)std::max<int64_t>(1, n) * sizeof(double));
    b.f64 = b.own.as<double>();
    launch_fill(b.f64, 0.0, n, s);
    plan->bufs.push_back(std::move(b));
    return (int)plan->bufs.size() - 1;
  };
  plan->buf_psi = own(ps.size_pad);
  plan->buf_sig = own(ps.size_pad);
  plan->buf_psit = own(ps.sizeT);
  auto ref_of = [&](const double* p) -> BufRef {
    auto it = buf_of_class.upper_bound(p);
    DMRG_REQUIRE(it != buf_of_class.begin(), kErrState, "plan_sigma: pointer outside operators");
    --it;
    return BufRef{it->second, (int64_t)(p - it->first)};
  };
  // pack / unpack / transpose tasks (API layout <-> padded)
  {
    std::vector<CopyTask> pk, up, tr;
    double* P = plan->bufs[plan->buf_psi].f64;
    double* S = plan->bufs[plan->buf_sig].f64;
    double* T = plan->bufs[plan->buf_psit].f64;
    for (size_t r = 0; r < br.size(); ++r) {
      for (auto& kv : ps.row_of[r]) {
        const int l = kv.first.first;
        const int64_t rp = ps.row_pad_of[r].at(kv.first);
        // API addresses are filled in at run time (offsets from the API base)
        pk.push_back({reinterpret_cast<const double*>((ps.off[r] + kv.second * br.d[r]) * sizeof(double)),
                      P + ps.off_pad[r] + rp * ps.ld[r], bl.d[l], br.d[r], br.d[r], ps.ld[r]});
        up.push_back({S + ps.off_pad[r] + rp * ps.ld[r],
                      reinterpret_cast<double*>((ps.off[r] + kv.second * br.d[r]) * sizeof(double)),
                      bl.d[l], br.d[r], ps.ld[r], br.d[r]});
      }
      if (ps.rows_pad[r] > 0)
        tr.push_back({P + ps.off_pad[r], T + ps.offT[r], (int)ps.rows_pad[r], br.d[r], ps.ld[r],
                      (int)ps.rows_pad[r]});
    }
    plan->n_pack = (int)pk.size();
    plan->n_trans = (int)tr.size();
    plan->pack_tasks.alloc(std::max<size_t>(1, pk.size()) * sizeof(CopyTask));
    plan->unpack_tasks.alloc(std::max<size_t>(1, up.size()) * sizeof(CopyTask));
    plan->trans_tasks.alloc(std::max<size_t>(1, tr.size()) * sizeof(CopyTask));
    plan->pack_host = pk;
    plan->unpack_host = up;
    DMRG_HIP(hipMemcpy(plan->trans_tasks.p, tr.data(), tr.size() * sizeof(CopyTask), hipMemcpyHostToDevice));
  }
  // stage-1 sizes per z
  const int nz = (int)plan->zops.size();
  std::vector<int64_t> zsize(nz, 0);
  for (int z = 0; z < nz; ++z)
    for (auto& blk : plan->zops[z].lay->blk)
      if (ps.rows_of[blk.c] > 0 && ps.rows_of[blk.r] > 0) zsize[z] += ps.rows_pad[blk.c] * br.d[blk.r];
  std::vector<std::pair<int, int>> chunks;
  {
    int z0 = 0;
    int64_t acc = 0;
    for (int z = 0; z < nz; ++z) {
      if (z > z0 && acc + zsize[z] > ws_budget) {
        chunks.push_back({z0, z});
        z0 = z;
        acc = 0;
      }
      acc += zsize[z];
      plan->ws_doubles = std::max(plan->ws_doubles, acc);
    }
    chunks.push_back({z0, nz});
  }
  plan->buf_ws = own(plan->ws_doubles);
  const int BP = plan->buf_psi, BS = plan->buf_sig, BW = plan->buf_ws, BT = plan->buf_psit;
  auto schedule = [&](bool pinned_set, const std::vector<std::pair<int, int>>& chunk_list,
                      std::vector<AStage>& out1, std::vector<AStage>& out2) {
    std::map<int, std::vector<int>> pairs_of_z;
    for (size_t k = 0; k < plan->pairs.size(); ++k)
      if (plan->pairs[k].pinned == pinned_set) pairs_of_z[plan->pairs[k].z].push_back((int)k);
    std::set<int> zused;
    for (auto& pz : pairs_of_z) zused.insert(pz.first);
    for (size_t ci = 0; ci < chunk_list.size(); ++ci) {
      const int z0 = chunk_list[ci].first, z1 = chunk_list[ci].second;
      AStage st1, st2;
      auto zin = [&](int z) { return z == -1 ? ci == 0 : (z >= z0 && z < z1); };
      // The row groups (l, n) of each Psi_r that stage 2 reads through right
      // operator z: stage 1 computes only those rows of T_{z,r}.
      std::map<std::pair<int, int>, std::map<int64_t, int>> reads;  // (z, r) -> padded row -> d_l
      for (auto& pz : pairs_of_z) {
        if (pz.first < 0 || !zin(pz.first)) continue;
        const Layout& Zl = *plan->zops[pz.first].lay;
        for (int k : pz.second) {
          const SigmaPair& pr = plan->pairs[k];
          for (int np = 0; np < 16; ++np)
            for (int n = 0; n < 16; ++n) {
              if (pr.y.m[np][n] == 0) continue;
              const QN qn = kSiteQN[n >> 2] + kSiteQN[n & 3];
              const QN qnp = kSiteQN[np >> 2] + kSiteQN[np & 3];
              for (auto& lb : pr.L.lay->blk) {
                const int l = lb.c, lp = lb.r;
                const int r = br.find(bl.q[l] + qn), rp = br.find(bl.q[lp] + qnp);
                if (r < 0 || rp < 0) continue;
                auto kr = ps.row_pad_of[r].find({l, n});
                if (kr == ps.row_pad_of[r].end() || !ps.row_pad_of[rp].count({lp, np})) continue;
                const Layout::Blk* zb = Zl.col(r);
                if (!zb || zb->r != rp) continue;
                reads[{pz.first, r}][kr->second] = bl.d[l];
              }
            }
        }
      }
      std::map<std::pair<int, int>, int64_t> tloc;  // (z, r) -> ws offset of T^T (d_r' x rows_pad_r)
      int64_t off = 0;
      for (int z = z0; z < z1; ++z) {
        if (!zused.count(z)) continue;
        const OpView& Z = plan->zops[z];
        for (auto& blk : Z.lay->blk) {
          const int r = blk.c, rp = blk.r;
          if (ps.rows_of[r] == 0 || ps.rows_of[rp] == 0) continue;
          auto rd = reads.find({z, r});
          if (rd == reads.end()) continue;  // no pair reads T_{z,r}
          tloc[{z, r}] = off;
          const double alpha = (plan->zpar[z] && (br.q[r].n & 1)) ? -1.0 : 1.0;
          // column ranges of T^T (padded psi rows): the groups read, merged
          // across gaps of at most kGap rows
          constexpr int64_t kGap = 32;
          std::vector<std::pair<int64_t, int64_t>> ranges;
          for (auto& g : rd->second) {
            const int64_t a = g.first, b = g.first + pad8(g.second);
            if (!ranges.empty() && a - ranges.back().second <= kGap) ranges.back().second = std::max(ranges.back().second, b);
            else ranges.push_back({a, b});
          }
          for (auto& rg : ranges) {
            const int64_t s0 = (int64_t)st1.segs.size();
            st1.segs.push_back({ref_of(Z.data + blk.off), {BP, ps.off_pad[r] + rg.first * ps.ld[r]}, blk.ld,
                                ps.ld[r], br.d[r], kTransB, alpha});
            // key: the psi sector, so that Psi_r stays in one XCD's L2
            st1.probs.push_back({{BW, off + rg.first}, (int)ps.rows_pad[r], br.d[rp], (int)(rg.second - rg.first),
                                 s0, s0 + 1, 0, r});
          }
          // real (unpadded) psi rows multiplied
          int64_t rows = 0;
          for (auto& g : ps.row_pad_of[r])
            for (auto& rg : ranges)
              if (g.second >= rg.first && g.second < rg.second) rows += bl.d[g.first.first];
          st1.flops += 2.0 * rows * br.d[rp] * br.d[r];
          off += ps.rows_pad[r] * br.d[rp];
        }
      }
      std::unordered_set<uint64_t> used;  // (z, r, l, n) row groups of stage 1 read by stage 2
      std::map<std::tuple<int, int64_t>, std::vector<ASeg>> outs;
      std::map<std::tuple<int, int64_t>, int> out_m, out_l;
      for (auto& pz : pairs_of_z) {
        if (!zin(pz.first)) continue;
        for (int k : pz.second) {
          const SigmaPair& pr = plan->pairs[k];
          const Layout& Ll = *pr.L.lay;
          const BufRef lref = ref_of(pr.L.data);
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
                BufRef bref;
                if (pr.z < 0) {
                  if (r != rp) continue;
                  bref = {BT, ps.offT[r] + kr->second};
                } else {
                  auto it = tloc.find({pr.z, r});
                  if (it == tloc.end()) continue;
                  const Layout::Blk* zb = plan->zops[pr.z].lay->col(r);
                  if (!zb || zb->r != rp) continue;
                  bref = {BW, it->second + kr->second};
                }
                const double sg = ((pr.ypar & 1) && (bl.q[l].n & 1)) ? -1.0 : 1.0;
                {
                  // the term's cheaper association order on this psi block
                  const double a = lb.dr, b = lb.dc, cr = br.d[r], cp = br.d[rp];
                  plan->flops_terms += pr.z < 0 ? 2.0 * a * b * cr
                                                : std::min(2.0 * a * b * cr + 2.0 * a * cr * cp,
                                                           2.0 * b * cr * cp + 2.0 * a * b * cp);
                  if (pr.z >= 0)
                    used.insert(((uint64_t)pr.z << 28) | ((uint64_t)r << 16) | ((uint64_t)l << 4) | (uint64_t)n);
                }
                if (LI && pr.lsrc == 0 && pr.lref.cls == LI->cls && pr.lref.idx == LI->idx)
                  plan->flops_s2_ident += 2.0 * lb.dr * br.d[rp] * lb.dc;
                auto ok = std::make_tuple(rp, krp->second);
                outs[ok].push_back({{lref.buf, lref.off + lb.off}, bref, lb.ld, (int)ps.rows_pad[r], lb.dc,
                                    kTransB, yv * sg});
                out_m[ok] = lb.dr;
                out_l[ok] = lp;
              }
            }
        }
      }
      for (auto& o : outs) {
        const int rp = std::get<0>(o.first);
        const int64_t row = std::get<1>(o.first);
        const int64_t s0 = (int64_t)st2.segs.size();
        const int mrows = out_m[o.first];
        for (auto& sgm : o.second) {
          st2.segs.push_back(sgm);
          st2.flops += 2.0 * mrows * br.d[rp] * sgm.k;
        }
        // key: the left sector of the output rows
        st2.probs.push_back({{BS, ps.off_pad[rp] + row * ps.ld[rp]}, ps.ld[rp], mrows, br.d[rp], s0,
                             (int64_t)st2.segs.size(), 1, out_l[o.first]});
      }
      for (uint64_t u : used) {
        const int z = (int)(u >> 28), r = (int)((u >> 16) & 0xfff), l = (int)((u >> 4) & 0xfff);
        const Layout::Blk* zb = plan->zops[z].lay->col(r);
        if (zb) plan->flops_s1_used += 2.0 * bl.d[l] * br.d[zb->r] * br.d[r];
      }
      plan->flops += st1.flops + st2.flops;
      plan->flops_stage1 += st1.flops;
      plan->flops_stage2 += st2.flops;
      out1.push_back(std::move(st1));
      out2.push_back(std::move(st2));
    }
  };
  schedule(false, chunks, plan->s1, plan->s2);
  if (std::getenv("DMRG_VERBOSE") && std::atoi(std::getenv("DMRG_VERBOSE")) > 1) {
    // per chunk: FLOPs of both stages, output problems, and the longest
    // segment list of stage 2 (summed k)
    for (size_t c = 0; c < plan->s1.size(); ++c) {
      const AStage& a = plan->s2[c];
      int64_t kmax = 0, ksum = 0;
      for (auto& pb : a.probs) {
        int64_t k = 0;
        for (int64_t q = pb.s0; q < pb.s1; ++q) k += a.segs[q].k;
        kmax = std::max(kmax, k);
        ksum += k;
      }
      fprintf(stderr, "[dmrg] chunk %zu: stage 1 %.3e flop, %zu problems; stage 2 %.3e flop, %zu problems, "
              "summed k per problem max %lld mean %.0f\n", c, plan->s1[c].flops, plan->s1[c].probs.size(),
              a.flops, a.probs.size(), (long long)kmax, a.probs.empty() ? 0.0 : (double)ksum / a.probs.size());
    }
    fprintf(stderr, "[dmrg] stage-2 FLOPs with the left identity as operand: %.3e\n", plan->flops_s2_ident);
    // MFMA work a BF16 launch issues per stage against the algorithmic
    // FLOPs, for square tiles of side T: whole tiles, or only the 16 x 16
    // blocks holding valid outputs; each segment's k in slabs of 32
    for (int st = 0; st < 2; ++st)
      for (int T : {64, 128, 256}) {
        double alg = 0, whole = 0, blocks = 0, kexact = 0;
        for (const AStage& a : st ? plan->s2 : plan->s1)
          for (const AProb& pb : a.probs) {
            double k32 = 0, k = 0;
            for (int64_t q = pb.s0; q < pb.s1; ++q) {
              k32 += 32.0 * ((a.segs[q].k + 31) / 32);
              k += a.segs[q].k;
            }
            const double m16 = 16.0 * ((pb.m + 15) / 16), n16 = 16.0 * ((pb.n + 15) / 16);
            const double mt = (double)T * ((pb.m + T - 1) / T), nt = (double)T * ((pb.n + T - 1) / T);
            alg += 2.0 * pb.m * pb.n * k;
            whole += 2.0 * mt * nt * k32;
            blocks += 2.0 * m16 * n16 * k32;
            kexact += 2.0 * m16 * n16 * k;
          }
        fprintf(stderr, "[dmrg] stage %d, %d x %d tiles: issued/algorithmic MFMA work %.2f (whole tiles), %.2f "
                "(valid 16x16 blocks), %.2f (valid blocks, exact k)\n", st + 1, T, T, whole / alg, blocks / alg,
                kexact / alg);
      }
  }
  {
    std::vector<AStage> a1, a2;
    schedule(true, {{0, nz}}, a1, a2);
    plan->p1 = std::move(a1[0]);
    plan->p2 = std::move(a2[0]);
  }
  plan->f64_s1.resize(plan->s1.size());
  plan->f64_s2.resize(plan->s2.size());
  for (size_t c = 0; c < plan->s1.size(); ++c) {
    materialize_f64(plan->bufs, plan->s1[c], plan->f64_s1[c], -1, nullptr, f64_sigma_tile(1));
    materialize_f64(plan->bufs, plan->s2[c], plan->f64_s2[c], -1, nullptr, f64_sigma_tile(2));
  }
  materialize_f64(plan->bufs, plan->p1, plan->f64_p1);
  materialize_f64(plan->bufs, plan->p2, plan->f64_p2);
  DMRG_HIP(hipStreamSynchronize(s));
  return plan;
}

bool plan_fixed_workspace(SigmaPlan& plan, double* ws, int64_t ws_doubles) {
  plan.fx_ready = false;
  if (!ws || plan.ws_doubles > ws_doubles) return false;
  plan.fx_s1.resize(plan.s1.size());
  plan.fx_s2.resize(plan.s2.size());
  for (size_t c = 0; c < plan.s1.size(); ++c) {
    materialize_f64(plan.bufs, plan.s1[c], plan.fx_s1[c], plan.buf_ws, ws, f64_sigma_tile(1));
    materialize_f64(plan.bufs, plan.s2[c], plan.fx_s2[c], plan.buf_ws, ws, f64_sigma_tile(2));
  }
  materialize_f64(plan.bufs, plan.p1, plan.fx_p1, plan.buf_ws, ws);
  materialize_f64(plan.bufs, plan.p2, plan.fx_p2, plan.buf_ws, ws);
  plan.fx_ready = true;
  return true;
}


// Tile shape of one output problem in the mixed configuration: the shape
// with the least padded area per unit of its dense throughput (relative
// rates of the shapes measured on large GEMMs).
static int mixed_shape(int m, int n, bool fp64_out) {
  // BF16-output stages (stage 1): four shapes, relative dense throughput;
  // FP64-output stages (stage 2): the 256 x 256 tile (twice the operand reuse
  // per byte of 128 x 128, measured 1.1x faster over a whole stage) or the
  // three-stage 128 x 128 tile, whichever pads the problem less per unit of
  // throughput
  static const int cand1[4] = {kShape128x128, kShape128x64, kShape64x128, kShape64x64};
  static const double rate1[4] = {1.0, 0.72, 0.72, 0.62};
  static const int cand2[2] = {kShape256x256, kShape128x128s3};
  static const double rate2[2] = {1.5, 1.0};
  const int* cand = fp64_out ? cand2 : cand1;
  const double* rate = fp64_out ? rate2 : rate1;
  int best = cand[0];
  double bc = 1e300;
  for (int q = 0; q < (fp64_out ? 2 : 4); ++q) {
    const int BM = shape_rows(cand[q]), BN = shape_cols(cand[q]);
    const double c = (double)((m + BM - 1) / BM * BM) * ((n + BN - 1) / BN * BN) / rate[q];
    if (c < bc) { bc = c; best = cand[q]; }
  }
  return best;
}

// Parts of a problem edge of length m in the split configuration: whole
// 128-blocks on 128-wide tiles, and a remainder of at most 64 on a 64-wide
// tile (a longer remainder stays on a 128-wide tile).  Returns the count;
// part p covers [lo[p], hi[p]), wide[p] = 1 for 128-wide tiles.
static int split_parts(int m, int (&lo)[2], int (&hi)[2], int (&wide)[2]) {
  const int rem = m % 128;
  lo[0] = 0;
  hi[0] = m;
  wide[0] = m > 64;
  if (m <= 64 || rem == 0 || rem > 64) return 1;
  hi[0] = m - rem;
  lo[1] = m - rem;
  hi[1] = m;
  wide[1] = 0;
  return 2;
}

static int split_shape(int wide_rows, int wide_cols) {
  if (wide_rows) return wide_cols ? kShape128x128s3 : kShape128x64;
  return wide_cols ? kShape64x128 : kShape64x64;
}

// BF16 descriptors of one stage (all chunks) for one launch configuration:
// tile shape (one for every problem, kShapeMixed: per problem, or
// kShapeSplit: per part of a problem), locality
// grouping of the tiles (0: each problem its own group, 1: the problems of
// one key together) and segment order (1: each problem's segments sorted by
// their A operand).  out[chunk] holds one launch per tile shape used.
static void build_bf_stage(SigmaPlan& plan, int stage, const BfChoice& ch,
                           std::vector<std::vector<DevGemmB>>& out) {
  auto bfp = [&](const BufRef& r) { return plan.bufs[r.buf].bf.as<uint16_t>() + r.off; };
  const std::vector<AStage>& st = stage == 1 ? plan.s1 : plan.s2;
  out.clear();
  out.resize(st.size());
  for (size_t ci = 0; ci < st.size(); ++ci) {
    const AStage& A = st[ci];
    // stage 1 writes BF16 hi/lo, which the eight-wave 256 x 256 tile does not
    const int uni = (stage == 1 && ch.shape == kShape256x256) ? kShape128x128s3 : ch.shape;
    std::vector<int> pshape(A.probs.size(), uni);
    if (ch.shape == kShapeMixed)
      for (size_t q = 0; q < A.probs.size(); ++q) pshape[q] = mixed_shape(A.probs[q].m, A.probs[q].n, stage == 2);
    std::vector<size_t> order(A.probs.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = q;
    if (ch.order == 1) order = by_key(A);
    for (int sh = 0; sh < kNumShapes; ++sh) {
      GemmBatchB b;
      b.shape = sh;
      std::vector<int> keys;
      std::vector<int64_t> perm;
      for (size_t q : order) {
        const AProb& pb = A.probs[q];
        // regions of this problem tiled by this launch: rows [r0, r1) x columns [c0, c1)
        int reg[4][4], nreg = 0;
        if (ch.shape == kShapeSplit) {
          int rl[2], rh[2], rw[2], cl[2], chh[2], cw[2];
          const int nr = split_parts(pb.m, rl, rh, rw), nc = split_parts(pb.n, cl, chh, cw);
          for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j)
              if (split_shape(rw[i], cw[j]) == sh) {
                reg[nreg][0] = rl[i];
                reg[nreg][1] = rh[i];
                reg[nreg][2] = cl[j];
                reg[nreg][3] = chh[j];
                ++nreg;
              }
        } else if (pshape[q] == sh) {
          reg[0][0] = 0;
          reg[0][1] = pb.m;
          reg[0][2] = 0;
          reg[0][3] = pb.n;
          nreg = 1;
        }
        if (nreg == 0) continue;
        const size_t s0 = b.segs.size();
        perm.clear();
        for (int64_t k = pb.s0; k < pb.s1; ++k) perm.push_back(k);
        if (ch.sort_a)
          std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) {
            return std::tie(A.segs[x].a.buf, A.segs[x].a.off) < std::tie(A.segs[y].a.buf, A.segs[y].a.off);
          });
        for (int64_t k : perm) {
          const ASeg& g = A.segs[k];
          DMRG_REQUIRE(g.flags == kTransB && g.lda % 8 == 0 && g.ldb % 8 == 0 && g.a.off % 8 == 0 &&
                           g.b.off % 8 == 0,
                       kErrState, "prepare_bf16: segment is not an aligned NT product");
          b.segs.push_back({bfp(g.a), bfp(g.b), plan.bufs[g.a.buf].n, plan.bufs[g.b.buf].n, g.lda,
                            g.ldb, g.k, g.flags, g.alpha});
        }
        for (int r = 0; r < nreg; ++r) {
          if (stage == 1)
            b.add_region(bfp(pb.c), plan.bufs[pb.c.buf].n, pb.ldc, reg[r][0], reg[r][1], reg[r][2],
                         reg[r][3], s0, b.segs.size(), 0);
          else
            b.add_region(plan.bufs[pb.c.buf].f64 + pb.c.off, 0, pb.ldc, reg[r][0], reg[r][1], reg[r][2],
                         reg[r][3], s0, b.segs.size(), pb.beta);
        }
        keys.resize(b.tiles.size(), ch.order == 1 ? pb.key : (int)q);
      }
      if (b.tiles.empty()) continue;
      auto tcost = [&](const GemmTileB& t) {
        double c = 0;
        for (int k = t.seg_begin; k < t.seg_end; ++k) c += b.segs[k].k + 32;
        return c;
      };
      if (std::getenv("DMRG_VERBOSE") && std::atoi(std::getenv("DMRG_VERBOSE")) > 1) {
        double tot = 0, mx = 0;
        for (auto& t : b.tiles) {
          const double c = tcost(t);
          tot += c;
          mx = std::max(mx, c);
        }
        fprintf(stderr, "[dmrg] stage %d chunk %zu shape %d: %zu tiles, %zu segments, max tile %.3g of total %.3g\n",
                stage, ci, sh, b.tiles.size(), b.segs.size(), mx, tot);
      }
      xcd_order(b.tiles, keys, tcost);
      out[ci].emplace_back();
      upload_gemm_bf16(b, out[ci].back());
    }
  }
}

int ozaki_kappa() {
  int k = 6;
  if (const char* e = std::getenv("DMRG_OZAKI_SLICES")) k = std::atoi(e);
  DMRG_REQUIRE(k >= kOzMinKappa && k <= kOzMaxKappa, kErrInvalidArg,
               "DMRG_OZAKI_SLICES must lie in [3, 7]");
  return k;
}

void prepare_ozaki(SigmaPlan& plan, hipStream_t s) {
  const int kappa = ozaki_kappa();
  if (plan.oz.kappa == kappa) return;
  DMRG_HIP(hipStreamSynchronize(s));
  plan.oz = OzPlan();
  OzPlan& oz = plan.oz;
  // distinct operands: (buffer, offset, ld, k, chunk of a workspace operand)
  struct Opnd {
    int cls;  // 0 static, 1 psi, 2 workspace
    int chunk;
    const double* src;
    int ld, k, rows;
    int64_t dst = 0, exp = 0;
  };
  std::vector<Opnd> ops;
  std::map<std::tuple<int, int64_t, int, int, int>, int> index;
  auto cls_of = [&](int buf) {
    if (buf == plan.buf_psi || buf == plan.buf_psit) return 1;
    if (buf == plan.buf_ws) return 2;
    return 0;
  };
  auto operand = [&](const BufRef& r, int ld, int k, int rows, int chunk) {
    const int cls = cls_of(r.buf);
    const int ch = cls == 2 ? chunk : -1;
    auto key = std::make_tuple(r.buf, r.off, ld, k, ch);
    auto it = index.find(key);
    if (it == index.end()) {
      it = index.emplace(key, (int)ops.size()).first;
      ops.push_back({cls, ch, plan.bufs[r.buf].f64 + r.off, ld, k, 0});
    }
    ops[it->second].rows = std::max(ops[it->second].rows, rows);
    return it->second;
  };
  const size_t nch = plan.s1.size();
  // per stage and chunk: the operands of each segment
  std::vector<std::vector<std::pair<int, int>>> segops[2];
  for (int st = 0; st < 2; ++st) {
    const std::vector<AStage>& S = st == 0 ? plan.s1 : plan.s2;
    segops[st].resize(nch);
    for (size_t c = 0; c < nch; ++c) {
      const AStage& A = S[c];
      segops[st][c].assign(A.segs.size(), {-1, -1});
      for (const AProb& pb : A.probs)
        for (int64_t q = pb.s0; q < pb.s1; ++q) {
          const ASeg& g = A.segs[(size_t)q];
          DMRG_REQUIRE(g.flags == kTransB, kErrState, "prepare_ozaki: segment is not an NT product");
          segops[st][c][(size_t)q] = {operand(g.a, g.lda, g.k, pb.m, (int)c), operand(g.b, g.ldb, g.k, pb.n, (int)c)};
        }
    }
  }
  // layout: static operands, psi operands, then one workspace region reused
  // by every chunk
  int64_t bytes = 0, rows = 0;
  auto place = [&](Opnd& o) {
    o.dst = bytes;
    o.exp = rows;
    bytes += (int64_t)kappa * o.rows * oz_kp(o.k);
    rows += o.rows;
  };
  for (Opnd& o : ops)
    if (o.cls == 0) place(o);
  oz.rows_static = rows;
  const int64_t psi_row0 = rows;
  for (Opnd& o : ops)
    if (o.cls == 1) place(o);
  oz.rows_psi = rows - psi_row0;
  const int64_t ws_bytes0 = bytes, ws_rows0 = rows;
  int64_t ws_bytes_max = 0, ws_rows_max = 0;
  oz.rows_ws.assign(nch, 0);
  for (size_t c = 0; c < nch; ++c) {
    bytes = ws_bytes0;
    rows = ws_rows0;
    for (Opnd& o : ops)
      if (o.cls == 2 && o.chunk == (int)c) place(o);
    ws_bytes_max = std::max(ws_bytes_max, bytes - ws_bytes0);
    ws_rows_max = std::max(ws_rows_max, rows - ws_rows0);
    oz.rows_ws[c] = rows - ws_rows0;
  }
  oz.arena_bytes = ws_bytes0 + ws_bytes_max;
  oz.arena.alloc((size_t)std::max<int64_t>(oz.arena_bytes, 256));
  oz.exps.alloc((size_t)std::max<int64_t>(ws_rows0 + ws_rows_max, 1) * sizeof(int32_t));
  int8_t* arena = oz.arena.as<int8_t>();
  int32_t* exps = oz.exps.as<int32_t>();
  // slicing passes
  auto slice_list = [&](int cls, int chunk, DevBuf& out, int& n) {
    std::vector<SliceOp> v;
    int64_t r0 = 0;
    for (const Opnd& o : ops) {
      if (o.cls != cls || (cls == 2 && o.chunk != chunk)) continue;
      SliceOp so{};
      so.src = o.src;
      so.dst = o.dst;
      so.plane = (int64_t)o.rows * oz_kp(o.k);
      so.exp = o.exp;
      so.row0 = r0;
      so.ld = o.ld;
      so.rows = o.rows;
      so.k = o.k;
      so.kp = oz_kp(o.k);
      so.colmajor = 0;
      r0 += o.rows;
      v.push_back(so);
    }
    n = (int)v.size();
    out.alloc(std::max<size_t>(1, v.size()) * sizeof(SliceOp));
    if (!v.empty()) DMRG_HIP(hipMemcpy(out.p, v.data(), v.size() * sizeof(SliceOp), hipMemcpyHostToDevice));
  };
  slice_list(0, -1, oz.ops_static, oz.n_static);
  slice_list(1, -1, oz.ops_psi, oz.n_psi);
  oz.ops_ws.resize(nch);
  oz.n_ws.assign(nch, 0);
  for (size_t c = 0; c < nch; ++c) slice_list(2, (int)c, oz.ops_ws[c], oz.n_ws[c]);
  // task lists
  oz.s1.resize(nch);
  oz.s2.resize(nch);
  for (int st = 0; st < 2; ++st)
    for (size_t c = 0; c < nch; ++c) {
      const AStage& A = (st == 0 ? plan.s1 : plan.s2)[c];
      GemmBatchO b;
      std::vector<int> keys;
      for (size_t q : by_key(A)) {
        const AProb& pb = A.probs[q];
        const size_t s0 = b.segs.size();
        for (int64_t k = pb.s0; k < pb.s1; ++k) {
          const ASeg& g = A.segs[(size_t)k];
          const Opnd& oa = ops[(size_t)segops[st][c][(size_t)k].first];
          const Opnd& ob = ops[(size_t)segops[st][c][(size_t)k].second];
          GemmSegO so{};
          so.a = arena + oa.dst;
          so.b = arena + ob.dst;
          so.ea = exps + oa.exp;
          so.eb = exps + ob.exp;
          so.a_plane = (int64_t)oa.rows * oz_kp(oa.k);
          so.b_plane = (int64_t)ob.rows * oz_kp(ob.k);
          so.lda = oz_kp(oa.k);
          so.ldb = oz_kp(ob.k);
          so.k = g.k;
          so.alpha = g.alpha;
          b.segs.push_back(so);
        }
        b.add_problem(plan.bufs[pb.c.buf].f64 + pb.c.off, pb.ldc, pb.m, pb.n, s0, b.segs.size(), pb.beta);
        keys.resize(b.tiles.size(), pb.key);
      }
      xcd_order(b.tiles, keys, [&](const GemmTileB& t) {
        double cst = 0;
        for (int k = t.seg_begin; k < t.seg_end; ++k) cst += b.segs[k].k + 64;
        return cst;
      });
      upload_gemm_oz(b, kappa, st == 0 ? oz.s1[c] : oz.s2[c]);
    }
  oz.kappa = kappa;
  if (std::getenv("DMRG_VERBOSE"))
    fprintf(stderr, "[dmrg] Ozaki plan: %d slices, %zu operands, %.2f GB of digit planes\n", kappa, ops.size(),
            oz.arena_bytes / 1e9);
}

static void launch_bf_chunk(const std::vector<DevGemmB>& d, int stage, bool x3, hipStream_t s) {
  for (const DevGemmB& g : d) launch_gemm_bf16(g, x3, stage == 1 ? kOutBf16 : kOutF64, stage, s);
}
static void launch_bf_stage(const std::vector<std::vector<DevGemmB>>& d, int stage, bool x3, hipStream_t s) {
  for (const auto& c : d) launch_bf_chunk(c, stage, x3, s);
}

// Event time (ms) of one stage over all chunks, best of reps after a warm-up.
// The launches write the stage's real outputs (workspace, sigma buffer), which
// every sigma overwrites or clears first.
static double time_bf_stage(const std::vector<std::vector<DevGemmB>>& d, int stage, bool x3, hipStream_t s,
                            int reps) {
  hipEvent_t a, b;
  DMRG_HIP(hipEventCreate(&a));
  DMRG_HIP(hipEventCreate(&b));
  double best = 1e300;
  launch_bf_stage(d, stage, x3, s);
  for (int r = 0; r < reps; ++r) {
    DMRG_HIP(hipEventRecord(a, s));
    launch_bf_stage(d, stage, x3, s);
    DMRG_HIP(hipEventRecord(b, s));
    DMRG_HIP(hipEventSynchronize(b));
    float ms = 0;
    DMRG_HIP(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

// Autotuner of the BF16 launch configuration: per stage, first the tile
// shape (with per-problem grouping, schedule order), then the grouping and
// segment order for that shape; every candidate is timed on this plan's own
// launches.  Small plans keep the default (their launches are too short to
// time reliably and the tuning would cost more than it saves).
static void autotune_bf16(SigmaPlan& plan, hipStream_t s) {
  const bool x3 = true;  // the mixed path's main precision
  const double t0 = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
  for (int stage = 1; stage <= 2; ++stage) {
    BfChoice best;
    double tbest = 1e300;
    std::vector<std::vector<DevGemmB>> d;
    auto trial = [&](const BfChoice& c) {
      build_bf_stage(plan, stage, c, d);
      const double t = time_bf_stage(d, stage, x3, s, 2);
      plan.tune_log.push_back({stage, c, t});
      if (t < tbest) { tbest = t; best = c; }
    };
    for (int sh = 0; sh <= kShapeSplit; ++sh)
      if (!(stage == 1 && sh == kShape256x256)) trial(BfChoice{sh, 0, 0});
    const int sh = best.shape;
    trial(BfChoice{sh, 1, 0});
    if (stage == 2) {
      trial(BfChoice{sh, 0, 1});
      trial(BfChoice{sh, 1, 1});
    }
    plan.bf_choice[stage - 1] = best;
  }
  plan.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count() - t0;
}

// BF16 hi/lo copies of every operator, the psi and workspace buffers, and the
// BF16 descriptors (built once per plan, on first use, after the autotuner).
void prepare_bf16(SigmaPlan& plan, hipStream_t s) {
  if (plan.bf_ready) return;
  for (size_t k = 0; k < plan.bufs.size(); ++k) {
    PlanBuf& b = plan.bufs[k];
    if ((int)k == plan.buf_sig) continue;
    b.bf.alloc((size_t)std::max<int64_t>(1, 2 * b.n) * sizeof(uint16_t));
    if (b.is_operator) launch_split_bf16(b.bf.as<uint16_t>(), b.f64, b.n, s);
    else launch_fill(reinterpret_cast<double*>(b.bf.p), 0.0, (int64_t)(b.bf.bytes / sizeof(double)), s);
  }
  // DMRG_BF16_SHAPE=0..7 fixes the tile shape of both stages (tests of each
  // kernel variant); otherwise DMRG_AUTOTUNE=0|1 switches the autotuner off or
  // on (default: on for plans above 5e10 FLOP per sigma).
  // DMRG_BF16_CONFIG="c1,c2" fixes the configuration of both stages (codes of
  // dmrg_sigma_info: shape + 16 * grouping + 256 * segment order), e.g. to
  // profile the configuration an earlier run chose.
  const char* fixed = std::getenv("DMRG_BF16_SHAPE");
  const char* env = std::getenv("DMRG_AUTOTUNE");
  const char* cfg = std::getenv("DMRG_BF16_CONFIG");
  if (cfg) {
    int c[2] = {-1, -1};
    DMRG_REQUIRE(std::sscanf(cfg, "%d,%d", &c[0], &c[1]) == 2, kErrInvalidArg,
                 "DMRG_BF16_CONFIG must be two codes \"c1,c2\"");
    for (int k = 0; k < 2; ++k) {
      BfChoice& b = plan.bf_choice[k];
      b.shape = c[k] & 15;
      b.order = (c[k] >> 4) & 15;
      b.sort_a = (c[k] >> 8) & 1;
      DMRG_REQUIRE(c[k] >= 0 && b.shape <= kShapeSplit && b.order <= 1, kErrInvalidArg,
                   "DMRG_BF16_CONFIG: unknown configuration code");
    }
  } else if (fixed) {
    const int sh = std::atoi(fixed);
    DMRG_REQUIRE(sh >= 0 && sh <= kShapeSplit, kErrInvalidArg, "DMRG_BF16_SHAPE must be 0 to 7");
    plan.bf_choice[0].shape = plan.bf_choice[1].shape = sh;
  } else if (env ? std::atoi(env) != 0 : plan.flops > 5e10) {
    autotune_bf16(plan, s);
    if (std::getenv("DMRG_VERBOSE"))
      for (auto& e : plan.tune_log)
        fprintf(stderr, "[dmrg] autotune stage %d shape %d order %d sort %d: %.2f ms\n", e.stage,
                e.choice.shape, e.choice.order, e.choice.sort_a, e.ms);
  }
  build_bf_stage(plan, 1, plan.bf_choice[0], plan.bf_s1);
  build_bf_stage(plan, 2, plan.bf_choice[1], plan.bf_s2);
  DMRG_HIP(hipStreamSynchronize(s));
  plan.bf_ready = true;
}

// The pack/unpack task lists hold API offsets; the run binds them to the
// caller's psi / sigma pointers (the lists are rebuilt only when the pointers
// change, so repeated calls on the same buffers do no host work).
static void bind_tasks(const std::vector<CopyTask>& host, DevBuf& dev, const double* api_src,
                       double* api_dst, bool src_is_api, const double*& bound) {
  const double* key = src_is_api ? api_src : api_dst;
  if (bound == key) return;
  std::vector<CopyTask> t = host;
  for (auto& x : t) {
    if (src_is_api) x.src = reinterpret_cast<const double*>(reinterpret_cast<const char*>(api_src) + reinterpret_cast<size_t>(x.src));
    else x.dst = reinterpret_cast<double*>(reinterpret_cast<char*>(api_dst) + reinterpret_cast<size_t>(x.dst));
  }
  DMRG_HIP(hipMemcpy(dev.p, t.data(), t.size() * sizeof(CopyTask), hipMemcpyHostToDevice));
  bound = key;
}

hipEvent_t SigmaTiming::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  DMRG_HIP(hipEventCreate(&e));
  return e;
}
void SigmaTiming::collect(hipStream_t s) {
  if (pending.empty()) return;
  DMRG_HIP(hipStreamSynchronize(s));
  for (auto& p : pending) {
    float t = 0;
    DMRG_HIP(hipEventElapsedTime(&t, p.second.first, p.second.second));
    ms[p.first] += t;
    launches[p.first] += 1;
    pool.push_back(p.second.first);
    pool.push_back(p.second.second);
  }
  pending.clear();
}
void SigmaTiming::reset() {
  for (int k = 0; k < 4; ++k) { ms[k] = 0; launches[k] = 0; }
  calls = 0;
}
SigmaTiming::~SigmaTiming() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

static void bind_psi(SigmaPlan& plan, const double* psi, hipStream_t s) {
  if (plan.bound_psi != psi) DMRG_HIP(hipStreamSynchronize(s));
  bind_tasks(plan.pack_host, plan.pack_tasks, psi, nullptr, true, plan.bound_psi);
}
static void enqueue_load_psi(SigmaPlan& plan, hipStream_t s) {
  launch_copy_tasks(plan.pack_tasks.as<CopyTask>(), plan.n_pack, false, s);
  launch_copy_tasks(plan.trans_tasks.as<CopyTask>(), plan.n_trans, true, s);
}

void plan_load_psi(SigmaPlan& plan, const double* psi, hipStream_t s) {
  bind_psi(plan, psi, s);
  enqueue_load_psi(plan, s);
}

// Device work of one sigma (no host synchronisation, so it can be captured).
static void enqueue_sigma(SigmaPlan& plan, int precision, hipStream_t s) {
  PlanBuf& P = plan.bufs[plan.buf_psi];
  PlanBuf& S = plan.bufs[plan.buf_sig];
  PlanBuf& T = plan.bufs[plan.buf_psit];
  enqueue_load_psi(plan, s);
  launch_fill(S.f64, 0.0, S.n, s);
  SigmaTiming& tm = plan.timing;
  // runs one launch, bracketed by events when timing is on
  auto timed = [&](int role, auto&& launch) {
    if (!tm.on) {
      launch();
      return;
    }
    hipEvent_t a = tm.get(), b = tm.get();
    DMRG_HIP(hipEventRecord(a, s));
    launch();
    DMRG_HIP(hipEventRecord(b, s));
    tm.record(role, a, b);
  };
  if (tm.on) ++tm.calls;
  // pairs pinned to FP64 first (they reuse the stage-1 workspace)
  timed(3, [&] { launch_gemm_f64(plan.f64_p1, s, 1); });
  timed(3, [&] { launch_gemm_f64(plan.f64_p2, s, 2); });
  if (precision == 0) {
    for (size_t c = 0; c < plan.f64_s1.size(); ++c) {
      timed(1, [&] { launch_gemm_f64(plan.f64_s1[c], s, 1); });
      timed(2, [&] { launch_gemm_f64(plan.f64_s2[c], s, 2); });
    }
  } else if (precision == 3) {
    OzPlan& oz = plan.oz;
    const int kappa = oz.kappa;
    if (!oz.statics_sliced) {
      launch_slice_oz(oz.ops_static.as<SliceOp>(), oz.n_static, oz.rows_static, oz.arena.as<int8_t>(),
                      oz.exps.as<int32_t>(), kappa, s);
      oz.statics_sliced = true;
    }
    timed(0, [&] {
      launch_slice_oz(oz.ops_psi.as<SliceOp>(), oz.n_psi, oz.rows_psi, oz.arena.as<int8_t>(),
                      oz.exps.as<int32_t>(), kappa, s);
    });
    for (size_t c = 0; c < oz.s1.size(); ++c) {
      timed(1, [&] { launch_gemm_oz(oz.s1[c], kappa, s); });
      timed(0, [&] {
        launch_slice_oz(oz.ops_ws[c].as<SliceOp>(), oz.n_ws[c], oz.rows_ws[c], oz.arena.as<int8_t>(),
                        oz.exps.as<int32_t>(), kappa, s);
      });
      timed(2, [&] { launch_gemm_oz(oz.s2[c], kappa, s); });
    }
  } else {
    launch_split_bf16(P.bf.as<uint16_t>(), P.f64, P.n, s);
    launch_split_bf16(T.bf.as<uint16_t>(), T.f64, T.n, s);
    const bool x3 = precision == 2;
    for (size_t c = 0; c < plan.bf_s1.size(); ++c) {
      timed(1, [&] { launch_bf_chunk(plan.bf_s1[c], 1, x3, s); });
      timed(2, [&] { launch_bf_chunk(plan.bf_s2[c], 2, x3, s); });
    }
  }
  launch_copy_tasks(plan.unpack_tasks.as<CopyTask>(), plan.n_pack, false, s);
}

SigmaGraphs::~SigmaGraphs() {
  for (auto& e : exec)
    if (e) (void)hipGraphExecDestroy(e);
  if (capture) (void)hipStreamDestroy(capture);
}

void run_sigma(SigmaPlan& plan, const double* psi, double* sigma, int precision, hipStream_t s) {
  // host-side preparation first: task lists bound to the caller's buffers,
  // BF16 copies, descriptors and the autotuner (whose trial launches write the
  // workspace and sigma buffers, both rewritten below)
  if (plan.bound_sigma != sigma) DMRG_HIP(hipStreamSynchronize(s));
  bind_tasks(plan.unpack_host, plan.unpack_tasks, nullptr, sigma, false, plan.bound_sigma);
  bind_psi(plan, psi, s);
  if (precision == 1 || precision == 2) prepare_bf16(plan, s);
  if (precision == 3) prepare_ozaki(plan, s);
  if (!plan.use_graphs || plan.timing.on || precision == 3) {
    enqueue_sigma(plan, precision, s);
    return;
  }
  // graph replay: the device work is captured once per precision (on a
  // stream of the plan's own: the caller's stream may be the null stream,
  // which cannot be captured) and launched on the caller's stream; the copy
  // kernels read their task lists from device memory, so the graph serves any
  // psi / sigma buffers
  hipGraphExec_t& ex = plan.graphs.exec[precision];
  if (!ex) {
    if (!plan.graphs.capture) DMRG_HIP(hipStreamCreateWithFlags(&plan.graphs.capture, hipStreamNonBlocking));
    hipStream_t cs = plan.graphs.capture;
    hipGraph_t g = nullptr;
    DMRG_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      enqueue_sigma(plan, precision, cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    DMRG_HIP(hipStreamEndCapture(cs, &g));
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    DMRG_HIP(e);
  }
  DMRG_HIP(hipGraphLaunch(ex, s));
}

void run_sigma_fixed_workspace(SigmaPlan& plan, const double* psi, double* sigma, hipStream_t s) {
  DMRG_REQUIRE(plan.fx_ready, kErrState, "sigma: no fixed-workspace schedule");
  if (plan.bound_sigma != sigma) DMRG_HIP(hipStreamSynchronize(s));
  bind_tasks(plan.unpack_host, plan.unpack_tasks, nullptr, sigma, false, plan.bound_sigma);
  bind_psi(plan, psi, s);
  enqueue_load_psi(plan, s);
  PlanBuf& S = plan.bufs[plan.buf_sig];
  launch_fill(S.f64, 0.0, S.n, s);
  launch_gemm_f64(plan.fx_p1, s, 1);
  launch_gemm_f64(plan.fx_p2, s, 2);
  for (size_t c = 0; c < plan.fx_s1.size(); ++c) {
    launch_gemm_f64(plan.fx_s1[c], s, 1);
    launch_gemm_f64(plan.fx_s2[c], s, 2);
  }
  launch_copy_tasks(plan.unpack_tasks.as<CopyTask>(), plan.n_pack, false, s);
}

}  // namespace dmrg
