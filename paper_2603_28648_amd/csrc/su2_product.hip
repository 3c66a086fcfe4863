// Renormalisation step of spin-adapted operators: the reduced blocks of a
// coupled product [A^k1 x B^k2]^k of operators on two subsystems (block and
// site), and their projection onto the kept multiplets of the enlarged
// block.  Every output block is the Kronecker product of one block of A and
// one block of B times the 9j-weighted coupling factor and the fermion sign
// (see dmrg_su2_product in include/dmrg.h); one workgroup writes each block.
#include "su2_product.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "gemm.h"
#include "su2.h"

namespace dmrg {

namespace {

bool triangle(int ta, int tb, int tc) { return tc >= std::abs(ta - tb) && tc <= ta + tb && (ta + tb + tc) % 2 == 0; }

// {j1 j2 j3; j4 j5 j6; j7 j8 j9} (doubled arguments) as the sum over x of
// (-1)^(2x) (2x + 1) {j1 j4 j7; j8 j9 x} {j2 j5 j8; j4 x j6} {j3 j6 j9; x j1 j2}
double wigner_9j(int j1, int j2, int j3, int j4, int j5, int j6, int j7, int j8, int j9) {
  const int lo = std::max(std::max(std::abs(j1 - j9), std::abs(j4 - j8)), std::abs(j2 - j6));
  const int hi = std::min(std::min(j1 + j9, j4 + j8), j2 + j6);
  double s = 0.0;
  for (int x = lo; x <= hi; x += 2)
    s += ((x & 1) ? -1.0 : 1.0) * (x + 1) * wigner_6j(j1, j4, j7, j8, j9, x) * wigner_6j(j2, j5, j8, j4, x, j6) *
         wigner_6j(j3, j6, j9, x, j1, j2);
  return s;
}

struct KronTask {
  const double* a;
  const double* b;
  double* out;
  int32_t ra, ca, rb, cb;
  double scale;
};

// out[(i rb + k), (j cb + l)] = scale a[i, j] b[k, l]
__global__ void k_kron_tasks(const KronTask* __restrict__ tasks) {
  const KronTask t = tasks[blockIdx.x];
  const int64_t cols = (int64_t)t.ca * t.cb, n = (int64_t)t.ra * t.rb * cols;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t r = e / cols, c = e % cols;
    const int i = (int)(r / t.rb), k = (int)(r % t.rb), j = (int)(c / t.cb), l = (int)(c % t.cb);
    t.out[e] = t.scale * t.a[(int64_t)i * t.ca + j] * t.b[(int64_t)k * t.cb + l];
  }
}

struct Side {
  std::vector<int> n, ts, d;
};

Side side(int k, const int32_t* n, const int32_t* ts, const int32_t* d) {
  DMRG_REQUIRE(k > 0 && n && ts && d, kErrInvalidArg, "su2_product: a subsystem needs sectors");
  Side s;
  for (int i = 0; i < k; ++i) {
    DMRG_REQUIRE(n[i] >= 0 && ts[i] >= 0 && (n[i] - ts[i]) % 2 == 0 && d[i] > 0, kErrInvalidArg,
                 "su2_product: a sector needs N, 2S >= 0 of equal parity and a positive dimension");
    s.n.push_back(n[i]);
    s.ts.push_back(ts[i]);
    s.d.push_back(d[i]);
  }
  return s;
}

}  // namespace

Su2Product su2_product_plan(const dmrg_su2_window& w, const dmrg_su2_operator& a, const dmrg_su2_operator& b,
                            int tk1, int tk2, int tk, int parity_b) {
  DMRG_REQUIRE(tk1 >= 0 && tk2 >= 0 && tk >= 0 && (parity_b == 0 || parity_b == 1), kErrInvalidArg,
               "su2_product: ranks must be >= 0 and the parity 0 or 1");
  const Side s1 = side(w.n_left, w.left_n, w.left_two_s, w.left_dim);
  const Side s2 = side(w.n_right, w.right_n, w.right_two_s, w.right_dim);
  const int n1 = (int)s1.n.size(), n2 = (int)s2.n.size();
  auto check = [](const dmrg_su2_operator& o, int ns) {
    DMRG_REQUIRE(o.n_blocks >= 0 && (o.n_blocks == 0 || (o.out_sector && o.in_sector)), kErrInvalidArg,
                 "su2_product: NULL operator array");
    for (int i = 0; i < o.n_blocks; ++i)
      DMRG_REQUIRE(o.out_sector[i] >= 0 && o.out_sector[i] < ns && o.in_sector[i] >= 0 && o.in_sector[i] < ns,
                   kErrInvalidArg, "su2_product: operator block sector out of range");
  };
  check(a, n1);
  check(b, n2);
  // coupled sectors (i1, i2, 2S), numbered i1 slowest, then i2, then 2S
  std::vector<int> first((size_t)n1 * n2 + 1, 0);
  for (int i1 = 0; i1 < n1; ++i1)
    for (int i2 = 0; i2 < n2; ++i2) {
      const int lo = std::abs(s1.ts[i1] - s2.ts[i2]), hi = s1.ts[i1] + s2.ts[i2];
      first[(size_t)i1 * n2 + i2 + 1] = first[(size_t)i1 * n2 + i2] + (hi - lo) / 2 + 1;
    }
  Su2Product p;
  for (int ja = 0; ja < a.n_blocks; ++ja)
    for (int jb = 0; jb < b.n_blocks; ++jb) {
      const int i1p = a.out_sector[ja], i1 = a.in_sector[ja], i2p = b.out_sector[jb], i2 = b.in_sector[jb];
      const int ta2 = s1.ts[i1p], ta = s1.ts[i1], tb2 = s2.ts[i2p], tb = s2.ts[i2];
      const double sign = (parity_b && (s1.n[i1] & 1)) ? -1.0 : 1.0;
      for (int tS = std::abs(ta - tb); tS <= ta + tb; tS += 2)
        for (int tS2 = std::abs(ta2 - tb2); tS2 <= ta2 + tb2; tS2 += 2) {
          if (!triangle(tS, tk, tS2)) continue;
          const double c = std::sqrt((tS + 1.0) * (tk + 1.0) * (ta2 + 1.0) * (tb2 + 1.0)) *
                           wigner_9j(ta2, ta, tk1, tb2, tb, tk2, tS2, tS, tk);
          if (c == 0.0) continue;
          Su2Product::Block blk;
          blk.out = first[(size_t)i1p * n2 + i2p] + (tS2 - std::abs(ta2 - tb2)) / 2;
          blk.in = first[(size_t)i1 * n2 + i2] + (tS - std::abs(ta - tb)) / 2;
          blk.offset = p.size;
          blk.ja = ja;
          blk.jb = jb;
          blk.ra = s1.d[i1p];
          blk.ca = s1.d[i1];
          blk.rb = s2.d[i2p];
          blk.cb = s2.d[i2];
          blk.scale = sign * c;
          p.blocks.push_back(blk);
          p.size += (int64_t)blk.ra * blk.rb * blk.ca * blk.cb;
        }
    }
  return p;
}

void su2_product_run(const Su2Product& p, const dmrg_su2_operator& a, const dmrg_su2_operator& b, double* data,
                     hipStream_t s) {
  if (p.blocks.empty()) return;
  DMRG_REQUIRE(data && a.data && b.data && a.offset && b.offset, kErrInvalidArg, "su2_product: NULL data");
  std::vector<KronTask> tasks;
  tasks.reserve(p.blocks.size());
  for (const Su2Product::Block& k : p.blocks)
    tasks.push_back({a.data + a.offset[k.ja], b.data + b.offset[k.jb], data + k.offset, k.ra, k.ca, k.rb, k.cb,
                     k.scale});
  DevBuf d(tasks.size() * sizeof(KronTask));
  DMRG_HIP(hipMemcpyAsync(d.p, tasks.data(), tasks.size() * sizeof(KronTask), hipMemcpyHostToDevice, s));
  for (size_t off = 0; off < tasks.size(); off += (size_t)1 << 30) {
    const unsigned cnt = (unsigned)std::min<size_t>(tasks.size() - off, (size_t)1 << 30);
    hipLaunchKernelGGL(k_kron_tasks, dim3(cnt), dim3(256), 0, s, d.as<KronTask>() + off);
  }
  DMRG_HIP(hipGetLastError());
  DMRG_HIP(hipStreamSynchronize(s));  // the task list is released on return
}

Su2Rotation su2_rotation_plan(const dmrg_su2_basis& basis, int n_blocks, const int32_t* out_sector,
                              const int32_t* in_sector) {
  const int nc = basis.n_coupled, ng = basis.n_groups;
  DMRG_REQUIRE(nc >= 0 && ng >= 0 && (nc == 0 || (basis.coupled_dim && basis.coupled_group)) &&
                   (ng == 0 || basis.group_dim),
               kErrInvalidArg, "su2_rotate: NULL basis array");
  for (int c = 0; c < nc; ++c)
    DMRG_REQUIRE(basis.coupled_dim[c] > 0 && basis.coupled_group[c] >= -1 && basis.coupled_group[c] < ng,
                 kErrInvalidArg, "su2_rotate: coupled sector with a bad dimension or group");
  for (int g = 0; g < ng; ++g)
    DMRG_REQUIRE(basis.group_dim[g] > 0, kErrInvalidArg, "su2_rotate: a new sector needs kept multiplets");
  DMRG_REQUIRE(n_blocks >= 0 && (n_blocks == 0 || (out_sector && in_sector)), kErrInvalidArg,
               "su2_rotate: NULL block array");
  std::map<std::pair<int, int>, std::vector<int>> by;
  for (int j = 0; j < n_blocks; ++j) {
    DMRG_REQUIRE(out_sector[j] >= 0 && out_sector[j] < nc && in_sector[j] >= 0 && in_sector[j] < nc,
                 kErrInvalidArg, "su2_rotate: block sector out of range");
    const int g2 = basis.coupled_group[out_sector[j]], g = basis.coupled_group[in_sector[j]];
    if (g2 >= 0 && g >= 0) by[{g2, g}].push_back(j);
  }
  Su2Rotation r;
  for (auto& kv : by) {
    r.outs.push_back({kv.first.first, kv.first.second, r.size, kv.second});
    r.size += (int64_t)basis.group_dim[kv.first.first] * basis.group_dim[kv.first.second];
  }
  return r;
}

void su2_rotation_run(const Su2Rotation& r, const dmrg_su2_basis& basis, const int32_t* out_sector,
                      const int32_t* in_sector, const int64_t* offset, const double* data, double* out,
                      hipStream_t s) {
  if (r.outs.empty()) return;
  DMRG_REQUIRE(basis.proj && data && out && offset, kErrInvalidArg, "su2_rotate: NULL data");
  const int32_t* dim = basis.coupled_dim;
  const int32_t* D = basis.group_dim;
  // stage 1: Y_j = X_j proj[in] (d_out x D_g), one problem per block
  int64_t ws = 0;
  for (const auto& o : r.outs)
    for (int j : o.blocks) ws += (int64_t)dim[out_sector[j]] * D[o.g];
  DevBuf buf((size_t)std::max<int64_t>(ws, 1) * sizeof(double));
  double* Y = buf.as<double>();
  GemmBatch b1, b2;
  int64_t at = 0;
  for (const auto& o : r.outs) {
    const size_t s2 = b2.segs.size();
    for (int j : o.blocks) {
      const int c2 = out_sector[j], c = in_sector[j];
      DMRG_REQUIRE(basis.proj[c] && basis.proj[c2], kErrInvalidArg, "su2_rotate: NULL projector of a kept sector");
      const size_t s0 = b1.segs.size();
      b1.segs.push_back({data + offset[j], basis.proj[c], dim[c], D[o.g], dim[c], 0, 1.0});
      b1.add_problem(Y + at, D[o.g], dim[c2], D[o.g], s0, s0 + 1, 0);
      // stage 2: O[g', g] += proj[c']^T Y_j
      b2.segs.push_back({basis.proj[c2], Y + at, D[o.g2], D[o.g], dim[c2], kTransA, 1.0});
      at += (int64_t)dim[c2] * D[o.g];
    }
    b2.add_problem(out + o.offset, D[o.g], D[o.g2], D[o.g], s2, b2.segs.size(), 0);
  }
  launch_gemm_f64(b1, s);
  launch_gemm_f64(b2, s);
  DMRG_HIP(hipStreamSynchronize(s));  // the workspace is released on return
}

}  // namespace dmrg
