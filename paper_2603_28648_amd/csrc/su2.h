// Spin-adapted (SU(2)) contraction of scalar products of tensor operators on
// the reduced window vector (see dmrg_su2_sigma in include/dmrg.h).
#pragma once
#include <cstdint>
#include <memory>
#include <vector>

#include <hip/hip_runtime.h>

#include "common.h"
#include "dmrg.h"
#include "gemm.h"
#include "gemm_bf16.h"

namespace dmrg {

// Length of the reduced window vector; throws Error(kErrInvalidArg) for an
// invalid window.
int64_t su2_psi_size(const dmrg_su2_window& w);

// Device descriptors of one window's spin-adapted sigma: per workspace
// chunk a stage-1 launch (T = psi B^T for the chunk's right operators) and a
// stage-2 launch (partial sums of sigma += W c A T), on plan-owned psi,
// partial sums and workspace; sigma is the sum of the partial sums.
struct Su2Plan {
  int64_t psi_size = 0;
  DevBuf psi, psi_b, ws;  // psi as given, psi regrouped by right sector, stage-1 workspace
  DevBuf regroup;          // copy tasks psi -> psi_b
  int n_regroup = 0;
  DevBuf part, ones;  // n_parts partial sums of sigma (psi_size each), and n_parts ones
  int n_parts = 1;
  std::vector<DevGemm> s1, s2;
  // split-BF16x3 plans: packed operator blocks, psi_b packed per call, the
  // BF16 hi/lo workspace and the descriptors
  int precision = DMRG_FP64;
  DevBuf opk, psi_pack, psi_pack_ops, wsk;
  int n_psi_pack = 0;
  int64_t psi_pack_chunks = 0;
  std::vector<DevGemmB> s1b, s2b;
  int64_t n_segments = 0, ws_doubles = 0;
  double flops1 = 0, flops2 = 0;
};

// Stage-2 product lists are split so that a launch has about this many
// pieces (DMRG_SU2_PARTS overrides), into at most kSu2MaxParts partial sums
// of at most kSu2PartialBudget doubles in all.
constexpr size_t kSu2PartsPerLaunch = 8192;
constexpr int kSu2MaxParts = 256;
constexpr int64_t kSu2PartialBudget = (int64_t)1 << 27;

// Builds the plan (host checks as dmrg_su2_sigma; precision DMRG_FP64 or
// DMRG_BF16X3; ws_budget in doubles).
std::unique_ptr<Su2Plan> su2_plan(const dmrg_su2_window& w, int n_left_ops, const dmrg_su2_operator* left_ops,
                                  int n_right_ops, const dmrg_su2_operator* right_ops, int n_pairs,
                                  const dmrg_su2_pair* pairs, int precision, int64_t ws_budget, hipStream_t s);

// sigma = the plan's contraction of psi, stream-ordered (no synchronisation).
void su2_run(Su2Plan& p, const double* psi, double* sigma, hipStream_t s);

// {j1 j2 j3; j4 j5 j6} for doubled arguments (Racah's formula); exposed for
// the recoupling factors.
double wigner_6j(int tj1, int tj2, int tj3, int tj4, int tj5, int tj6);

}  // namespace dmrg
