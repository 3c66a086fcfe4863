// Davidson eigensolver on the sigma plan of a window.
#pragma once
#include <vector>

#include "engine.h"

namespace dmrg {

struct DiagTask {
  const double* src;  // top-left element of a square block (row stride = ld)
  double* dst;        // d consecutive outputs
  int32_t d, ld;
};

struct DavidsonOpts {
  int max_iter = 100;     // correction vectors added (sigma products excluding restarts)
  int max_subspace = 24;
  int restart = 6;        // Ritz vectors kept at a thick restart
  int precondition = 2;   // 2: Olsen-corrected diag(H_eff), 1: plain diag, 0: none
  int refine = 0;         // 1: residual refinement instead of FP64 Davidson after a reduced stage
  double tol = 1e-6;      // ||H u - theta u||_2 with ||u|| = 1, last ladder stage
  int n_ladder = 1;       // number of precision stages
  int ladder[4] = {0, 0, 0, 0};
  double ladder_tol[4] = {0, 0, 0, 0};  // residual that ends stage s (< n_ladder-1)
};

struct DavidsonResult {
  double energy = 0, residual = 0, time_ms = 0, sigma_ms = 0;
  int iterations = 0;
  bool converged = false;
  int n_sigma[4] = {0, 0, 0, 0};
  std::vector<double> residual_history;
  std::vector<int> stage_history;
};

// diag(H_eff) for the preconditioner (stored in plan.diag).
void build_diagonal(SigmaPlan& plan, const Bond& bl, const Bond& br, hipStream_t s);
// Lowest eigenpair; psi is the start vector on input and the normalised Ritz
// vector on output.  Returns kOk or kWarnNotConverged.
int davidson(SigmaPlan& plan, double* psi, const DavidsonOpts& o, DavidsonResult& res,
             hipStream_t s);

}  // namespace dmrg
