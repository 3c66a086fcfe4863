// Spin-adapted (SU(2)) contraction of scalar products of tensor operators on
// the reduced window vector (see dmrg_su2_sigma in include/dmrg.h).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

#include "dmrg.h"

namespace dmrg {

// Length of the reduced window vector; throws Error(kErrInvalidArg) for an
// invalid window.
int64_t su2_psi_size(const dmrg_su2_window& w);

// sigma = sum over pairs of c [A^k x B^k]^0 psi on the stream (synchronised
// before returning: the stage-1 workspace is freed).
void su2_sigma(hipStream_t s, const dmrg_su2_window& w, int n_left_ops, const dmrg_su2_operator* left_ops,
               int n_right_ops, const dmrg_su2_operator* right_ops, int n_pairs, const dmrg_su2_pair* pairs,
               const double* psi, double* sigma);

// {j1 j2 j3; j4 j5 j6} for doubled arguments (Racah's formula); exposed for
// the recoupling factors.
double wigner_6j(int tj1, int tj2, int tj3, int tj4, int tj5, int tj6);

}  // namespace dmrg
