// Reverse mode of the two-site sigma with respect to the integrals.
#pragma once
#include "engine.h"

namespace dmrg {

struct BackwardStats {
  double ms_chain = 0;   // rebuilding both blocks with provenance
  double ms_window = 0;  // window adjoints
  double ms_adjoint = 0; // adjoint renormalisation and integral contractions
  int64_t n_groups = 0;  // component groups visited
};

// For fixed window vectors psi and lam (API layout of the window) and the
// fixed MPS, f(h, eri) = <lam, H_eff(h, eri) psi> is linear in the integrals.
// Writes its gradient to grad (host, K*K entries for h followed by K^4 for
// eri, same index order as the integrals; overwritten).  precision 0: FP64
// contractions; 1 / 2: BF16 / split-BF16x3 contractions with FP32
// accumulation flushed into FP64 (the blocks are rebuilt in FP64).
BackwardStats sigma_backward(const Problem& P, const Mps& m, int window, const double* psi,
                             const double* lam, double* grad, int64_t ws_budget, hipStream_t s,
                             int precision = 0);

// Orbital gradient of the energy from the RDMs of sigma_backward: with
// gamma = dh and Gamma = 2 deri (device, K*K and K^4), the generalised Fock
// matrix F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst (qr|st) and
// g_pq = dE/dkappa_pq = 2 (F_qp - F_pq) for orbitals rotated by
// U = exp(kappa) at a fixed state (device outputs, K*K; fock may be null).
void orbital_gradient(const Problem& P, const double* dh, const double* deri, double* fock,
                      double* grad, hipStream_t s);

}  // namespace dmrg
