"""Orbital gradient of the energy from the RDMs (the consumer of the backward).

TEST INFRASTRUCTURE ONLY.  With real orbitals rotated by U = exp(kappa),
kappa antisymmetric, the integrals transform as h' = U^T h U and
(pq|rs)' = sum U_ap U_bq U_cr U_ds (ab|cd).  At fixed state coefficients the
energy E(kappa) = sum h'_pq gamma_pq + 1/2 sum (pq|rs)' Gamma_pqrs has, at
kappa = 0, the derivative (the DMRG-SCF / CASSCF orbital gradient)

    dE / dkappa_pq = 2 (F_qp - F_pq),
    F_pq = sum_r gamma_pr h_qr + sum_rst Gamma_prst (qr|st)   (generalised Fock),

for the independent parameters kappa_pq (p > q), kappa_qp = -kappa_pq.  (With
h' = h + h kappa - kappa h to first order, the one-body part is
sum gamma (h kappa - kappa h) = 2 [(gamma h)_qp - (gamma h)_pq]; texts that
rotate with exp(-kappa) carry the opposite sign.)

Pins: tests/test_oracle_orbital.py (central differences of <psi|H(kappa)|psi>
with rotated integrals through the raw Hamiltonian matvec, antisymmetry).
"""
import numpy as np
import scipy.linalg as sla


def generalized_fock(h, eri, gamma, Gamma):
    K = h.shape[0]
    F = gamma @ h.T
    F = F + Gamma.reshape(K, K ** 3) @ eri.reshape(K, K ** 3).T
    return F


def orbital_gradient(h, eri, gamma, Gamma):
    """g[p, q] = dE/dkappa_pq = 2 (F_qp - F_pq), U = exp(kappa)."""
    F = generalized_fock(h, eri, gamma, Gamma)
    return 2.0 * (F.T - F)


def rotate_integrals(h, eri, kappa):
    """h' = U^T h U and (pq|rs)' with U = exp(kappa)."""
    U = sla.expm(kappa)
    h2 = U.T @ h @ U
    e2 = np.einsum("ap,bq,cr,ds,abcd->pqrs", U, U, U, U, eri, optimize=True)
    return h2, e2
