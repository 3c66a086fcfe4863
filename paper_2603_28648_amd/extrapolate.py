"""Sweep convergence rule and truncation-free extrapolations (host-side
analysis of sweep energies; no device work).

* Sweep stopping rule (Numerical procedure section): the energies of three
  subsequent sweeps agree, max(|E_s - E_(s-1)|, |E_(s-1) - E_(s-2)|) < tol,
  with tol = 1e-5 Ha in the paper.
* The two extrapolations to the truncation-free limit (Numerical benchmark
  section, Fig. 2): a second-order polynomial in 1/D evaluated at 1/D = 0,
  and a second-order polynomial in the largest truncation error of the last
  sweep evaluated at zero truncation error.
"""
import numpy as np


def sweep_converged(energies, tol=1e-5):
    """True once the last three sweep energies agree within tol."""
    if len(energies) < 3:
        return False
    e = energies[-3:]
    return max(abs(e[2] - e[1]), abs(e[1] - e[0])) < tol


def _poly_at_zero(x, y, order):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if len(x) < order + 1:
        raise ValueError(f"a polynomial of order {order} needs at least {order + 1} points")
    coef = np.polynomial.polynomial.polyfit(x, y, order)
    return float(coef[0]), coef


def extrapolate_inverse_bond(bond_dims, energies, order=2):
    """E(1/D -> 0) from a polynomial fit of E against 1/D; returns
    (E_ext, coefficients in increasing powers of 1/D)."""
    return _poly_at_zero(1.0 / np.asarray(bond_dims, dtype=np.float64), energies, order)


def extrapolate_truncation(trunc_errors, energies, order=2):
    """E(eps_tr -> 0) from a polynomial fit of E against the largest
    truncation error of the last sweep; returns (E_ext, coefficients)."""
    return _poly_at_zero(trunc_errors, energies, order)
