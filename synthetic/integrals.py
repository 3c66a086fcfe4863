"""Seeded synthetic one- and two-electron integrals.

The paper's production integrals (Fe4S4 CAS(54,36), Fe5S12H4 CAS(89,102))
are not available, so every workload uses integrals drawn from this recipe,
taking only the active-space *shape* from the paper:

* h: symmetric K x K.  Diagonal = linspace(-2, -0.2, K) (most bound orbital
  first); strict upper triangle iid N(0, 0.1), mirrored.
* (pq|rs) = sum_{L<24} B_L[p,q] B_L[r,s] with every B_L symmetric, upper
  triangle (diagonal included) iid N(0, 0.15), mirrored.  This makes the ERI
  tensor 8-fold symmetric and positive semidefinite as a (pq),(rs) matrix,
  like a real Coulomb matrix.

Draw order from numpy.random.default_rng(seed): the off-diagonal of h, then
B_0 ... B_23.  Arrays are float64, row-major, chemists' notation.
"""
import numpy as np


def make_integrals(n_orb: int, seed: int, n_aux: int = 24,
                   sd_h: float = 0.1, sd_b: float = 0.15):
    """Return (h, eri) with shapes (K, K) and (K, K, K, K), float64."""
    K = int(n_orb)
    rng = np.random.default_rng(seed)
    h = np.zeros((K, K))
    h[np.diag_indices(K)] = np.linspace(-2.0, -0.2, K)
    iu = np.triu_indices(K, 1)
    off = rng.normal(0.0, sd_h, size=len(iu[0]))
    h[iu] = off
    h[(iu[1], iu[0])] = off
    iu0 = np.triu_indices(K, 0)
    B = np.zeros((n_aux, K, K))
    for L in range(n_aux):
        v = rng.normal(0.0, sd_b, size=len(iu0[0]))
        B[L][iu0] = v
        B[L][(iu0[1], iu0[0])] = v
    Bm = B.reshape(n_aux, K * K)
    eri = (Bm.T @ Bm).reshape(K, K, K, K)
    return np.ascontiguousarray(h), np.ascontiguousarray(eri)
