"""Pins of the oracle's orbital gradient (oracle.orbital).

The generalised-Fock formula is checked against central differences of
<psi|H(kappa)|psi> with rotated integrals and a fixed state, the energy taken
from the E_pq-form Hamiltonian matvec (not from the RDM contraction)."""
import numpy as np

from oracle.fock import DetSpace, rdm12
from oracle.orbital import orbital_gradient, rotate_integrals
from synthetic.integrals import make_integrals


def test_orbital_gradient_matches_rotated_energy_differences():
    K, N = 4, 4
    space = DetSpace.sector(K, N, 0)
    h, eri = make_integrals(K, 3)
    v = np.random.default_rng(2).normal(size=space.dim)
    v /= np.linalg.norm(v)
    g, G = rdm12(space, v, v)
    grad = orbital_gradient(h, eri, g, G)
    assert np.allclose(grad, -grad.T, atol=1e-13)

    def energy(kappa):
        h2, e2 = rotate_integrals(h, eri, kappa)
        return v @ space.hamiltonian_matvec(h2, e2)(v)

    d = 1e-5
    for (p, q) in [(1, 0), (3, 1), (2, 0), (3, 2)]:
        kap = np.zeros((K, K))
        kap[p, q], kap[q, p] = d, -d
        fd = (energy(kap) - energy(-kap)) / (2 * d)
        assert abs(fd - grad[p, q]) <= 1e-7 * max(1.0, abs(grad[p, q])), (p, q, fd, grad[p, q])


def test_orbital_gradient_vanishes_for_a_rotation_invariant_case():
    """A single determinant with h and (pq|rs) diagonal in the orbital basis
    and only occupied-occupied / virtual-virtual couplings absent: every
    rotation between two occupied (or two virtual) orbitals leaves E unchanged."""
    K = 4
    space = DetSpace.sector(K, 4, 0)
    h = np.diag([-2.0, -1.0, 0.5, 1.0])
    eri = np.zeros((K,) * 4)
    for p in range(K):
        for q in range(K):
            eri[p, p, q, q] = 0.3 + 0.1 * (p == q)
    det = 0b00001111  # orbitals 0 and 1 doubly occupied
    v = np.zeros(space.dim)
    v[space.index([det])[0]] = 1.0
    g, G = rdm12(space, v, v)
    grad = orbital_gradient(h, eri, g, G)
    assert abs(grad[1, 0]) < 1e-13 and abs(grad[3, 2]) < 1e-13
