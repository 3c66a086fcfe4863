"""Pins of the oracle's total spin <S^2> (CPU).

* closed forms: a high-spin determinant (S = N/2), a closed shell (S = 0),
  the open-shell singlet and the Sz = 0 triplet of two electrons (which fix
  the relative sign of the two determinants, so a sign error in S_+ swaps
  them);
* the spin-free Hamiltonian commutes with S^2 on a sector, and its
  eigenvectors have <S^2> = S(S+1);
* the identity <S^2> = -N(N-4)/4 - 1/2 sum_pq Gamma_pqqp with the 2-RDM of
  rdm12, on random vectors (not spin eigenstates).
"""
import numpy as np
import pytest

from oracle.fock import DetSpace, fci, rdm12, s_squared
from synthetic import make_integrals


def _vec(space, coeffs):
    v = np.zeros(space.dim)
    for det, c in coeffs:
        v[space.index([det])[0]] = c
    return v


def test_high_spin_and_closed_shell_determinants():
    sp3 = DetSpace.sector(4, 3, 3)  # three up electrons in orbitals 0, 1, 2
    v = _vec(sp3, [((1 << 0) | (1 << 2) | (1 << 4), 1.0)])
    assert s_squared(sp3, v) == pytest.approx(3.75, abs=1e-14)
    sp4 = DetSpace.sector(3, 4, 0)  # orbitals 0 and 1 doubly occupied
    v = _vec(sp4, [(0b1111, 1.0)])
    assert s_squared(sp4, v) == pytest.approx(0.0, abs=1e-14)


def test_two_electron_singlet_and_triplet():
    sp = DetSpace.sector(2, 2, 0)
    a_up_b_dn = (1 << 0) | (1 << 3)  # a+_{0 up} a+_{1 dn} |vac>
    a_dn_b_up = (1 << 1) | (1 << 2)  # a+_{0 dn} a+_{1 up} |vac>
    r = 1 / np.sqrt(2)
    singlet = _vec(sp, [(a_up_b_dn, r), (a_dn_b_up, -r)])
    triplet = _vec(sp, [(a_up_b_dn, r), (a_dn_b_up, r)])
    assert s_squared(sp, singlet) == pytest.approx(0.0, abs=1e-14)
    assert s_squared(sp, triplet) == pytest.approx(2.0, abs=1e-14)


def test_fci_states_are_spin_eigenstates():
    h, eri = make_integrals(5, 5)
    w, v, space = fci(5, 4, 0, h, eri, nroots=6)
    for j in range(v.shape[1]):
        s2 = s_squared(space, v[:, j])
        S = (-1 + np.sqrt(1 + 4 * s2)) / 2
        assert abs(S - round(S)) < 1e-8, (j, s2)


@pytest.mark.parametrize("K,N,tsz", [(4, 4, 0), (4, 3, 1), (5, 4, 2)])
def test_s_squared_from_the_two_rdm(K, N, tsz):
    space = DetSpace.sector(K, N, tsz)
    v = np.random.default_rng(K * 10 + N).normal(size=space.dim)
    v /= np.linalg.norm(v)
    _, G = rdm12(space, v, v)
    via_rdm = -N * (N - 4) / 4 - 0.5 * np.einsum("pqqp->", G)
    assert via_rdm == pytest.approx(s_squared(space, v), abs=1e-12)
