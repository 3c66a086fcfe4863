"""Pins of the FCI oracle against closed forms and the raw definition (CPU)."""
import numpy as np
import pytest

from oracle.fock import DetSpace, fci, raw_hamiltonian
from synthetic import make_integrals


def test_spin_free_form_equals_raw_spin_orbital_sum():
    # H from E_pq products must equal the literal four-operator sum of the
    # Method-section Hamiltonian (chemists' notation), on every sector.
    for K in (2, 3):
        h, eri = make_integrals(K, 40 + K)
        sp = DetSpace.full(K)
        A = sp.hamiltonian(h, eri).toarray()
        B = raw_hamiltonian(sp, h, eri).toarray()
        assert np.max(np.abs(A - B)) < 1e-12


def test_one_body_closed_form():
    # g = 0: E = sum of the N_a + N_b lowest orbital energies of h.
    K = 6
    h, _ = make_integrals(K, 7)
    eri = np.zeros((K,) * 4)
    w = np.linalg.eigvalsh(h)
    for N, tsz in [(6, 0), (5, 1), (4, 2), (7, -1)]:
        na, nb = (N + tsz) // 2, (N - tsz) // 2
        E, _, _ = fci(K, N, tsz, h, eri)
        assert abs(E[0] - (w[:na].sum() + w[:nb].sum())) < 1e-11


@pytest.mark.parametrize("t,U", [(1.0, 3.0), (0.7, 5.0), (1.3, 0.0)])
def test_two_site_hubbard_closed_form(t, U):
    # h = -t off-diagonal, (pq|rs) = U delta_pqrs, half filling, Sz = 0:
    # E0 = (U - sqrt(U^2 + 16 t^2)) / 2.
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    E, _, _ = fci(2, 2, 0, h, eri)
    assert abs(E[0] - (U - np.sqrt(U * U + 16 * t * t)) / 2) < 1e-12


def test_single_orbital():
    h = np.array([[-1.3]])
    eri = np.array([[[[0.8]]]])
    assert abs(fci(1, 2, 0, h, eri)[0][0] - (2 * -1.3 + 0.8)) < 1e-14
    assert abs(fci(1, 1, 1, h, eri)[0][0] - (-1.3)) < 1e-14


def test_number_and_spin_are_conserved_and_h_is_symmetric():
    K = 3
    h, eri = make_integrals(K, 3)
    sp = DetSpace.full(K)
    H = sp.hamiltonian(h, eri)
    N, S = sp.number_op(), sp.sz2_op()
    assert abs(H - H.T).max() < 1e-13
    assert abs(H @ N - N @ H).max() < 1e-12
    assert abs(H @ S - S @ H).max() < 1e-12


def test_sector_is_a_block_of_the_full_space():
    K = 3
    h, eri = make_integrals(K, 5)
    full = DetSpace.full(K)
    Hf = full.hamiltonian(h, eri).toarray()
    sec = DetSpace.sector(K, 3, 1)
    Hs = sec.hamiltonian(h, eri).toarray()
    idx = full.index(sec.dets)
    assert np.max(np.abs(Hf[np.ix_(idx, idx)] - Hs)) < 1e-13


def test_matvec_equals_matrix():
    K = 5
    h, eri = make_integrals(K, 9)
    sp = DetSpace.sector(K, 5, 1)
    H = sp.hamiltonian(h, eri)
    x = np.random.default_rng(0).normal(size=sp.dim)
    assert np.max(np.abs(sp.hamiltonian_matvec(h, eri)(x) - H @ x)) < 1e-11
