"""Pins of the projected-Hamiltonian oracle P^T H P (CPU)."""
import numpy as np
import pytest

from oracle.fock import fci
from oracle.projection import ProjectedHamiltonian, left_states, right_states
from synthetic import make_integrals, make_mps


def test_left_and_right_states_are_orthonormal():
    m = make_mps(7, 7, 1, 20, 3, 11)
    L, R = left_states(m, 3), right_states(m, 3)
    assert np.max(np.abs(L.T @ L - np.eye(L.shape[1]))) < 1e-13
    assert np.max(np.abs(R.T @ R - np.eye(R.shape[1]))) < 1e-13


@pytest.mark.parametrize("K,N,tsz,i", [(4, 4, 0, 1), (6, 6, 0, 2), (6, 5, -1, 2)])
def test_complete_bonds_reproduce_fci(K, N, tsz, i):
    # bonds i and i+2 hold every state of their blocks: P spans the FCI sector
    h, eri = make_integrals(K, 20 + K)
    m = make_mps(K, N, tsz, 10 ** 6, i, 3)
    Hd, _ = ProjectedHamiltonian(m, h, eri).dense()
    E = fci(K, N, tsz, h, eri)[0][0]
    assert abs(np.linalg.eigvalsh(Hd)[0] - E) < 1e-10
    assert np.max(np.abs(Hd - Hd.T)) < 1e-12 * np.max(np.abs(Hd))


def test_cas8_complete_window_reproduces_fci():
    # 8 orbitals / 8 electrons: D=64 keeps every state of 3 orbitals, so the
    # middle window spans the whole FCI space of dimension C(8,4)^2 = 4900
    h, eri = make_integrals(8, 8)
    m = make_mps(8, 8, 0, 64, 3, 1008)
    assert m.psi_size() == 4900
    E = fci(8, 8, 0, h, eri)[0][0]
    PH = ProjectedHamiltonian(m, h, eri)
    import scipy.sparse.linalg as spla
    keys = sorted(m.psi)
    n = m.psi_size()

    def mv(x):
        out, o = {}, 0
        for k in keys:
            dl, dr = m.psi[k].shape
            out[k] = x[o:o + dl * dr].reshape(dl, dr)
            o += dl * dr
        s = PH.apply(out)
        return np.concatenate([s[k].ravel() for k in keys])
    w = spla.eigsh(spla.LinearOperator((n, n), matvec=mv), k=1, which="SA", tol=1e-12)[0]
    assert abs(w[0] - E) < 1e-9


def test_truncated_window_is_variational():
    h, eri = make_integrals(6, 6)
    E = fci(6, 6, 0, h, eri)[0][0]
    for D, seed in [(6, 1), (9, 2), (12, 3)]:
        m = make_mps(6, 6, 0, D, 2, seed)
        Hd, _ = ProjectedHamiltonian(m, h, eri).dense()
        assert np.linalg.eigvalsh(Hd)[0] >= E - 1e-12


def test_two_site_chain_is_plain_fci():
    # K = 2, window (0,1): both blocks are the vacuum, H_eff is H itself
    t, U = 0.9, 2.5
    h = np.array([[0.1, -t], [-t, -0.2]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0], eri[1, 1, 1, 1] = U, 0.5 * U
    m = make_mps(2, 2, 0, 16, 0, 1)
    Hd, _ = ProjectedHamiltonian(m, h, eri).dense()
    w = np.linalg.eigvalsh(Hd)
    wf = np.linalg.eigvalsh(__import__("oracle.fock", fromlist=["DetSpace"]).DetSpace
                            .sector(2, 2, 0).hamiltonian(h, eri).toarray())
    assert np.max(np.abs(w - wf)) < 1e-13
