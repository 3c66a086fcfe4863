"""Pins of the oracle's transition RDMs (oracle.fock.rdm12).

Each check uses something other than rdm12's own formula: the closed form of
a single determinant, the raw four-operator Hamiltonian (contraction and
finite differences), particle-number traces and the permutation symmetries
of the definitions.
"""
import numpy as np
import pytest

from oracle.fock import DetSpace, raw_hamiltonian, rdm12
from synthetic.integrals import make_integrals


def _vecs(space, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=space.dim), rng.normal(size=space.dim)


@pytest.mark.parametrize("K,N,tsz", [(3, 3, 1), (4, 4, 0), (3, 2, 0)])
def test_contraction_equals_raw_hamiltonian(K, N, tsz):
    """<bra|H|ket> = sum h gamma + 1/2 sum (pq|rs) Gamma with H built from
    spin-orbital strings, non-symmetric bra/ket."""
    space = DetSpace.sector(K, N, tsz)
    h, eri = make_integrals(K, 7 + K)
    a, b = _vecs(space, K)
    g, G = rdm12(space, a, b)
    H = raw_hamiltonian(space, h, eri)
    ref = a @ (H @ b)
    got = np.sum(h * g) + 0.5 * np.sum(eri * G)
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_finite_differences_of_raw_hamiltonian():
    """Every entry of h and (pq|rs) is an independent input: central
    differences of <bra|H|ket> (linear, so exact up to rounding)."""
    K = 3
    space = DetSpace.sector(K, 3, 1)
    h, eri = make_integrals(K, 3)
    a, b = _vecs(space, 5)
    g, G = rdm12(space, a, b)
    f = lambda hh, ee: a @ (raw_hamiltonian(space, hh, ee) @ b)
    rng = np.random.default_rng(1)
    d = 1e-5
    for _ in range(4):
        p, q = rng.integers(0, K, size=2)
        hp, hm = h.copy(), h.copy()
        hp[p, q] += d
        hm[p, q] -= d
        fd = (f(hp, eri) - f(hm, eri)) / (2 * d)
        assert abs(fd - g[p, q]) <= 1e-8 * max(1.0, abs(g[p, q]))
    for _ in range(6):
        idx = tuple(rng.integers(0, K, size=4))
        ep, em = eri.copy(), eri.copy()
        ep[idx] += d
        em[idx] -= d
        fd = (f(h, ep) - f(h, em)) / (2 * d)
        assert abs(fd - 0.5 * G[idx]) <= 1e-8 * max(1.0, abs(G[idx]))


def test_single_determinant_closed_form():
    """For one determinant |D>: gamma = diag(n_p), and
    Gamma_pqrs = d_pq d_rs (n_p n_r - d_pr n_p) - d_ps d_qr (1 - d_pr) sum_s n_ps n_rs."""
    K = 4
    space = DetSpace.sector(K, 5, 1)
    rng = np.random.default_rng(3)
    for _ in range(5):
        j = int(rng.integers(space.dim))
        v = np.zeros(space.dim)
        v[j] = 1.0
        det = int(space.dets[j])
        occ = np.array([[(det >> (2 * p + s)) & 1 for s in (0, 1)] for p in range(K)], dtype=float)
        n = occ.sum(1)
        g, G = rdm12(space, v, v)
        assert np.allclose(g, np.diag(n), atol=1e-14)
        ref = np.zeros((K,) * 4)
        for p in range(K):
            for r in range(K):
                ref[p, p, r, r] += n[p] * n[r] - (p == r) * n[p]
                if p != r:
                    ref[p, r, r, p] -= occ[p] @ occ[r]
        assert np.allclose(G, ref, atol=1e-14)


def test_traces_and_symmetries():
    K, N = 4, 4
    space = DetSpace.sector(K, N, 0)
    a, b = _vecs(space, 11)
    g, G = rdm12(space, a, b)
    ov = a @ b
    assert abs(np.trace(g) - N * ov) < 1e-11
    assert abs(np.einsum("pprr->", G) - N * (N - 1) * ov) < 1e-10
    assert np.allclose(np.einsum("pqrr->pq", G), (N - 1) * g, atol=1e-11)
    # transition RDMs: swapping bra and ket transposes the operator strings
    g2, G2 = rdm12(space, b, a)
    assert np.allclose(g2, g.T, atol=1e-12)
    assert np.allclose(G2, G.transpose(1, 0, 3, 2), atol=1e-12)
    # a real state: Gamma_pqrs = Gamma_rspq = Gamma_qpsr
    g, G = rdm12(space, a, a)
    assert np.allclose(G, G.transpose(2, 3, 0, 1), atol=1e-12)
    assert np.allclose(G, G.transpose(1, 0, 3, 2), atol=1e-12)
    assert np.allclose(g, g.T, atol=1e-12)
