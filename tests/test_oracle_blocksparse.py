"""Pin of the block-sparse normal/complementary oracle against P^T H P (CPU)."""
import numpy as np
import pytest

from oracle.blocksparse import BlockSparseSigma
from oracle.projection import ProjectedHamiltonian
from synthetic import make_integrals, make_mps

CASES = [(2, 2, 0, 16, 0), (4, 4, 0, 100, 0), (4, 4, 0, 100, 1), (4, 4, 0, 100, 2),
         (5, 5, 1, 8, 1), (5, 4, -2, 12, 3), (6, 6, 0, 12, 2), (6, 5, 1, 10, 0),
         (6, 7, -1, 10, 4), (6, 6, 2, 12, 3), (7, 7, 1, 30, 2)]


def _rel(a, b):
    return (np.sqrt(sum(np.sum((a[k] - b[k]) ** 2) for k in b))
            / np.sqrt(sum(np.sum(b[k] ** 2) for k in b)))


@pytest.mark.parametrize("K,N,tsz,D,i", CASES)
def test_blocksparse_equals_projection(K, N, tsz, D, i):
    h, eri = make_integrals(K, 11 + K)
    m = make_mps(K, N, tsz, D, i, 5 + i)
    ref = ProjectedHamiltonian(m, h, eri).apply(m.psi)
    got = BlockSparseSigma(m, h, eri).apply(m.psi)
    assert _rel(got, ref) < 1e-12


@pytest.mark.slow
def test_blocksparse_equals_projection_cas8():
    h, eri = make_integrals(8, 8)
    for (D, i) in [(64, 3), (24, 1), (24, 5)]:
        m = make_mps(8, 8, 0, D, i, 1008)
        ref = ProjectedHamiltonian(m, h, eri).apply(m.psi)
        got = BlockSparseSigma(m, h, eri).apply(m.psi)
        assert _rel(got, ref) < 1e-12


def test_planted_sign_error_is_caught():
    # dropping the Jordan-Wigner sign of the partition terms must break parity
    import oracle.blocksparse as bs
    h, eri = make_integrals(5, 3)
    m = make_mps(5, 5, 1, 12, 1, 2)
    ref = ProjectedHamiltonian(m, h, eri).apply(m.psi)
    b = BlockSparseSigma(m, h, eri)
    flipped = [(c, XL, XR) for (c, XL, XR) in b.terms]
    # remove the JW sign by pretending every right operator is even
    class Even:
        def __init__(self, op):
            self.__dict__.update(op.__dict__)
        parity = 0
    bad = [(c, XL, Even(XR) if XR is not None else None) for (c, XL, XR) in flipped]
    got = b.from_matrix(b.apply_matrix(b.to_matrix(m.psi), bad), {k: v.shape for k, v in m.psi.items()})
    assert _rel(got, ref) > 1e-3


@pytest.mark.parametrize("K,N,tsz,D,i", [(4, 4, 0, 100, 1), (5, 4, -2, 12, 3), (6, 6, 2, 12, 3),
                                         (6, 5, 1, 10, 0), (7, 7, 1, 30, 2)])
def test_diagonal_equals_dense_projection(K, N, tsz, D, i):
    """diag(H_eff) of the partition equals the diagonal of the dense P^T H P."""
    from oracle.projection import psi_template
    h, eri = make_integrals(K, 11 + K)
    m = make_mps(K, N, tsz, D, i, 5 + i)
    dense, keys = ProjectedHamiltonian(m, h, eri).dense()
    tmpl = psi_template(m)
    got = BlockSparseSigma(m, h, eri).diagonal(tmpl)
    flat = np.concatenate([got[k].ravel() for k in keys])
    assert np.max(np.abs(flat - np.diag(dense))) < 1e-12 * np.max(np.abs(np.diag(dense)))
