"""Host side of the spin-adapted contraction: the packed vector length the
library reports (dmrg_su2_psi_size, no GPU) against the oracle's coupled
blocks, and the errors an invalid window raises."""
import numpy as np
import pytest

from oracle import su2
from paper_2603_28648_amd import DMRGError
from paper_2603_28648_amd._binding import su2_psi_size
from synthetic.su2 import sector_window


@pytest.mark.parametrize("n,tS,seed", [(8, 0, 1), (9, 1, 2), (10, 4, 3), (12, 2, 4), (3, 3, 5)])
def test_psi_size_is_the_sum_of_the_coupled_blocks(n, tS, seed):
    lsec, rsec = sector_window(n, tS, 50, np.random.default_rng(seed))
    want = sum(lsec[a][2] * rsec[b][2] for a, b in su2.coupled_blocks(lsec, rsec, n, tS))
    assert su2_psi_size(lsec, rsec, n, tS) == want


def test_psi_size_of_a_window_without_coupled_blocks_is_zero():
    assert su2_psi_size([(1, 1, 4)], [(1, 1, 3)], 2, 4) == 0  # S = 2 is not in 1/2 x 1/2
    assert su2_psi_size([(1, 1, 4)], [(1, 1, 3)], 2, 2) == 12


@pytest.mark.parametrize("lsec,rsec,n,tS", [
    ([(2, 1, 4)], [(1, 1, 3)], 3, 1),   # N and 2S of a sector with different parity
    ([(2, 0, 0)], [(1, 1, 3)], 3, 1),   # empty sector
    ([(2, 0, 4)], [(1, 1, 3)], 3, 0),   # total N and 2S with different parity
    ([(2, 0, 4)], [(1, 1, 3)], 3, -1),  # negative spin
    ([], [(1, 1, 3)], 1, 1),            # no left sector
])
def test_invalid_window_is_an_error(lsec, rsec, n, tS):
    with pytest.raises(DMRGError):
        su2_psi_size(lsec, rsec, n, tS)


def test_cas89_102_window_shape():
    """The spin-adapted workload's sectors: 2048 multiplets on each side,
    N and 2S of equal parity, and the packed vector the library sizes as
    the oracle's coupled blocks."""
    from synthetic.su2 import cas89_102_window, hamiltonian_pair_types, operator_layout
    lsec, rsec, n, tS = cas89_102_window(np.random.default_rng(102))
    assert (n, tS) == (89, 5)
    for secs in (lsec, rsec):
        assert sum(d for _, _, d in secs) == 2048
        assert all(N >= 0 and ts >= 0 and (N - ts) % 2 == 0 and d >= 1 for N, ts, d in secs)
        assert len(set((N, ts) for N, ts, _ in secs)) == len(secs)
    want = sum(lsec[a][2] * rsec[b][2] for a, b in su2.coupled_blocks(lsec, rsec, n, tS))
    assert su2_psi_size(lsec, rsec, n, tS) == want
    types = hamiltonian_pair_types(51, 51)
    assert sum(t[0] for t in types) == 2 + 4 * 51 + 2 * (1326 + 1275) + 2 * 2601
    for count, dnl, tk, dnr, parity in types:
        assert dnl + dnr == 0 and parity == abs(dnl) % 2  # particle number kept; fermion parity of the right side
        blocks, size = operator_layout(lsec, dnl, tk)
        assert blocks and size == sum(lsec[o][2] * lsec[i][2] for o, i, _ in blocks)
        for o, i, _ in blocks:  # particle change and the rank's triangle condition
            assert lsec[o][0] == lsec[i][0] + dnl and abs(lsec[o][1] - lsec[i][1]) <= tk <= lsec[o][1] + lsec[i][1]
