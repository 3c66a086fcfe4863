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
