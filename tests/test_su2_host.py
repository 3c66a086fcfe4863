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


def _host_op(blocks):
    """A dmrg_su2_operator with host sector arrays only (no data)."""
    import ctypes
    from paper_2603_28648_amd._binding import Su2Operator, _ptr
    b = np.asarray(blocks, dtype=np.int64).reshape(-1, 2)
    o = np.ascontiguousarray(b[:, 0], dtype=np.int32)
    i = np.ascontiguousarray(b[:, 1], dtype=np.int32)
    off = np.zeros(len(b), dtype=np.int64)
    op = Su2Operator(len(b), _ptr(o, ctypes.c_int32), _ptr(i, ctypes.c_int32), _ptr(off, ctypes.c_int64), None)
    return op, (o, i, off)


@pytest.mark.parametrize("dn1,tk1,dn2,tk2,tk", [(1, 1, 0, 0, 1), (1, 1, 1, 1, 2), (0, 2, -1, 1, 3), (2, 0, -1, 1, 1)])
def test_product_size_matches_the_oracle_blocks(dn1, tk1, dn2, tk2, tk):
    """dmrg_su2_product_size (host only) counts the blocks and elements of
    the oracle's product_operator on the same sectors."""
    import ctypes
    from paper_2603_28648_amd._binding import Su2Window, load_library, _su2_window
    from synthetic.su2 import random_operator
    rng = np.random.default_rng(3 + tk)
    sec1, _ = sector_window(8, 0, 30, rng)
    sec2 = [(0, 0, 1), (1, 1, 1), (2, 0, 1)]  # one orbital's multiplets
    t1 = random_operator(sec1, dn1, tk1, rng, keep=1.0)
    t2 = random_operator(sec2, dn2, tk2, rng, keep=1.0)
    want = su2.product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, abs(dn2) % 2)
    want = {k: v for k, v in want.items() if np.any(v != 0)}
    keep = []
    w = _su2_window(sec1, sec2, 0, 0, keep)
    a, ka = _host_op(sorted(t1))
    b, kb = _host_op(sorted(t2))
    nb, ne = ctypes.c_int32(), ctypes.c_int64()
    lib = load_library()
    assert lib.dmrg_su2_product_size(ctypes.byref(w), ctypes.byref(a), ctypes.byref(b), tk1, tk2, tk,
                                     ctypes.byref(nb), ctypes.byref(ne)) == 0
    assert nb.value == len(want) > 0
    assert ne.value == sum(v.size for v in want.values())


def test_rotate_size_and_errors():
    """dmrg_su2_rotate_size (host only): one output per pair of kept new
    sectors that receives a block, D_g' x D_g elements each; bad indices are
    errors."""
    import ctypes
    from paper_2603_28648_amd._binding import Su2Basis, load_library, _ptr
    lib = load_library()
    cd = np.array([2, 3, 1, 4], dtype=np.int32)
    cg = np.array([0, 0, 1, -1], dtype=np.int32)
    gd = np.array([4, 1], dtype=np.int32)
    ptrs = (ctypes.c_void_p * 4)()
    basis = Su2Basis(4, _ptr(cd, ctypes.c_int32), _ptr(cg, ctypes.c_int32), 2, _ptr(gd, ctypes.c_int32), ptrs)
    bo = np.array([0, 1, 2, 3, 2], dtype=np.int32)
    bi = np.array([1, 2, 0, 0, 2], dtype=np.int32)
    nb, ne = ctypes.c_int32(), ctypes.c_int64()
    assert lib.dmrg_su2_rotate_size(ctypes.byref(basis), 5, _ptr(bo, ctypes.c_int32), _ptr(bi, ctypes.c_int32),
                                    ctypes.byref(nb), ctypes.byref(ne)) == 0
    # (0,0) from blocks 0; (0,1) from block 1; (1,0) from block 2; (1,1) from block 4; block 3 is kept out
    assert nb.value == 4 and ne.value == 4 * 4 + 4 * 1 + 1 * 4 + 1 * 1
    bad = np.array([4, 1, 2, 3, 2], dtype=np.int32)
    assert lib.dmrg_su2_rotate_size(ctypes.byref(basis), 5, _ptr(bad, ctypes.c_int32), _ptr(bi, ctypes.c_int32),
                                    ctypes.byref(nb), ctypes.byref(ne)) == -1
    cg_bad = np.array([0, 0, 2, -1], dtype=np.int32)
    basis_bad = Su2Basis(4, _ptr(cd, ctypes.c_int32), _ptr(cg_bad, ctypes.c_int32), 2, _ptr(gd, ctypes.c_int32), ptrs)
    assert lib.dmrg_su2_rotate_size(ctypes.byref(basis_bad), 5, _ptr(bo, ctypes.c_int32), _ptr(bi, ctypes.c_int32),
                                    ctypes.byref(nb), ctypes.byref(ne)) == -1
