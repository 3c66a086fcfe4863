"""Pins of the truncation oracle (CPU).

The oracle's per-sector SVD, global selection and truncation error are
checked against a dense SVD of the unblocked two-site matrix and, at small
sizes, against the Schmidt values of the full Fock vector at the cut; the
moved state against the orthogonal projection of the original Fock vector
(Eckart-Young: squared distance = discarded weight); the new tensors for
canonical form; the tie rule on an exactly degenerate spectrum.
"""
import numpy as np
import pytest

from oracle.projection import psi_to_fock
from oracle.truncation import middle_sectors, truncate
from synthetic import make_mps

CASES = [  # K, N, 2Sz, D of the MPS, window, direction, kept D
    (5, 5, 1, 12, 1, +1, 6), (5, 5, 1, 12, 2, -1, 5),
    (6, 6, 0, 16, 2, +1, 9), (6, 6, 0, 16, 2, -1, 9),
    (6, 5, -1, 14, 0, +1, 3), (6, 7, 1, 14, 4, -1, 3),
    (6, 6, 2, 12, 3, +1, 8),
]


def _dense_matrix(m):
    """Unblocked two-site matrix: rows (left state of bond i, n1), columns (n2,
    right state of bond i+2), zero outside the allowed blocks."""
    i = m.window
    bl, br = m.bonds[i], m.bonds[i + 2]
    lo = np.cumsum([0] + [s[2] for s in bl])
    ro = np.cumsum([0] + [s[2] for s in br])
    ridx = {(s[0], s[1]): k for k, s in enumerate(br)}
    M = np.zeros((lo[-1] * 4, 4 * ro[-1]))
    QN = ((0, 0), (1, 1), (1, -1), (2, 0))
    for (li, n1, n2), blk in m.psi.items():
        q = (bl[li][0] + QN[n1][0] + QN[n2][0], bl[li][1] + QN[n1][1] + QN[n2][1])
        r = ridx[q]
        rows = 4 * np.arange(lo[li], lo[li + 1]) + n1
        cols = n2 * ro[-1] + np.arange(ro[r], ro[r + 1])
        M[np.ix_(rows, cols)] = blk
    return M


def _all_sv(res):
    return np.sort(np.concatenate([s for (_, s, _) in res["sectors"]]))[::-1]


@pytest.mark.parametrize("K,N,tsz,D,i,d,keep", CASES)
def test_spectrum_and_error_match_dense_svd(K, N, tsz, D, i, d, keep):
    m = make_mps(K, N, tsz, D, i, 40 + i)
    res = truncate(m, m.psi, d, keep)
    s = np.linalg.svd(_dense_matrix(m), compute_uv=False)
    ours = _all_sv(res)
    n = len(ours)
    assert np.allclose(ours, s[:n], atol=1e-13)
    assert np.all(s[n:] < 1e-12)
    w = s * s
    assert abs(res["eps"] - w[keep:].sum() / w.sum()) < 1e-13
    assert sum(b[2] for b in res["bond"]) == min(keep, int(np.sum(w > 1e-14 * w[0])))


@pytest.mark.parametrize("K,N,tsz,D,i,d,keep", CASES)
def test_spectrum_equals_fock_schmidt_values(K, N, tsz, D, i, d, keep):
    """Singular values of the Fock vector regrouped at the cut between
    orbitals i and i+1 (determinant integer = left + 4^(i+1) right)."""
    m = make_mps(K, N, tsz, D, i, 40 + i)
    res = truncate(m, m.psi, d, keep)
    v = psi_to_fock(m, m.psi).reshape(4 ** (K - i - 1), 4 ** (i + 1))
    s = np.linalg.svd(v, compute_uv=False)
    ours = _all_sv(res)
    assert np.allclose(ours, s[:len(ours)], atol=1e-13)
    assert np.all(s[len(ours):] < 1e-12)


@pytest.mark.parametrize("K,N,tsz,D,i,d,keep", CASES)
def test_moved_state_is_the_projection(K, N, tsz, D, i, d, keep):
    """Eckart-Young: the moved state is the orthogonal projection of the
    original onto the kept Schmidt states; squared distance = eps."""
    m = make_mps(K, N, tsz, D, i, 40 + i)
    res = truncate(m, m.psi, d, keep)
    v0 = psi_to_fock(m, m.psi)
    mv = res["mps"]
    assert mv.window == i + d
    v1 = psi_to_fock(mv, mv.psi)
    n0 = v0 @ v0
    assert abs((v0 - v1) @ (v0 - v1) - res["eps"] * n0) < 1e-12
    assert abs(v1 @ (v0 - v1)) < 1e-12
    assert abs(v1 @ v1 - (1 - res["eps"]) * n0) < 1e-12
    assert res["eps"] > 1e-6  # the cases truncate


@pytest.mark.parametrize("K,N,tsz,D,i,d", [(5, 5, 1, 12, 1, +1), (6, 6, 0, 16, 2, -1),
                                           (6, 6, 2, 12, 3, +1), (4, 4, 0, 100, 1, -1)])
def test_keeping_everything_reproduces_the_state(K, N, tsz, D, i, d):
    m = make_mps(K, N, tsz, D, i, 7)
    res = truncate(m, m.psi, d, 10 ** 6)
    assert res["eps"] < 1e-14
    v0 = psi_to_fock(m, m.psi)
    v1 = psi_to_fock(res["mps"], res["mps"].psi)
    assert np.max(np.abs(v0 - v1)) < 1e-13


@pytest.mark.parametrize("K,N,tsz,D,i,d,keep", CASES)
def test_new_tensors_are_canonical(K, N, tsz, D, i, d, keep):
    m = make_mps(K, N, tsz, D, i, 40 + i)
    res = truncate(m, m.psi, d, keep)
    bond = res["bond"]
    for qk, (qn, qt, dq) in enumerate(bond):
        acc = np.zeros((dq, dq))
        for (a, n), blk in res["site"].items():
            if d == +1:
                QN = ((0, 0), (1, 1), (1, -1), (2, 0))
                s = m.bonds[i][a]
                if (s[0] + QN[n][0], s[1] + QN[n][1]) == (qn, qt):
                    acc += blk.T @ blk
            elif a == qk:
                acc += blk @ blk.T
        assert np.max(np.abs(acc - np.eye(dq))) < 1e-12


def test_tie_rule_on_a_degenerate_spectrum():
    """Every sector carries singular values exactly 1: the selection fills
    the sectors in ascending quantum-number order."""
    m = make_mps(6, 6, 0, 16, 2, 3)
    secs = middle_sectors(m)
    psi = {k: np.zeros_like(v) for k, v in m.psi.items()}
    counts = []
    for q, (rows, cols) in secs.items():
        # an identity pattern on M_q: row t meets column t
        nr, nc = sum(r[2] for r in rows), sum(c[2] for c in cols)
        ro = 0
        for (li, n1, dl) in rows:
            co = 0
            for (n2, r, dr) in cols:
                blk = psi.get((li, n1, n2))
                if blk is not None:
                    for a in range(dl):
                        b = ro + a - co
                        if 0 <= b < dr:
                            blk[a, b] = 1.0
                co += dr
            ro += dl
        counts.append(min(nr, nc))
    keep = counts[0] + counts[1] // 2 + 1
    res = truncate(m, psi, +1, keep)
    kept = [k for (_, _, k) in res["sectors"]]
    assert kept[0] == counts[0]
    assert kept[1] == min(counts[1], keep - counts[0])
    assert sum(kept[2:]) == max(0, keep - counts[0] - counts[1])
    for (_, s, _) in res["sectors"]:
        assert np.allclose(s[:len(s)][s > 0.5], 1.0)


def test_planted_mistake_in_the_guess_is_caught():
    """Skipping the singular values in the carried-over guess (C = V^T
    instead of S V^T) breaks the projection property."""
    import oracle.truncation as tr
    m = make_mps(6, 6, 0, 16, 2, 42)
    good = tr.truncate(m, m.psi, +1, 9)
    real_svd = np.linalg.svd

    def no_s(M, full_matrices=False):
        U, s, Vt = real_svd(M, full_matrices=full_matrices)
        return U, np.ones_like(s) * (s > 0), Vt

    tr.np.linalg.svd = no_s
    try:
        bad = tr.truncate(m, m.psi, +1, 9)
    finally:
        tr.np.linalg.svd = real_svd
    v0 = psi_to_fock(m, m.psi)
    v1 = psi_to_fock(bad["mps"], bad["mps"].psi)
    assert abs((v0 - v1) @ (v0 - v1) - good["eps"]) > 1e-3


def test_stored_oracle_sigma_reproduces():
    """The stored oracle results of tests/golden/ (used by the GPU parity test
    at 22 and 36 orbitals) are the oracle's: one file recomputed here."""
    import os
    from oracle.blocksparse import BlockSparseSigma
    from synthetic import make_integrals, pack_psi
    path = os.path.join(os.path.dirname(__file__), "golden", "sigma_k22_n22_sz0_d48_w10.npz")
    z = np.load(path)
    K, N, tsz, D, i, iseed, mseed = (int(v) for v in z["case"])
    h, eri = make_integrals(K, iseed)
    m = make_mps(K, N, tsz, D, i, mseed)
    assert np.array_equal(pack_psi(m.bonds, i, m.psi), z["psi"])
    sig = pack_psi(m.bonds, i, BlockSparseSigma(m, h, eri).apply(m.psi))
    assert np.max(np.abs(sig - z["sigma"])) <= 1e-13 * np.max(np.abs(sig))
