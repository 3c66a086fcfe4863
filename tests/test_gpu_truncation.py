"""Two-site truncation and window move of the library against the oracle (GPU).

dmrg_truncate keeps the D largest reduced-density-matrix weights over all
middle-bond sectors and moves the window; the oracle does the same with a
per-sector SVD (oracle/truncation.py, pinned on the CPU by a dense SVD, the
Fock-space Schmidt values and Eckart-Young).  Compared here, at bond
dimensions that truncate, in both directions and at 2S_z != 0:

* the truncation error (discarded weight / total weight), to 1e-10 of the
  total weight;
* the new middle bond: its sectors and their kept dimensions, exactly;
* the updated site tensor out of the library (dmrg_get_site): canonical to
  1e-12, and its per-sector projector U U^T (gauge invariant) equal to the
  oracle's to 1e-9;
* the moved state: the Fock vector of the library's new MPS (its site
  tensor, bond and carried-over window vector from dmrg_get_psi) equals the
  oracle's element by element to 1e-10 (the projection of the original state
  onto the kept space is unique when the weights at the cut are not
  degenerate, which each case checks first).
Site tensors themselves are gauge dependent and are never compared
element by element.
"""
from dataclasses import replace

import numpy as np
import pytest

from synthetic import pack_psi, unpack_psi
from tests.helpers import case, lib_load

pytestmark = pytest.mark.gpu

CASES = [  # K, N, 2Sz, D of the MPS, window, direction, kept D
    (8, 8, 0, 20, 3, +1, 12), (8, 8, 0, 20, 3, -1, 12),
    (8, 8, 2, 24, 2, +1, 10), (8, 7, -1, 24, 4, -1, 9),
    (10, 10, 2, 30, 4, +1, 16), (10, 10, 0, 30, 5, -1, 20),
    (8, 8, 0, 20, 3, +1, 400),  # keeps everything: error 0, state unchanged
]


def _site_blocks(bonds, b, flat):
    """Unpack a packed site tensor into {(l, n): block}."""
    from synthetic.mps import site_block_list
    out, off = {}, 0
    for (li, n, ri, dl, dr) in site_block_list(bonds, b):
        out[(li, n)] = flat[off:off + dl * dr].reshape(dl, dr)
        off += dl * dr
    assert off == flat.size
    return out


def _projectors(bonds, b, blocks, side):
    """Per new-bond sector: the projector onto the kept space (U U^T for a
    left-canonical tensor over rows (l, n); V^T V over columns (n, r) for a
    right-canonical one)."""
    QN = ((0, 0), (1, 1), (1, -1), (2, 0))
    if side > 0:
        left, right = bonds[b], bonds[b + 1]
        out = {}
        for ri, sr in enumerate(right):
            rows = [blocks[(li, n)] for li, sl in enumerate(left) for n in range(4)
                    if (sl[0] + QN[n][0], sl[1] + QN[n][1]) == (sr[0], sr[1]) and (li, n) in blocks]
            U = np.vstack(rows)
            out[(sr[0], sr[1])] = U @ U.T
        return out
    left, right = bonds[b], bonds[b + 1]
    ridx = {(s[0], s[1]): k for k, s in enumerate(right)}
    out = {}
    for li, sl in enumerate(left):
        cols = []
        for n in range(4):
            q = (sl[0] + QN[n][0], sl[1] + QN[n][1])
            if q in ridx and (li, n) in blocks:
                cols.append(blocks[(li, n)])
        V = np.hstack(cols)
        out[(sl[0], sl[1])] = V.T @ V
    return out


@pytest.mark.parametrize("K,N,tsz,D,i,d,keep", CASES)
def test_truncation_matches_oracle(ctx, K, N, tsz, D, i, d, keep):
    import torch
    from oracle.projection import psi_to_fock
    from oracle.truncation import truncate
    print(f"truncation: K={K} N={N} 2Sz={tsz} D={D} window={i} direction={d:+d} keep={keep}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = truncate(m, m.psi, d, keep)
    w = np.sort(np.concatenate([s * s for (_, s, _) in ref["sectors"]]))[::-1]
    kept = sum(b[2] for b in ref["bond"])
    if kept < len(w):
        gap = (w[kept - 1] - w[kept]) / w[0]
        print(f"  relative weight gap at the cut {gap:.2e}", flush=True)
        assert gap > 1e-6, "degenerate cut: pick another case"
    lib_load(ctx, h, eri, m)
    psi = torch.from_numpy(pack_psi(m.bonds, i, m.psi)).cuda()
    eps, kept_lib = ctx.truncate(psi, d, keep)
    print(f"  eps library {eps:.6e} oracle {ref['eps']:.6e}; kept {kept_lib} / {kept}", flush=True)
    assert abs(eps - ref["eps"]) <= 1e-10
    assert kept_lib == kept
    j = i + d
    nb = ctx.get_bond(i + 1)
    assert nb == [tuple(b) for b in ref["bond"]]
    # the updated site tensor
    s = i if d > 0 else i + 1
    bonds = list(ref["mps"].bonds)
    site = _site_blocks(bonds, s, ctx.get_site(s))
    P_lib = _projectors(bonds, s, site, d)
    P_ref = _projectors(bonds, s, ref["site"], d)
    assert set(P_lib) == set(P_ref)
    for q in P_ref:
        A = P_lib[q]
        tr = np.trace(A)
        assert abs(tr - round(tr)) < 1e-12 and abs(np.trace(A @ A) - tr) < 1e-10  # canonical
        assert np.max(np.abs(A - P_ref[q])) < 1e-9, q
    # the moved state
    ctx.build_ops(j, d)
    nxt = torch.empty(ctx.psi_size(), dtype=torch.float64, device="cuda")
    ctx.get_psi(nxt)
    torch.cuda.synchronize()
    sites = list(ref["mps"].sites)
    sites[s] = site
    moved = replace(ref["mps"], sites=sites, psi=unpack_psi(bonds, j, nxt.cpu().numpy()))
    f_lib = psi_to_fock(moved, moved.psi)
    f_ref = psi_to_fock(ref["mps"], ref["psi"])
    f_old = psi_to_fock(m, m.psi)
    err = float(np.max(np.abs(f_lib - f_ref)))
    print(f"  moved state: max |lib - oracle| = {err:.2e}; "
          f"|psi - moved|^2 / |psi|^2 = {np.sum((f_old - f_lib) ** 2) / np.sum(f_old ** 2):.6e}", flush=True)
    assert err <= 1e-10 * float(np.max(np.abs(f_ref)))
    if keep >= 400:
        assert eps == 0.0 or eps < 1e-14
        assert np.max(np.abs(f_lib - f_old)) <= 1e-10 * float(np.max(np.abs(f_old)))


def test_truncation_of_a_ground_state(ctx):
    """The same comparison on a Davidson ground state (fast-decaying weights)."""
    import torch
    from oracle.truncation import truncate
    print("truncation of a ground state: K=8 N=8 D=64 window 3, keep 24", flush=True)
    h, eri, m = case(8, 8, 0, 64, 3)
    lib_load(ctx, h, eri, m)
    psi = torch.from_numpy(pack_psi(m.bonds, 3, m.psi)).cuda()
    ctx.davidson(psi, tol=1e-8)
    gs = unpack_psi(m.bonds, 3, psi.cpu().numpy())
    ref = truncate(m, gs, +1, 24)
    eps, kept = ctx.truncate(psi, +1, 24)
    print(f"  eps library {eps:.6e} oracle {ref['eps']:.6e}", flush=True)
    assert kept == sum(b[2] for b in ref["bond"])
    assert abs(eps - ref["eps"]) <= 1e-10 * max(1.0, ref["eps"]) + 1e-13
    assert ctx.get_bond(4) == [tuple(b) for b in ref["bond"]]
