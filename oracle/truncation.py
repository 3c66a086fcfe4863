"""Two-site truncation and window move (CPU, FP64) -- TEST INFRASTRUCTURE ONLY.

The Method section gives the MPS of eq. (1) with a bond dimension D and the
truncation error as the weight of the discarded Schmidt states; the
Numerical-procedure section runs the two-site algorithm at fixed D.  The
step written out here is the standard two-site update (White 1992; White
1996 for the guess carried into the next window):

* The optimised window psi of (i, i+1) is regrouped, for every quantum
  number q of the middle bond (q = Q_l + Q_n1), into the matrix
  M_q[(l, n1), (n2, r)] = psi[(l, n1, n2) -> r].
  Rows run over (l, n1) in ascending (l, n1), columns over (n2, r) in
  ascending (n2, r).
* Each M_q is decomposed by a plain SVD, M_q = U_q S_q V_q^T.
* Weights w = s^2 over all sectors are ranked, largest first; ties are
  broken by lower sector (ascending q), then lower in-sector index.  The
  first min(D, #candidates) are kept, where a candidate has
  w > max(cutoff, 1e-14) * w_max.
* The truncation error is eps = (sum of discarded w) / (sum of all w).
* Moving right (direction +1): the new left-canonical site tensor of site i
  is A[(l, n1) -> (q, k)] = U_q[(l, n1), k] for the kept k, and the guess for
  window (i+1, i+2) is
      psi'[((q, k), n2, n3) -> r'] = sum_r (S_q V_q^T)[k, (n2, r)] B_{i+2}[(r, n3) -> r'].
* Moving left (direction -1): the new right-canonical site tensor of site
  i+1 is B[(q, k) -> (n2, r)] = V_q^T[k, (n2, r)], and the guess for window
  (i-1, i) is
      psi'[(l', n0, n1) -> (q, k)] = sum_l A_{i-1}[(l', n0) -> l] (U_q S_q)[(l, n1), k].
* The new middle bond lists the sectors with at least one kept state, in
  ascending (N, 2Sz), with their kept counts as dimensions.

The layouts are those of ``synthetic.mps`` (site blocks (l, n) -> r with l at
the left bond; psi blocks (l, n1, n2) -> r).

Pins (tests/test_oracle_truncation.py): the singular values and eps equal
those of a dense SVD of the unblocked two-site matrix; at K <= 6 they equal
the Schmidt values of the full Fock vector at the cut; the moved state's
Fock vector is the orthogonal projection of the original one with squared
distance eps (Eckart-Young); keeping every state reproduces the original
Fock vector; the new tensors are left/right canonical; the tie rule holds on
an exactly degenerate spectrum.
"""
from dataclasses import replace

import numpy as np

_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _add(q, n):
    return (q[0] + _QN[n][0], q[1] + _QN[n][1])


def middle_sectors(mps):
    """{q: (rows, cols)} of the window's regrouped matrices M_q.

    rows: list of (l, n1, d_l) in ascending (l, n1); cols: list of
    (n2, r, d_r) in ascending (n2, r).  Only q with at least one row and one
    column appear."""
    i = mps.window
    bl, br = mps.bonds[i], mps.bonds[i + 2]
    ridx = {(s[0], s[1]): k for k, s in enumerate(br)}
    out = {}
    for li, sl in enumerate(bl):
        for n1 in range(4):
            q = _add((sl[0], sl[1]), n1)
            cols = []
            for n2 in range(4):
                rq = _add(q, n2)
                if rq in ridx:
                    r = ridx[rq]
                    cols.append((n2, r, br[r][2]))
            if not cols:
                continue
            rows, _ = out.setdefault(q, ([], cols))
            rows.append((li, n1, sl[2]))
    return {q: out[q] for q in sorted(out)}


def regroup(mps, psi, q, rows, cols):
    """M_q assembled block by block from psi."""
    M = np.zeros((sum(r[2] for r in rows), sum(c[2] for c in cols)))
    ro = 0
    for (li, n1, dl) in rows:
        co = 0
        for (n2, r, dr) in cols:
            blk = psi.get((li, n1, n2))
            if blk is not None:
                M[ro:ro + dl, co:co + dr] = blk
            co += dr
        ro += dl
    return M


def truncate(mps, psi, direction, max_bond_dim, cutoff=0.0):
    """One two-site truncation and window move (see the module docstring).

    mps: a synthetic.mps.RandomMPS whose window is (i, i+1) (its own psi is
    not used); psi: the optimised window blocks.  Returns a dict with
      eps        discarded weight / total weight
      sectors    [(q, singular values descending, kept count)] in ascending q
      bond       new middle bond [(N, 2Sz, kept)]
      site       new site tensor blocks (site i for +1, site i+1 for -1)
      psi        guess for the new window
      mps        a RandomMPS at the new window carrying the new bond, the new
                 site tensor and psi' (the other tensors shared with the input)
    """
    if direction not in (1, -1):
        raise ValueError("direction must be +1 or -1")
    i, K = mps.window, mps.n_orb
    if direction == 1 and i + 1 > K - 2:
        raise ValueError("cannot move right from the last window")
    if direction == -1 and i == 0:
        raise ValueError("cannot move left from the first window")
    secs = middle_sectors(mps)
    dec = {}
    cand = []  # (weight, sector rank, in-sector index)
    for rank, (q, (rows, cols)) in enumerate(secs.items()):
        M = regroup(mps, psi, q, rows, cols)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        dec[q] = (U, s, Vt, rows, cols)
        for j, sv in enumerate(s):
            cand.append((sv * sv, rank, j))
    total = sum(c[0] for c in cand)
    if total <= 0:
        raise ValueError("psi is zero")
    wmax = max(c[0] for c in cand)
    cand.sort(key=lambda c: (-c[0], c[1], c[2]))
    thresh = max(cutoff, 1e-14) * wmax
    keep = [c for c in cand if c[0] > thresh][:max_bond_dim]
    qs = list(secs)
    kept = {q: 0 for q in qs}
    for (_, rank, j) in keep:
        kept[qs[rank]] += 1
    # the kept states of a sector are its leading singular vectors (the
    # ranking within a sector follows the descending singular values)
    eps = max(0.0, (total - sum(c[0] for c in keep)) / total)
    new_bond = [(q[0], q[1], kept[q]) for q in qs if kept[q] > 0]
    sectors = [(q, dec[q][1].copy(), kept[q]) for q in qs]
    bidx = {(b[0], b[1]): k for k, b in enumerate(new_bond)}
    site, nxt = {}, {}
    if direction == 1:
        for q in qs:
            U, s, Vt, rows, cols = dec[q]
            k = kept[q]
            if k == 0:
                continue
            ro = 0
            for (li, n1, dl) in rows:
                site[(li, n1)] = U[ro:ro + dl, :k].copy()
                ro += dl
        # psi' on window (i+1, i+2): C_q = S V^T (kept rows) contracted with B_{i+2}
        b3 = mps.bonds[i + 3]
        r3 = {(s_[0], s_[1]): k for k, s_ in enumerate(b3)}
        B = mps.sites[i + 2]
        for qk, (qn, qt, dq) in enumerate(new_bond):
            q = (qn, qt)
            U, s, Vt, rows, cols = dec[q]
            C = (s[:dq, None] * Vt[:dq, :])
            co = 0
            for (n2, r, dr) in cols:
                Cr = C[:, co:co + dr]
                co += dr
                for n3 in range(4):
                    blk = B.get((r, n3))
                    if blk is None:
                        continue
                    rq = _add(_add(q, n2), n3)
                    rp = r3[rq]
                    key = (qk, n2, n3)
                    nxt[key] = nxt.get(key, np.zeros((dq, b3[rp][2]))) + Cr @ blk
        new_bonds = list(mps.bonds)
        new_bonds[i + 1] = new_bond
        sites = list(mps.sites)
        sites[i] = site
        sites[i + 1] = None
        sites[i + 2] = None
        moved = replace(mps, window=i + 1, bonds=new_bonds, sites=sites, psi=nxt)
    else:
        br = mps.bonds[i + 2]
        for qk, (qn, qt, dq) in enumerate(new_bond):
            q = (qn, qt)
            U, s, Vt, rows, cols = dec[q]
            co = 0
            for (n2, r, dr) in cols:
                site[(qk, n2)] = Vt[:dq, co:co + dr].copy()
                co += dr
        # psi' on window (i-1, i): A_{i-1} contracted with C_q = U S (kept columns)
        b0, bl = mps.bonds[i - 1], mps.bonds[i]
        A = mps.sites[i - 1]
        for qk, (qn, qt, dq) in enumerate(new_bond):
            q = (qn, qt)
            U, s, Vt, rows, cols = dec[q]
            C = U[:, :dq] * s[None, :dq]
            ro = 0
            for (li, n1, dl) in rows:
                Cl = C[ro:ro + dl, :]
                ro += dl
                for lp, sp in enumerate(b0):
                    for n0 in range(4):
                        blk = A.get((lp, n0))
                        if blk is None or _add((sp[0], sp[1]), n0) != (bl[li][0], bl[li][1]):
                            continue
                        key = (lp, n0, n1)
                        nxt[key] = nxt.get(key, np.zeros((sp[2], dq))) + blk @ Cl
        new_bonds = list(mps.bonds)
        new_bonds[i + 1] = new_bond
        sites = list(mps.sites)
        sites[i + 1] = site
        sites[i - 1] = None
        sites[i] = None
        moved = replace(mps, window=i - 1, bonds=new_bonds, sites=sites, psi=nxt)
    # every allowed block of the new window, zero where nothing contributed
    full = {}
    j = moved.window
    lb, rb = moved.bonds[j], moved.bonds[j + 2]
    ridx = {(s_[0], s_[1]): k for k, s_ in enumerate(rb)}
    for li, sl in enumerate(lb):
        for n1 in range(4):
            for n2 in range(4):
                rq = _add(_add((sl[0], sl[1]), n1), n2)
                if rq in ridx:
                    full[(li, n1, n2)] = nxt.get((li, n1, n2), np.zeros((sl[2], rb[ridx[rq]][2])))
    moved = replace(moved, psi=full)
    return {"eps": eps, "sectors": sectors, "bond": new_bond, "site": site, "psi": full,
            "mps": moved}
