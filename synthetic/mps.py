"""Seeded random U(1) block-sparse MPS with a two-site window.

Exchange format (the same one the C-ABI library reads):

* Sites 0..K-1, one spatial orbital each, local basis |0>, |up>, |dn>, |updn>
  (indices 0..3) carrying (N, 2Sz) = (0,0), (1,+1), (1,-1), (2,0).
* Bond b (0..K) sits left of site b.  A bond sector is labelled by the
  quantum numbers (N, 2Sz) of the LEFT part (sites 0..b-1); sectors of a bond
  are sorted ascending by (N, 2Sz).  Bond 0 is the vacuum (0,0) of dim 1 and
  bond K is (N_tot, 2Sz_tot) of dim 1.
* Site tensor b has blocks (l, n) -> r with Q_l + Q_n = Q_r (l a sector of
  bond b, r a sector of bond b+1).  Packed order: l ascending, then n
  ascending; each block is row-major d_l x d_r.  Blocks whose r sector does
  not exist are absent.
* The two-site wavefunction of window (i, i+1) has blocks (l, n1, n2) -> r
  (l at bond i, r at bond i+2) with Q_l + Q_n1 + Q_n2 = Q_r, packed
  right-sector-major: ascending r, then ascending (l, n1, n2); each block is
  row-major d_l x d_r, so the blocks of one r stack into a dense matrix.
* Sites left of the window are left-canonical (sum_{l,n} A^T A = 1), sites
  right of it right-canonical (sum_{n,r} B B^T = 1).

Sector sizes follow a "converged-like" recipe: at a bond with b orbitals on
the left, sector (N_L, 2Sz_L) gets weight
exp(-(N_L - N b/K)^2/(2*1.5^2) - (2Sz_L - 2Sz b/K)^2/(2*2.0^2)),
dims are D*w/sum(w) capped by the exact dimension min(left, right Fock
sector size), sectors below 8 are dropped unless at their cap, and the
remainder goes to the largest sectors.  Dims are then clipped so every
canonical tensor can be an isometry.  Tensors are random N(0,1) blocks made
orthonormal by QR; psi is N(0,1) on its allowed blocks, normalised.

Only random numbers and layout live here: no Hamiltonian arithmetic.
"""
from dataclasses import dataclass, field
from math import comb

import numpy as np

SITE_QN = ((0, 0), (1, 1), (1, -1), (2, 0))


def _space_dim(norb, n, tsz):
    if n < 0 or (n + tsz) % 2:
        return 0
    na, nb = (n + tsz) // 2, (n - tsz) // 2
    if na < 0 or nb < 0 or na > norb or nb > norb:
        return 0
    return comb(norb, na) * comb(norb, nb)


def _allowed(K, N, tsz, b):
    """Left-part quantum numbers allowed at bond b with their exact caps."""
    out = {}
    for nl in range(0, min(2 * b, N) + 1):
        for tl in range(-nl, nl + 1, 2):
            dl = _space_dim(b, nl, tl)
            dr = _space_dim(K - b, N - nl, tsz - tl)
            if dl and dr:
                out[(nl, tl)] = min(dl, dr)
    return out


def _target_dims(K, N, tsz, b, D, limit=None):
    caps = _allowed(K, N, tsz, b)
    if limit is not None:  # only sectors reachable from the neighbouring bond
        caps = {q: min(c, limit.get(q, 0)) for q, c in caps.items()}
        caps = {q: c for q, c in caps.items() if c > 0}
    if not caps:
        return {}
    total_cap = sum(caps.values())
    if total_cap <= D:
        return dict(caps)
    keys = sorted(caps)
    w = np.array([np.exp(-(q[0] - N * b / K) ** 2 / (2 * 1.5 ** 2)
                         - (q[1] - tsz * b / K) ** 2 / (2 * 2.0 ** 2)) for q in keys])
    w = w / w.sum()
    d = {q: min(caps[q], int(round(D * wi))) for q, wi in zip(keys, w)}
    d = {q: v for q, v in d.items() if v >= 8 or v == caps[q]}
    if not d:  # keep the heaviest sector at least
        q = keys[int(np.argmax(w))]
        d = {q: min(caps[q], D)}
    order = sorted(d, key=lambda q: (-d[q], q))
    rem = D - sum(d.values())
    while rem > 0:
        grew = False
        for q in order:
            if rem == 0:
                break
            if d[q] < caps[q]:
                d[q] += 1
                rem -= 1
                grew = True
        if not grew:
            break
    # small D: kept sectors are at their caps; re-admit dropped ones by weight
    for q, wi in sorted(zip(keys, w), key=lambda t: (-t[1], t[0])):
        if rem <= 0:
            break
        if q not in d:
            d[q] = min(caps[q], rem)
            rem -= d[q]
            order.append(q)
    while rem < 0:  # rounding overshoot: trim the largest sectors
        for q in order:
            if rem == 0:
                break
            if d[q] > 1:
                d[q] -= 1
                rem += 1
    return d


def _add(q, n):
    return (q[0] + SITE_QN[n][0], q[1] + SITE_QN[n][1])


@dataclass
class RandomMPS:
    n_orb: int
    n_elec: int
    two_sz: int
    window: int
    bonds: list            # K+1 lists of (N, 2Sz, dim)
    sites: list            # K entries: dict {(l, n): block} or None inside the window
    psi: dict              # {(l, n1, n2): block}
    extras: dict = field(default_factory=dict)

    def bond_index(self, b):
        return {(s[0], s[1]): k for k, s in enumerate(self.bonds[b])}

    def psi_size(self):
        return int(sum(v.size for v in self.psi.values()))


def site_block_list(bonds, b):
    """Packed block order of site tensor b: list of (l, n, r, d_l, d_r)."""
    left, right = bonds[b], bonds[b + 1]
    ridx = {(s[0], s[1]): k for k, s in enumerate(right)}
    out = []
    for li, sl in enumerate(left):
        for n in range(4):
            q = _add((sl[0], sl[1]), n)
            if q in ridx:
                ri = ridx[q]
                out.append((li, n, ri, sl[2], right[ri][2]))
    return out


def psi_block_list(bonds, i):
    """Packed block order of the two-site psi at window (i, i+1)."""
    left, right = bonds[i], bonds[i + 2]
    ridx = {(s[0], s[1]): k for k, s in enumerate(right)}
    out = []
    for li, sl in enumerate(left):
        for n1 in range(4):
            for n2 in range(4):
                q = _add(_add((sl[0], sl[1]), n1), n2)
                if q in ridx:
                    ri = ridx[q]
                    out.append((li, n1, n2, ri, sl[2], right[ri][2]))
    out.sort(key=lambda t: (t[3], t[0], t[1], t[2]))
    return out


def mps_arrays(mps):
    """Flat arrays of the exchange format (bond offsets, sectors, site data)."""
    K = mps.n_orb
    offs, sn, ss, sd = [0], [], [], []
    for b in range(K + 1):
        for (n, t, d) in mps.bonds[b]:
            sn.append(n)
            ss.append(t)
            sd.append(d)
        offs.append(len(sn))
    sites = []
    for b in range(K):
        if mps.sites[b] is None:
            sites.append(None)
        else:
            sites.append(np.ascontiguousarray(pack_site(mps.bonds, b, mps.sites[b])))
    return {"bond_offsets": np.array(offs, dtype=np.int32),
            "sector_n": np.array(sn, dtype=np.int32),
            "sector_2sz": np.array(ss, dtype=np.int32),
            "sector_dim": np.array(sd, dtype=np.int32),
            "sites": sites}


def pack_site(bonds, b, blocks):
    parts = [np.ascontiguousarray(blocks[(li, n)], dtype=np.float64).ravel()
             for (li, n, ri, dl, dr) in site_block_list(bonds, b)]
    return np.concatenate(parts) if parts else np.zeros(0)


def pack_psi(bonds, i, psi):
    parts = [np.ascontiguousarray(psi[(li, n1, n2)], dtype=np.float64).ravel()
             for (li, n1, n2, ri, dl, dr) in psi_block_list(bonds, i)]
    return np.concatenate(parts) if parts else np.zeros(0)


def unpack_psi(bonds, i, flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for (li, n1, n2, ri, dl, dr) in psi_block_list(bonds, i):
        out[(li, n1, n2)] = flat[off:off + dl * dr].reshape(dl, dr).copy()
        off += dl * dr
    assert off == flat.size, (off, flat.size)
    return out


def _bond_structure(K, N, tsz, D, window):
    dims = [dict() for _ in range(K + 1)]
    dims[0] = {(0, 0): 1}
    dims[K] = {(N, tsz): 1}

    def from_left(prev):
        avail = {}
        for q, d in prev.items():
            for n in range(4):
                qq = _add(q, n)
                avail[qq] = avail.get(qq, 0) + d
        return avail

    def from_right(nxt, b):
        avail = {}
        for q in _allowed(K, N, tsz, b):
            avail[q] = sum(nxt.get(_add(q, n), 0) for n in range(4))
        return avail

    # left-canonical sites 0..window-1 feed bonds 1..window
    for b in range(1, window + 1):
        dims[b] = _target_dims(K, N, tsz, b, D, from_left(dims[b - 1]))
    # right-canonical sites K-1..window+2 feed bonds K-1..window+2
    for b in range(K - 1, window + 1, -1):
        dims[b] = _target_dims(K, N, tsz, b, D, from_right(dims[b + 1], b))
    # the bond inside the window: bounded from both sides
    b = window + 1
    if 0 < b < K:
        la, ra = from_left(dims[b - 1]), from_right(dims[b + 1], b)
        dims[b] = _target_dims(K, N, tsz, b, D, {q: min(la.get(q, 0), ra.get(q, 0)) for q in la})
    return [[(q[0], q[1], dims[b][q]) for q in sorted(dims[b])] for b in range(K + 1)]


def make_mps(n_orb, n_elec, two_sz, D, window, seed):
    """Random MPS for window (window, window+1); see the module docstring."""
    K, N, tsz = int(n_orb), int(n_elec), int(two_sz)
    if not (0 <= window <= K - 2):
        raise ValueError("window must satisfy 0 <= i <= K-2")
    if N < 0 or N > 2 * K or abs(tsz) > min(N, 2 * K - N) or (N - tsz) % 2:
        raise ValueError("invalid (N, 2Sz) for K orbitals")
    bonds = _bond_structure(K, N, tsz, D, window)
    rng = np.random.default_rng(seed)
    sites = [None] * K
    for b in range(K):
        if b in (window, window + 1):
            continue
        left, right = bonds[b], bonds[b + 1]
        blocks = {}
        if b < window:  # left-canonical: columns per right sector orthonormal
            for ri, sr in enumerate(right):
                rows = []
                for li, sl in enumerate(left):
                    for n in range(4):
                        if _add((sl[0], sl[1]), n) == (sr[0], sr[1]):
                            rows.append((li, n, sl[2]))
                tot = sum(r[2] for r in rows)
                X = rng.normal(size=(tot, sr[2]))
                Q, _ = np.linalg.qr(X)
                off = 0
                for (li, n, dl) in rows:
                    blocks[(li, n)] = Q[off:off + dl, :].copy()
                    off += dl
        else:  # right-canonical: rows per left sector orthonormal
            for li, sl in enumerate(left):
                cols = []
                for n in range(4):
                    q = _add((sl[0], sl[1]), n)
                    for ri, sr in enumerate(right):
                        if (sr[0], sr[1]) == q:
                            cols.append((n, ri, sr[2]))
                tot = sum(c[2] for c in cols)
                X = rng.normal(size=(sl[2], tot))
                Q, _ = np.linalg.qr(X.T)
                Qt = Q.T
                off = 0
                for (n, ri, dr) in cols:
                    blocks[(li, n)] = Qt[:, off:off + dr].copy()
                    off += dr
        sites[b] = blocks
    psi = {}
    for (li, n1, n2, ri, dl, dr) in psi_block_list(bonds, window):
        psi[(li, n1, n2)] = rng.normal(size=(dl, dr))
    nrm = np.sqrt(sum(float(np.sum(v * v)) for v in psi.values()))
    for k in psi:
        psi[k] /= nrm
    return RandomMPS(K, N, tsz, window, bonds, sites, psi)
