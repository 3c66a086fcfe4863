"""Seeded synthetic inputs for the spin-adapted contraction: multiplet
sectors (N, 2S, dimension) of a two-block window, random reduced blocks of
tensor operators, and the packed layout of the window vector (blocks by
left then right sector, each row-major).  Holds none of the method's
arithmetic: the only rules here are the particle-number and angular-momentum
triangle conditions that say which blocks exist."""
import numpy as np


def _tri(a, b, c):
    return abs(a - b) <= c <= a + b and (a + b + c) % 2 == 0


def sector_window(n, tS, dmax, rng):
    """Left and right sectors (N, 2S, d) around n/2 electrons a side, with
    dimensions drawn up to dmax (largest near the middle N and low spin)."""
    def side():
        out = []
        for N in range(max(0, n // 2 - 3), n // 2 + 4):
            for ts in range(N % 2, N % 2 + 7, 2):
                if ts > N + 2:
                    continue
                d = int(rng.integers(1, dmax + 1) * (1.0 if ts <= 2 else 0.5)) or 1
                out.append((N, ts, d))
        return out
    return side(), side()


def random_operator(sectors, dn, tk, rng, keep=0.8):
    """Reduced blocks {(out sector, in sector): d_out x d_in} of a rank-k
    tensor operator with particle change dn; each allowed block kept with
    probability keep."""
    op = {}
    for i2, (n2, s2, d2) in enumerate(sectors):
        for i, (n1, s1, d1) in enumerate(sectors):
            if n2 == n1 + dn and _tri(s1, tk, s2) and rng.random() < keep:
                op[(i2, i)] = rng.normal(size=(d2, d1))
    return op


def _blocks(lsec, rsec, n, tS):
    return [(a, b) for a, (na, sa, _) in enumerate(lsec) for b, (nb, sb, _) in enumerate(rsec)
            if na + nb == n and _tri(sa, sb, tS)]


def unpack(lsec, rsec, n, tS, flat):
    """Packed vector (blocks by left then right sector, each row-major) to
    a dict of blocks."""
    out, off = {}, 0
    for a, b in _blocks(lsec, rsec, n, tS):
        da, db = lsec[a][2], rsec[b][2]
        out[(a, b)] = np.asarray(flat[off:off + da * db]).reshape(da, db)
        off += da * db
    assert off == len(flat)
    return out


def pack(lsec, rsec, n, tS, blocks):
    parts = [blocks[k].ravel() for k in _blocks(lsec, rsec, n, tS)]
    return np.concatenate(parts) if parts else np.zeros(0)


def operator_layout(sectors, dn, tk):
    """Every allowed reduced block of a rank-k operator with particle change
    dn, as (out sector, in sector, element offset) in a packed row-major
    array, and the array's length."""
    blocks, off = [], 0
    for i2, (n2, s2, d2) in enumerate(sectors):
        for i, (n1, s1, d1) in enumerate(sectors):
            if n2 == n1 + dn and _tri(s1, tk, s2):
                blocks.append((i2, i, off))
                off += d2 * d1
    return blocks, off


def multiplet_sectors(n_center, two_s_max, dim_total, width, rng):
    """Multiplet sectors (N, 2S, d) of one block at a bipartition: N within
    3 width of n_center, 2S from N's parity up to two_s_max, dimensions
    proportional to a Gaussian in N times (2S + 1) exp(-2S / 4) with a
    random factor in [0.7, 1.3], rounded, summing to dim_total."""
    lo, hi = int(np.floor(n_center - 3 * width)), int(np.ceil(n_center + 3 * width))
    keys, w = [], []
    for N in range(max(0, lo), hi + 1):
        for ts in range(N % 2, min(two_s_max, N) + 1, 2):
            keys.append((N, ts))
            w.append(np.exp(-0.5 * ((N - n_center) / width) ** 2) * (ts + 1) * np.exp(-ts / 4.0)
                     * rng.uniform(0.7, 1.3))
    w = np.asarray(w) / np.sum(w)
    d = np.maximum(1, np.floor(w * dim_total)).astype(int)
    order = np.argsort(-w)
    k = 0
    while d.sum() < dim_total:
        d[order[k % len(d)]] += 1
        k += 1
    while d.sum() > dim_total:
        j = order[k % len(d)]
        if d[j] > 1:
            d[j] -= 1
        k += 1
    return [(N, ts, int(x)) for (N, ts), x in zip(keys, d)]


def cas89_102_window(rng, dim=2048):
    """The spin-adapted middle bipartition of a CAS(89,102)-shaped active
    space with total spin S = 5/2: two 51-orbital blocks of dim multiplets
    each, centred on 44 and 45 electrons (44.5 each side on average)."""
    left = multiplet_sectors(44.5, 9, dim, 2.0, rng)
    right = multiplet_sectors(44.5, 9, dim, 2.0, rng)
    return left, right, 89, 5


def hamiltonian_pair_types(n_left_orb, n_right_orb):
    """Operator pair types of the spin-adapted sigma at a bipartition, as
    (count, left particle change, rank 2k, right particle change, right
    parity): the two block Hamiltonians, the one-index pairs (a creator or
    annihilator of one side with its complementary operator on the other,
    rank 1/2), and the two-index pairs A_pq P_pq and B_pq Q_pq of the left
    orbitals with ranks 0 and 1 (normal operators on the left, complementary
    ones on the right)."""
    n_ab = n_left_orb * (n_left_orb + 1) // 2  # p <= q: rank 0
    n_ab1 = n_left_orb * (n_left_orb - 1) // 2  # p < q: rank 1
    nb = n_left_orb * n_left_orb
    return [
        (1, 0, 0, 0, 0), (1, 0, 0, 0, 0),  # H_L x 1, 1 x H_R
        (n_left_orb, 1, 1, -1, 1), (n_left_orb, -1, 1, 1, 1),
        (n_right_orb, 1, 1, -1, 1), (n_right_orb, -1, 1, 1, 1),
        (n_ab, 2, 0, -2, 0), (n_ab, -2, 0, 2, 0), (n_ab1, 2, 2, -2, 0), (n_ab1, -2, 2, 2, 0),
        (nb, 0, 0, 0, 0), (nb, 0, 2, 0, 0),
    ]


def cas89_102_workload(seed=102, dim=2048, device="cuda"):
    """The CAS(89,102)-shaped spin-adapted sigma workload on the device:
    sectors of both 51-orbital blocks, one left and one right operator per
    pair of hamiltonian_pair_types with every allowed block filled by
    normal random numbers (one float64 tensor per side, drawn by a seeded
    torch generator on the device), pair coefficients from N(0, 1) and a
    random window vector.  Returns a dict with the sectors, n, 2S, the
    operator lists in the (blocks, data, base) form of the binding, their
    layouts, the pairs and psi."""
    import torch
    rng = np.random.default_rng(seed)
    lsec, rsec, n, tS = cas89_102_window(rng, dim)
    lay_l, lay_r, pairs = [], [], []
    for count, dnl, tk, dnr, par in hamiltonian_pair_types(51, 51):
        bl, sl = operator_layout(lsec, dnl, tk)
        br, sr = operator_layout(rsec, dnr, tk)
        for _ in range(count):
            pairs.append((len(lay_l), len(lay_r), tk, par, float(rng.normal())))
            lay_l.append((bl, sl))
            lay_r.append((br, sr))
    g = torch.Generator(device=device)
    g.manual_seed(seed)

    def side(lay):
        bases = np.concatenate([[0], np.cumsum([s for _, s in lay])])
        data = torch.randn(int(bases[-1]), dtype=torch.float64, device=device, generator=g)
        return [(b, data, int(bases[i])) for i, (b, _) in enumerate(lay)], data

    left_ops, ldata = side(lay_l)
    right_ops, rdata = side(lay_r)
    size = sum(lsec[a][2] * rsec[b][2] for a, b in _blocks(lsec, rsec, n, tS))
    psi = torch.randn(size, dtype=torch.float64, device=device, generator=g)
    return {"left_sectors": lsec, "right_sectors": rsec, "n": n, "two_s": tS, "left_ops": left_ops,
            "right_ops": right_ops, "pairs": pairs, "psi": psi, "left_data": ldata, "right_data": rdata}
