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
