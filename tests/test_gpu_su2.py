"""Spin-adapted contraction of the HIP library (dmrg_su2_sigma) against the
oracle's block-by-block rule (GPU).

oracle.su2.contract_scalar_products is pinned on the CPU against the scalar
products built component by component on the Fock space; here random
reduced operators on synthetic multiplet sectors (dimensions that span
several 128-row tiles with ragged tails, blocks missing at random, right
operators shared by several pairs) are contracted by both.  Bar: every
element within 1e-10 * max|sigma| (FP64 arithmetic, rounding only).
"""
import numpy as np
import pytest

from oracle import su2
from synthetic.su2 import sector_window, random_operator, pack, unpack

pytestmark = pytest.mark.gpu

TOL = 1e-10


def run(ctx, lsec, rsec, n, tS, lops, rops, pairs, psi_flat):
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    def ops(lst):
        out = []
        for o in lst:
            blocks, data = pack_blocks(o)
            out.append((blocks, dev(data)))
        return out
    left, right = ops(lops), ops(rops)
    psi = dev(psi_flat)
    out = torch.full_like(psi, float("nan"))
    ctx.su2_sigma(lsec, rsec, n, tS, left, right, [(l, r, tk, pb, c) for l, r, tk, pb, c in pairs], psi, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def pack_blocks(op):
    """(block list [(out, in, element offset)], concatenated row-major data)."""
    blocks, parts, off = [], [], 0
    for (i2, i), t in sorted(op.items()):
        blocks.append((i2, i, off))
        parts.append(t.ravel())
        off += t.size
    return blocks, (np.concatenate(parts) if parts else np.zeros(1))


def oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, psi_flat):
    psi = unpack(lsec, rsec, n, tS, psi_flat)
    got = su2.contract_scalar_products(lsec, rsec, n, tS, psi,
                                       [(c, tk, pb, lops[l], rops[r]) for l, r, tk, pb, c in pairs])
    return pack(lsec, rsec, n, tS, got)


CASES = [  # n, 2S, largest sector dimension, seed
    (8, 0, 40, 1),
    (9, 1, 150, 2),
    (10, 2, 300, 3),
    (12, 0, 260, 4),
    (11, 3, 90, 5),
]


@pytest.mark.parametrize("n,tS,dmax,seed", CASES)
def test_su2_sigma_matches_the_oracle(ctx, n, tS, dmax, seed):
    print(f"su2 sigma: n={n} 2S={tS} dmax={dmax} seed={seed}", flush=True)
    rng = np.random.default_rng(seed)
    lsec, rsec = sector_window(n, tS, dmax, rng)
    lops, rops, pairs = [], [], []
    for dn, tk in [(0, 0), (0, 2), (1, 1), (-1, 1), (2, 0), (-2, 2), (1, 3)]:
        rops.append(random_operator(rsec, -dn, tk, rng))
        for _ in range(2):  # two left operators per right operator: shared stage-1 products
            lops.append(random_operator(lsec, dn, tk, rng))
            pairs.append((len(lops) - 1, len(rops) - 1, tk, abs(dn) % 2, float(rng.normal())))
    size = sum(lsec[a][2] * rsec[b][2] for a, b in su2.coupled_blocks(lsec, rsec, n, tS))
    psi = rng.normal(size=size)
    ref = oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, psi)
    got = run(ctx, lsec, rsec, n, tS, lops, rops, pairs, psi)
    assert size > 1000 and np.abs(ref).max() > 1e-3
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


def test_su2_sigma_without_pairs_is_zero(ctx):
    rng = np.random.default_rng(7)
    lsec, rsec = sector_window(6, 0, 20, rng)
    size = sum(lsec[a][2] * rsec[b][2] for a, b in su2.coupled_blocks(lsec, rsec, 6, 0))
    got = run(ctx, lsec, rsec, 6, 0, [], [], [], rng.normal(size=size))
    assert np.all(got == 0.0)


def test_su2_sigma_rank_that_couples_nothing(ctx):
    """A pair whose operators have no block (a particle change no sector
    pair reaches) contributes nothing: only the other pair is seen."""
    rng = np.random.default_rng(8)
    n, tS = 8, 0
    lsec, rsec = sector_window(n, tS, 30, rng)
    a = random_operator(lsec, 0, 0, rng)
    b = random_operator(rsec, 0, 0, rng)
    far = random_operator(lsec, 7, 1, rng)
    rfar = random_operator(rsec, -7, 1, rng)
    assert not far and not rfar
    lops, rops = [a, far], [b, rfar]
    pairs = [(0, 0, 0, 0, 1.5), (1, 1, 1, 1, 2.0)]
    size = sum(lsec[i][2] * rsec[j][2] for i, j in su2.coupled_blocks(lsec, rsec, n, tS))
    psi = rng.normal(size=size)
    ref = oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs[:1], psi)
    got = run(ctx, lsec, rsec, n, tS, lops, rops, pairs, psi)
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()
