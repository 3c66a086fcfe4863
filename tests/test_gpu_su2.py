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
from synthetic.su2 import sector_window, random_operator, pack, unpack, cas89_102_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10
# split-BF16x3: operands and the stage-1 intermediate as BF16 hi + lo carry
# a relative error of about 2^-18 (3.8e-6) per element, products accumulate
# in FP32 and are flushed into FP64 per product; measured 6.3e-6
TOL_X3 = 2e-5
INVALID_ARG = -1  # DMRG_ERR_INVALID_ARG


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def device_ops(lst):
    out = []
    for o in lst:
        blocks, data = pack_blocks(o)
        out.append((blocks, dev(data)))
    return out


def run(ctx, lsec, rsec, n, tS, lops, rops, pairs, psi_flat):
    import torch
    psi = dev(psi_flat)
    out = torch.full_like(psi, float("nan"))
    ctx.su2_sigma(lsec, rsec, n, tS, device_ops(lops), device_ops(rops), pairs, psi, out)
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


def case_ops(n, tS, dmax, seed):
    rng = np.random.default_rng(seed)
    lsec, rsec = sector_window(n, tS, dmax, rng)
    lops, rops, pairs = [], [], []
    for dn, tk in [(0, 0), (0, 2), (1, 1), (-1, 1), (2, 0), (-2, 2), (1, 3)]:
        rops.append(random_operator(rsec, -dn, tk, rng))
        for _ in range(2):  # two left operators per right operator: shared stage-1 products
            lops.append(random_operator(lsec, dn, tk, rng))
            pairs.append((len(lops) - 1, len(rops) - 1, tk, abs(dn) % 2, float(rng.normal())))
    size = sum(lsec[a][2] * rsec[b][2] for a, b in su2.coupled_blocks(lsec, rsec, n, tS))
    return lsec, rsec, lops, rops, pairs, size, rng


def close(got, ref):
    return np.abs(got - ref).max() <= TOL * np.abs(ref).max()


@pytest.mark.parametrize("n,tS,dmax,seed", CASES)
def test_su2_sigma_matches_the_oracle(ctx, n, tS, dmax, seed):
    print(f"su2 sigma: n={n} 2S={tS} dmax={dmax} seed={seed}", flush=True)
    lsec, rsec, lops, rops, pairs, size, rng = case_ops(n, tS, dmax, seed)
    psi = rng.normal(size=size)
    ref = oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, psi)
    got = run(ctx, lsec, rsec, n, tS, lops, rops, pairs, psi)
    assert size > 1000 and np.abs(ref).max() > 1e-3
    assert close(got, ref)


def test_su2_plan_applied_twice_and_in_place(ctx):
    """One plan, two window vectors, then sigma written over psi itself."""
    import torch
    n, tS = 10, 2
    lsec, rsec, lops, rops, pairs, size, rng = case_ops(n, tS, 300, 3)
    L, R = device_ops(lops), device_ops(rops)
    with ctx.su2_plan(lsec, rsec, n, tS, L, R, pairs) as plan:
        info = plan.info()
        assert info["psi_size"] == size and info["n_chunks"] == 1 and info["flops_stage2"] > 0
        for seed in (1, 2):
            x = np.random.default_rng(seed).normal(size=size)
            out = torch.full((size,), float("nan"), dtype=torch.float64, device="cuda")
            plan.sigma(dev(x), out)
            torch.cuda.synchronize()
            assert close(out.cpu().numpy(), oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, x))
        buf = dev(x)
        plan.sigma(buf, buf)
        torch.cuda.synchronize()
        assert close(buf.cpu().numpy(), oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, x))


@pytest.mark.parametrize("n,tS,dmax,seed", CASES)
def test_su2_bf16x3_plan_matches_the_oracle(ctx, n, tS, dmax, seed):
    """The split-BF16x3 plan against the oracle: relative error of the whole
    vector below TOL_X3, and no element off by more than TOL_X3 max|sigma|."""
    import torch
    print(f"su2 bf16x3 sigma: n={n} 2S={tS} dmax={dmax} seed={seed}", flush=True)
    lsec, rsec, lops, rops, pairs, size, rng = case_ops(n, tS, dmax, seed)
    psi = rng.normal(size=size)
    ref = oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, psi)
    L, R = device_ops(lops), device_ops(rops)
    with ctx.su2_plan(lsec, rsec, n, tS, L, R, pairs, precision="bf16x3") as plan:
        out = torch.full((size,), float("nan"), dtype=torch.float64, device="cuda")
        plan.sigma(dev(psi), out)
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  relative error {rel:.2e}", flush=True)
    assert rel <= TOL_X3 and rel > 0
    assert np.abs(got - ref).max() <= TOL_X3 * np.abs(ref).max()


def test_su2_plan_in_workspace_chunks():
    """A context with a 1 MiB stage-1 budget splits the right operators
    into several chunks; the result is the oracle's."""
    import os
    import torch
    from paper_2603_28648_amd import Context
    old = os.environ.get("DMRG_WS_BUDGET_MB")
    os.environ["DMRG_WS_BUDGET_MB"] = "1"
    try:
        c = Context(0)
    finally:
        if old is None:
            del os.environ["DMRG_WS_BUDGET_MB"]
        else:
            os.environ["DMRG_WS_BUDGET_MB"] = old
    try:
        n, tS = 12, 0
        lsec, rsec, lops, rops, pairs, size, rng = case_ops(n, tS, 260, 4)
        psi = rng.normal(size=size)
        L, R = device_ops(lops), device_ops(rops)
        ref = oracle_sigma(lsec, rsec, n, tS, lops, rops, pairs, psi)
        for precision in ("fp64", "bf16x3"):
            with c.su2_plan(lsec, rsec, n, tS, L, R, pairs, precision=precision) as plan:
                info = plan.info()
                print(f"su2 chunks ({precision}): {info}", flush=True)
                # a chunk holds at least one right operator, so one whose products
                # exceed the budget gets a chunk of its own
                assert info["n_chunks"] > 1
                out = torch.empty(size, dtype=torch.float64, device="cuda")
                plan.sigma(dev(psi), out)
                torch.cuda.synchronize()
            got = out.cpu().numpy()
            if precision == "fp64":
                assert close(got, ref)
            else:
                assert np.linalg.norm(got - ref) <= TOL_X3 * np.linalg.norm(ref)
    finally:
        c.close()


def test_su2_plan_of_another_context_is_an_error(ctx):
    """A plan is only valid with the context that made it, and not after
    it was destroyed (host-side checks, no kernel runs)."""
    import torch
    from paper_2603_28648_amd import Context
    n, tS = 8, 0
    lsec, rsec, lops, rops, pairs, size, rng = case_ops(n, tS, 20, 6)
    L, R = device_ops(lops), device_ops(rops)
    x = torch.zeros(size, dtype=torch.float64, device="cuda")
    other = Context(0)
    try:
        plan = other.su2_plan(lsec, rsec, n, tS, L, R, pairs)
        h = plan.h
        assert ctx.lib.dmrg_su2_plan_sigma(ctx.h, h, x.data_ptr(), x.data_ptr()) == INVALID_ARG
        assert b"plan" in ctx.lib.dmrg_last_error(ctx.h)
        plan.close()
        assert other.lib.dmrg_su2_plan_sigma(other.h, h, x.data_ptr(), x.data_ptr()) == INVALID_ARG
    finally:
        other.close()


def test_su2_sigma_cas89_102_sampled(ctx):
    """The CAS(89,102)-shaped workload (S = 5/2, 2048 multiplets a side,
    10,610 operator pairs of the spin-adapted Hamiltonian's structure,
    random reduced blocks) through the plan the benchmark times, checked
    on sampled output blocks: the largest and two drawn at random, each
    computed by the oracle from every operator block that feeds it."""
    import torch
    w = cas89_102_workload()
    lsec, rsec, n, tS = w["left_sectors"], w["right_sectors"], w["n"], w["two_s"]
    print(f"su2 CAS(89,102): {len(w['pairs'])} pairs, psi {w['psi'].numel()}", flush=True)
    with ctx.su2_plan(lsec, rsec, n, tS, w["left_ops"], w["right_ops"], w["pairs"]) as plan:
        info = plan.info()
        print(f"su2 CAS(89,102) plan: {info}", flush=True)
        out = torch.full_like(w["psi"], float("nan"))
        plan.sigma(w["psi"], out)
        torch.cuda.synchronize()
    with ctx.su2_plan(lsec, rsec, n, tS, w["left_ops"], w["right_ops"], w["pairs"], precision="bf16x3") as plan:
        out3 = torch.full_like(w["psi"], float("nan"))
        plan.sigma(w["psi"], out3)
        torch.cuda.synchronize()
    rel3 = float(torch.linalg.norm(out3 - out) / torch.linalg.norm(out))
    print(f"su2 CAS(89,102) bf16x3 against FP64: relative error {rel3:.2e}", flush=True)
    assert rel3 <= TOL_X3
    got = unpack(lsec, rsec, n, tS, out.cpu().numpy())
    got3 = unpack(lsec, rsec, n, tS, out3.cpu().numpy())
    psi = unpack(lsec, rsec, n, tS, w["psi"].cpu().numpy())
    blocks = su2.coupled_blocks(lsec, rsec, n, tS)
    sizes = [lsec[a][2] * rsec[b][2] for a, b in blocks]
    rng = np.random.default_rng(7)
    picks = [blocks[int(np.argmax(sizes))]] + [blocks[i] for i in rng.choice(len(blocks), 2, replace=False)]
    lset, rset = {a for a, _ in picks}, {b for _, b in picks}

    def restricted(ops, sectors, keep_out):
        """{op: {(out, in): block}} for the blocks whose out sector is kept,
        copied from the device in one gather."""
        spans = []
        for k, (blocks_k, _, base) in enumerate(ops):
            for o, i, off in blocks_k:
                if o in keep_out:
                    spans.append((k, o, i, base + off, sectors[o][2], sectors[i][2]))
        data = ops[0][1]
        idx = np.concatenate([np.arange(s, s + d2 * d1) for _, _, _, s, d2, d1 in spans])
        vals = data[torch.from_numpy(idx).cuda()].cpu().numpy()
        res = [dict() for _ in ops]
        pos = 0
        for k, o, i, _, d2, d1 in spans:
            res[k][(o, i)] = vals[pos:pos + d2 * d1].reshape(d2, d1)
            pos += d2 * d1
        return res

    A = restricted(w["left_ops"], lsec, lset)
    B = restricted(w["right_ops"], rsec, rset)
    ref = su2.contract_scalar_products(lsec, rsec, n, tS, psi,
                                       [(c, tk, pb, A[l], B[r]) for l, r, tk, pb, c in w["pairs"]])
    assert info["psi_size"] == w["psi"].numel() and info["n_segments"] > 10 ** 6
    for k in picks:
        print(f"su2 CAS(89,102) block {k}: max|ref| {np.abs(ref[k]).max():.3e}", flush=True)
        assert np.abs(ref[k]).max() > 1.0
        assert np.abs(got[k] - ref[k]).max() <= TOL * np.abs(ref[k]).max()
        assert np.abs(got3[k] - ref[k]).max() <= TOL_X3 * np.abs(ref[k]).max()


def test_su2_operator_past_its_tensor_is_refused(ctx):
    """The binding checks every block against its data tensor before the
    library sees the pointers (no kernel runs)."""
    import torch
    lsec, rsec = [(1, 1, 4)], [(1, 1, 3)]
    short = torch.zeros(15, dtype=torch.float64, device="cuda")  # a 4 x 4 block needs 16
    ok = torch.zeros(9, dtype=torch.float64, device="cuda")
    psi = torch.zeros(12, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.su2_sigma(lsec, rsec, 2, 0, [([(0, 0, 0)], short)], [([(0, 0, 0)], ok)], [(0, 0, 0, 0, 1.0)],
                      psi, psi.clone())
    full = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):  # the right block starts one element in: it ends past the tensor
        ctx.su2_sigma(lsec, rsec, 2, 0, [([(0, 0, 0)], full)], [([(0, 0, 0)], ok, 1)], [(0, 0, 0, 0, 1.0)],
                      psi, psi.clone())
    out = psi.clone()
    ctx.su2_sigma(lsec, rsec, 2, 0, [([(0, 0, 0)], full)], [([(0, 0, 0)], ok, 0)], [(0, 0, 0, 0, 1.0)],
                  psi, out)
    assert torch.all(out == 0)


def coupled_sector_keys(sec1, sec2):
    """(i1, i2, 2S) of every coupled sector, in the library's numbering."""
    keys = []
    for i1, (_, s1, _) in enumerate(sec1):
        for i2, (_, s2, _) in enumerate(sec2):
            keys += [(i1, i2, ts) for ts in range(abs(s1 - s2), s1 + s2 + 1, 2)]
    return keys


@pytest.mark.parametrize("dn1,tk1,dn2,tk2,tk,site", [(1, 1, 0, 0, 1, True), (0, 0, 1, 1, 1, True),
                                                     (1, 1, 1, 1, 0, True), (1, 1, -1, 1, 2, True),
                                                     (0, 2, -1, 1, 3, True), (1, 1, 1, 1, 2, False),
                                                     (0, 2, 0, 2, 2, False)])
def test_su2_product_matches_the_oracle(ctx, dn1, tk1, dn2, tk2, tk, site):
    """The renormalisation step's coupled product [A^k1 x B^k2]^k
    (dmrg_su2_product) against the oracle's product_operator, block by
    block: a block operator with sectors up to 120 multiplets times a
    one-orbital site operator, or one with sectors up to 40 times a second
    block's operator (sectors up to 6)."""
    print(f"su2 product: dn1={dn1} 2k1={tk1} dn2={dn2} 2k2={tk2} 2k={tk} site={site}", flush=True)
    rng = np.random.default_rng(11 + tk1 + 3 * tk + 5 * dn1)
    sec1, _ = sector_window(8, 0, 120 if site else 40, rng)
    # a one-orbital site, or a second block of small sectors (its blocks
    # multiply the Kronecker products' sizes)
    sec2 = [(0, 0, 1), (1, 1, 1), (2, 0, 1)] if site else sector_window(8, 0, 6, rng)[1]
    t1 = random_operator(sec1, dn1, tk1, rng)
    t2 = random_operator(sec2, dn2, tk2, rng, keep=1.0)
    p2 = abs(dn2) % 2
    want = su2.product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, p2)
    ops = device_ops([t1, t2])
    blocks, data = ctx.su2_product(sec1, sec2, ops[0], ops[1], tk1, tk2, tk, p2)
    torch_data = data.cpu().numpy()
    keys = coupled_sector_keys(sec1, sec2)
    nz = {k: v for k, v in want.items() if np.any(v != 0)}
    assert len(blocks) == len(nz) > 0
    scale = max(np.abs(v).max() for v in nz.values())
    for out, inn, off in blocks:
        k = (keys[out], keys[inn])
        ref = nz[k]
        got = torch_data[off:off + ref.size].reshape(ref.shape)
        assert np.abs(got - ref).max() <= TOL * scale


@pytest.mark.parametrize("dn1,tk1,dn2,tk2,tk,seed", [(1, 1, 0, 2, 1, 1), (1, 1, -1, 1, 2, 2), (0, 2, 1, 1, 1, 3)])
def test_su2_renormalisation_matches_the_oracle(ctx, dn1, tk1, dn2, tk2, tk, seed):
    """The renormalisation of a block operator times a site operator: the
    coupled product (dmrg_su2_product) projected onto a truncated basis of
    every (N, S) sector of the enlarged block (dmrg_su2_rotate), against the
    oracle's product_operator and rotate_operator."""
    print(f"su2 renormalisation: dn1={dn1} 2k1={tk1} dn2={dn2} 2k2={tk2} 2k={tk} seed={seed}", flush=True)
    rng = np.random.default_rng(100 + seed)
    sec1, _ = sector_window(8, 0, 90, rng)
    sec2 = [(0, 0, 1), (1, 1, 1), (2, 0, 1)]
    t1 = random_operator(sec1, dn1, tk1, rng)
    t2 = random_operator(sec2, dn2, tk2, rng, keep=1.0)
    p2 = abs(dn2) % 2
    ops = device_ops([t1, t2])
    blocks, data = ctx.su2_product(sec1, sec2, ops[0], ops[1], tk1, tk2, tk, p2)
    keys = coupled_sector_keys(sec1, sec2)
    cdim = [sec1[i1][2] * sec2[i2][2] for i1, i2, _ in keys]
    groups = sorted({(sec1[i1][0] + sec2[i2][0], ts) for i1, i2, ts in keys})
    cgroup = [groups.index((sec1[i1][0] + sec2[i2][0], ts)) for i1, i2, ts in keys]
    gsize = [sum(cdim[c] for c in range(len(keys)) if cgroup[c] == g) for g in range(len(groups))]
    gdim = [max(1, (3 * n) // 4) for n in gsize]  # truncated: three quarters of each sector kept
    cgroup = [g if g % 5 else -1 for g in cgroup]  # every fifth new sector kept out
    proj_np, row = [], [0] * len(groups)
    U = [rng.normal(size=(gsize[g], gdim[g])) for g in range(len(groups))]
    for c in range(len(keys)):
        g = groups.index((sec1[keys[c][0]][0] + sec2[keys[c][1]][0], keys[c][2]))
        proj_np.append(U[g][row[g]:row[g] + cdim[c]] if cgroup[c] >= 0 else None)
        row[g] += cdim[c]
    proj = [dev(p) if p is not None else None for p in proj_np]
    out_blocks, out = ctx.su2_rotate(blocks, data, cdim, cgroup, gdim, proj)
    want_prod = su2.product_operator(sec1, sec2, t1, t2, tk1, tk2, tk, p2)
    index = {k: i for i, k in enumerate(keys)}
    keyed = {(index[k2], index[k]): v for (k2, k), v in want_prod.items() if np.any(v != 0)}
    want = {k: v for k, v in su2.rotate_operator(keyed, proj_np, cgroup).items()}
    got_np = out.cpu().numpy()
    assert len(out_blocks) == len(want) > 0
    scale = max(np.abs(v).max() for v in want.values())
    for g2, g, off in out_blocks:
        ref = want[(g2, g)]
        got = got_np[off:off + ref.size].reshape(ref.shape)
        assert np.abs(got - ref).max() <= TOL * scale


def test_su2_rotate_refuses_bad_projectors(ctx):
    """The binding checks projector shapes and block ranges before the
    library sees the pointers (no kernel runs)."""
    import torch
    data = torch.zeros(8, dtype=torch.float64, device="cuda")
    cdim, cgroup, gdim = [2, 2], [0, 0], [3]
    good = [torch.zeros(2, 3, dtype=torch.float64, device="cuda") for _ in range(2)]
    bad = [torch.zeros(2, 2, dtype=torch.float64, device="cuda"), good[1]]
    with pytest.raises(ValueError):  # projector of the wrong shape
        ctx.su2_rotate([(0, 1, 0)], data, cdim, cgroup, gdim, bad)
    with pytest.raises(ValueError):  # a kept sector without a projector
        ctx.su2_rotate([(0, 1, 0)], data, cdim, cgroup, gdim, [None, good[1]])
    with pytest.raises(ValueError):  # a block past the data tensor
        ctx.su2_rotate([(0, 1, 6)], data, cdim, cgroup, gdim, good)
    blocks, out = ctx.su2_rotate([(0, 1, 0), (1, 0, 4)], data, cdim, cgroup, gdim, good)
    assert blocks == [(0, 0, 0)] and torch.all(out == 0)


@pytest.mark.parametrize("n,tS", [(4, 0), (4, 2), (3, 1)])
def test_su2_sigma_of_the_window_hamiltonian(ctx, n, tS):
    """The library's spin-adapted sigma (dmrg_su2_sigma) with the window
    Hamiltonian's scalar products (oracle window_pairs, four orbitals split
    2 | 2) equals the spin-adapted H_eff by its definition, whose spectrum
    is the full-CI spectrum of spin S."""
    from synthetic import make_integrals
    K, nl = 4, 2
    h, eri = make_integrals(K, K)
    left, right = su2.multiplets(nl), su2.multiplets(K - nl)
    lsec = [(M.n, M.tS, M.dim) for M in left]
    rsec = [(M.n, M.tS, M.dim) for M in right]
    pairs = su2.window_pairs(h, eri, left, right, nl, K - nl)
    m, basis = su2.heff_su2(h, eri, left, right, nl, K - nl, n, tS)
    psi_flat = np.random.default_rng(9 + n).normal(size=len(basis))
    blocks = su2.coupled_blocks(lsec, rsec, n, tS)
    psi = {k: np.zeros((lsec[k[0]][2], rsec[k[1]][2])) for k in blocks}
    for c, (ia, al, ib, be) in enumerate(basis):
        psi[(ia, ib)][al, be] = psi_flat[c]
    packed = pack(lsec, rsec, n, tS, psi)
    lops = [p[3] for p in pairs]
    rops = [p[4] for p in pairs]
    lib_pairs = [(i, i, p[1], p[2], p[0]) for i, p in enumerate(pairs)]
    got = unpack(lsec, rsec, n, tS, run(ctx, lsec, rsec, n, tS, lops, rops, lib_pairs, packed))
    got_flat = np.array([got[(ia, ib)][al, be] for (ia, al, ib, be) in basis])
    ref = m @ psi_flat
    assert np.abs(ref).max() > 1e-2
    assert np.abs(got_flat - ref).max() <= TOL * np.abs(ref).max()
