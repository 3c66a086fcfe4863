"""Oracle parity of the paths the benchmark takes (GPU).

* 22 and 36 orbitals (the CAS(22,22) and CAS(54,36) shapes at bond
  dimensions the oracle can reach), 2S_z = 0 and 4, the middle window and an
  off-centre one: the library's sigma in every precision and its diag(H_eff)
  against the oracle's block-sparse sigma and diagonal.  The oracle needs
  10-60 s per window here, so its results are stored in tests/golden/ by
  make_sigma_golden.py, which calls only the oracle; the test regenerates the
  seeded input and checks it against the stored one first.
* The workspace chunking of the headline run: these windows run in a context
  whose stage-1 workspace budget is 1 MiB (DMRG_WS_BUDGET_MB), so the right
  operators are split over many chunks (asserted >= 3), and the schedule's
  chunk boundaries (block-Hamiltonian pairs only in chunk 0, per-chunk BF16
  and Ozaki launches and slicing) are compared with the oracle.
* The mixed and emulated precisions against the oracle directly (not only
  against the library's own FP64 sigma), and diag(H_eff) against the
  oracle's at small and mid sizes.
* The chunked backward against the single-chunk one.

Bars: FP64 1e-10 relative (norm-wise) and per element 1e-10 of max|sigma|;
Ozaki 1e-12 (47 bits); split-BF16x3 1e-5 (the 3e-6 per-product error the
Davidson ladder assumes, with margin); BF16 2e-2 (2^-8 per operand);
diag(H_eff) per element 1e-10 of its largest entry (FP64).
"""
import glob
import os

import numpy as np
import pytest

from synthetic import make_integrals, make_mps, mps_arrays, pack_psi, unpack_psi
from tests.helpers import case, lib_load, lib_sigma_flat, rel_err, max_abs

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = sorted(glob.glob(os.path.join(HERE, "golden", "sigma_*.npz")))
REL = {"fp64": 1e-10, "ozaki": 1e-12, "bf16x3": 1e-5, "bf16": 2e-2}


@pytest.fixture(scope="module")
def chunked():
    """A context whose stage-1 workspace budget is 1 MiB."""
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
    yield c
    torch.cuda.synchronize()
    c.close()


def _flat_rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[6:-4] for p in GOLDEN])
def test_sigma_and_diag_match_stored_oracle_in_chunks(chunked, path):
    import torch
    z = np.load(path)
    K, N, tsz, D, i, iseed, mseed = (int(v) for v in z["case"])
    print(f"stored oracle sigma: K={K} N={N} 2Sz={tsz} D={D} window={i} (1 MiB workspace)", flush=True)
    h, eri = make_integrals(K, iseed)
    m = make_mps(K, N, tsz, D, i, mseed)
    psi = pack_psi(m.bonds, i, m.psi)
    assert psi.shape == z["psi"].shape and np.array_equal(psi, z["psi"]), "synthetic input changed"
    lib_load(chunked, h, eri, m)
    info = chunked.sigma_info()
    print(f"  {info['n_chunks']} workspace chunks, {info['n_pairs']} pairs", flush=True)
    assert info["n_chunks"] >= 3
    ref = z["sigma"]
    scale = float(np.max(np.abs(ref)))
    for prec in ("fp64", "ozaki", "bf16x3", "bf16"):
        got = lib_sigma_flat(chunked, psi, prec)
        rel = _flat_rel(got, ref)
        worst = float(np.max(np.abs(got - ref))) / scale
        print(f"  {prec}: relative {rel:.2e}, max element error / max|sigma| {worst:.2e}", flush=True)
        assert rel <= REL[prec]
        if prec == "fp64":
            assert worst <= 1e-10
    d = torch.empty(psi.size, dtype=torch.float64, device="cuda")
    chunked.debug_diag(d)
    torch.cuda.synchronize()
    dd = d.cpu().numpy()
    derr = float(np.max(np.abs(dd - z["diag"]))) / float(np.max(np.abs(z["diag"])))
    print(f"  diag(H_eff): max element error / max|diag| {derr:.2e}", flush=True)
    assert derr <= 1e-10


MID = [(12, 12, 0, 256, 5), (10, 9, 1, 200, 2), (12, 14, 2, 150, 7)]


@pytest.mark.parametrize("K,N,tsz,D,i", MID)
def test_mixed_and_emulated_sigma_against_oracle(ctx, K, N, tsz, D, i):
    from oracle.blocksparse import BlockSparseSigma
    print(f"mixed sigma vs block-sparse oracle: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = BlockSparseSigma(m, h, eri).apply(m.psi)
    lib_load(ctx, h, eri, m)
    flat = pack_psi(m.bonds, i, m.psi)
    for prec in ("ozaki", "bf16x3", "bf16"):
        got = unpack_psi(m.bonds, i, lib_sigma_flat(ctx, flat, prec))
        r = rel_err(got, ref)
        print(f"  {prec}: relative {r:.2e}", flush=True)
        assert r <= REL[prec]


DIAG = [(6, 6, 0, 12, 2), (6, 5, 1, 10, 0), (8, 6, 2, 30, 5), (12, 12, 0, 256, 5), (10, 9, 1, 200, 2)]


@pytest.mark.parametrize("K,N,tsz,D,i", DIAG)
def test_diag_matches_oracle(ctx, K, N, tsz, D, i):
    import torch
    from oracle.blocksparse import BlockSparseSigma
    from oracle.projection import psi_template
    print(f"diag(H_eff) vs oracle: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = BlockSparseSigma(m, h, eri).diagonal(psi_template(m))
    n = lib_load(ctx, h, eri, m)
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.debug_diag(d)
    torch.cuda.synchronize()
    got = unpack_psi(m.bonds, i, d.cpu().numpy())
    scale = max(float(np.max(np.abs(v))) for v in ref.values() if v.size)
    err = max_abs(got, ref) / scale
    print(f"  max element error / max|diag| {err:.2e}", flush=True)
    assert err <= 1e-10


def test_chunked_backward_equals_single_chunk(ctx, chunked):
    import torch
    print("backward, 1 MiB workspace against one chunk: K=12 D=256 window 5", flush=True)
    h, eri, m = case(12, 12, 0, 256, 5)
    flat = pack_psi(m.bonds, 5, m.psi)
    flat /= np.linalg.norm(flat)
    out = []
    for c in (ctx, chunked):
        lib_load(c, h, eri, m)
        p = torch.from_numpy(flat.copy()).cuda()
        dh, deri = c.sigma_backward(p)
        torch.cuda.synchronize()
        out.append((dh.cpu().numpy(), deri.cpu().numpy()))
    assert chunked.sigma_info()["n_chunks"] >= 3
    for a, b in zip(out[0], out[1]):
        r = _flat_rel(b, a)
        print(f"  relative difference {r:.2e}", flush=True)
        assert r <= 1e-12
