"""Davidson solve on the GPU against exact eigenvalues from the oracle (GPU)."""
import numpy as np
import pytest

from tests.helpers import case, lib_load

pytestmark = pytest.mark.gpu

MIXED = (("bf16", 1e-2), ("bf16x3", 1e-4), ("fp64", None))


def _oracle_lowest(h, eri, m):
    import scipy.sparse.linalg as spla
    from oracle.blocksparse import BlockSparseSigma
    from synthetic import pack_psi, unpack_psi
    bs = BlockSparseSigma(m, h, eri)
    n = m.psi_size()
    mv = lambda x: pack_psi(m.bonds, m.window, bs.apply(unpack_psi(m.bonds, m.window, x)))
    w = spla.eigsh(spla.LinearOperator((n, n), matvec=mv), k=1, which="SA", tol=1e-13,
                   v0=np.ones(n))[0]
    return float(w[0])


def _start(ctx, m):
    import torch
    from synthetic import pack_psi
    return torch.from_numpy(pack_psi(m.bonds, m.window, m.psi)).cuda()


def test_davidson_fp64_reaches_fci_on_complete_window(ctx):
    from oracle.fock import fci
    print("davidson fp64 K=8 D=64 (complete window) vs FCI", flush=True)
    h, eri, m = case(8, 8, 0, 64, 3, iseed=8, mseed=1008)
    lib_load(ctx, h, eri, m)
    psi = _start(ctx, m)
    r = ctx.davidson(psi, tol=1e-8)
    e_fci = fci(8, 8, 0, h, eri)[0][0]
    print(f"  E={r['energy']:.12f} FCI={e_fci:.12f} iters={r['iterations']}", flush=True)
    assert r["converged"] and r["residual"] < 1e-8
    assert abs(r["energy"] - e_fci) < 1e-10


@pytest.mark.parametrize("K,N,tsz,D,i", [(10, 9, 1, 200, 2), (12, 12, 0, 256, 5)])
def test_davidson_fp64_matches_oracle_eigenvalue(ctx, K, N, tsz, D, i):
    print(f"davidson fp64 K={K} D={D} vs oracle eigsh", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    lib_load(ctx, h, eri, m)
    r = ctx.davidson(_start(ctx, m), tol=1e-7)
    e_ref = _oracle_lowest(h, eri, m)
    print(f"  E={r['energy']:.12f} ref={e_ref:.12f} iters={r['iterations']} res={r['residual']:.2e} hist={[round(x, 9) for x in r['residual_history'][-8:]]}", flush=True)
    assert r["converged"]
    assert abs(r["energy"] - e_ref) < 1e-9 * max(1.0, abs(e_ref))


@pytest.mark.parametrize("K,N,tsz,D,i", [(12, 12, 0, 256, 5), (14, 14, 0, 400, 6)])
def test_mixed_ladder_energy_within_1e6_of_fp64(ctx, K, N, tsz, D, i):
    print(f"davidson mixed ladder K={K} D={D}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    lib_load(ctx, h, eri, m)
    r64 = ctx.davidson(_start(ctx, m), tol=1e-6)
    rmx = ctx.davidson(_start(ctx, m), tol=1e-6, ladder=MIXED)
    print(f"  E64={r64['energy']:.12f} Emix={rmx['energy']:.12f} n_sigma={rmx['n_sigma']} "
          f"fp64 n_sigma={r64['n_sigma']}", flush=True)
    assert r64["converged"] and rmx["converged"]
    assert abs(rmx["energy"] - r64["energy"]) < 1e-6


def test_davidson_warns_when_iterations_run_out(ctx):
    h, eri, m = case(12, 12, 0, 256, 5)
    lib_load(ctx, h, eri, m)
    r = ctx.davidson(_start(ctx, m), tol=1e-12, max_iter=2)
    assert r["status"] == 1 and not r["converged"]
    assert np.isfinite(r["energy"])


@pytest.mark.parametrize("K,N,tsz,D,i", [(10, 9, 1, 200, 2), (12, 12, 0, 256, 5)])
def test_refined_ladder_matches_oracle_eigenvalue(ctx, K, N, tsz, D, i):
    """Split-BF16x3 Davidson, then residual refinement (FP64 residuals,
    corrections solved on split-BF16x3 sigmas): the oracle's eigenvalue, with
    a handful of FP64 sigma products."""
    print(f"davidson bf16x3 + refinement K={K} D={D} vs oracle eigsh", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    lib_load(ctx, h, eri, m)
    r = ctx.davidson(_start(ctx, m), tol=1e-7, max_iter=400,
                     ladder=(("bf16x3", 1e-4), ("fp64", None)), refine=True)
    e_ref = _oracle_lowest(h, eri, m)
    print(f"  E={r['energy']:.12f} ref={e_ref:.12f} iters={r['iterations']} res={r['residual']:.2e} "
          f"n_sigma={r['n_sigma']}", flush=True)
    assert r["converged"] and r["residual"] < 1e-7
    assert abs(r["energy"] - e_ref) < 1e-9 * max(1.0, abs(e_ref))
    assert r["n_sigma"]["fp64"] <= 14


def test_refined_full_ladder_matches_fp64(ctx):
    print("davidson bf16 -> bf16x3 -> refinement K=14 D=400 vs FP64 Davidson", flush=True)
    h, eri, m = case(14, 14, 0, 400, 6)
    lib_load(ctx, h, eri, m)
    r64 = ctx.davidson(_start(ctx, m), tol=1e-6, max_iter=400)
    rrf = ctx.davidson(_start(ctx, m), tol=1e-6, max_iter=400, ladder=MIXED, refine=True)
    print(f"  E64={r64['energy']:.12f} Erefined={rrf['energy']:.12f} n_sigma={rrf['n_sigma']} "
          f"fp64 n_sigma={r64['n_sigma']}", flush=True)
    assert r64["converged"] and rrf["converged"]
    assert abs(rrf["energy"] - r64["energy"]) < 1e-6
