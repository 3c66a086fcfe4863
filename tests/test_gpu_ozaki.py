"""Ozaki-scheme FP64 emulation on INT8 MFMA (precision "ozaki"), on the GPU.

Kernel level (dmrg_debug_gemm): against an FP64 product computed on the CPU,
element-wise within the bound the scheme guarantees.  Each row of A (and
of B's n x k storage) is scaled by 2^-e with |x| < (127/128) 2^e and
rounded to p = 8 kappa - 1 bits, so each entry carries an error of at most
2^(e - p - 1); the digit products dropped (weights below kappa - 1) add at
most 1.004 (kappa - 1) k 2^(e_i + f_j - 8 kappa); so
    |C - AB|_ij <= |alpha| k 2^(e_i + f_j) (2^-p + 1.01 (kappa - 1) 2^(-8 kappa))
plus the FP64 rounding of the reference (k 2^-52 sum |a||b|).

Sigma level: the Ozaki sigma against the FP64 sigma at several windows and
at 16 orbitals / D = 512 (relative 1e-12 at kappa = 6, the 47-bit setting).
"""
import numpy as np
import pytest

from synthetic import pack_psi
from tests.helpers import case, lib_load, lib_sigma_flat

pytestmark = pytest.mark.gpu


def _exps(rows):
    """Row exponents as the slicer picks them (|x| < (127/128) 2^e)."""
    mx = np.max(np.abs(rows), axis=1)
    e = np.frexp(mx * (128.0 / 127.0))[1].astype(np.int64)  # ilogb + 1
    e[mx == 0] = 0
    return e


def _run(ctx, A, Bt, alpha=1.0, beta=0, C0=None, trans_a=False, trans_b=True):
    import torch
    m, k = A.shape
    n = Bt.shape[0]
    a = A.T.copy() if trans_a else A
    b = Bt if trans_b else Bt.T.copy()
    da = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    db = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    c = torch.from_numpy(np.zeros((m, n)) if C0 is None else C0.copy()).cuda()
    ctx.debug_gemm(da, db, c, trans_a=trans_a, trans_b=trans_b, alpha=alpha, beta=beta, precision="ozaki")
    torch.cuda.synchronize()
    return c.cpu().numpy()


def _check(A, Bt, got, kappa, alpha=1.0, C0=None):
    m, k = A.shape
    ref = alpha * (A @ Bt.T) + (0 if C0 is None else C0)
    p = 8 * kappa - 1
    ea, eb = _exps(A), _exps(Bt)
    scale = np.ldexp(1.0, (ea[:, None] + eb[None, :]).astype(np.int64))
    bound = abs(alpha) * k * scale * (2.0 ** -p + 1.01 * (kappa - 1) * 2.0 ** (-8 * kappa))
    bound += k * 2.0 ** -52 * (np.abs(A) @ np.abs(Bt).T) * abs(alpha) + 2.0 ** -52 * np.abs(ref)
    err = np.abs(got - ref)
    worst = float(np.max(err / np.maximum(bound, 1e-300)))
    return worst


@pytest.mark.parametrize("kappa", [3, 4, 5, 6, 7])
def test_ozaki_gemm_within_bound_each_kappa(ctx, kappa, monkeypatch):
    monkeypatch.setenv("DMRG_OZAKI_SLICES", str(kappa))
    rng = np.random.default_rng(kappa)
    m, n, k = 131, 70, 203  # ragged in every dimension
    A = rng.normal(size=(m, k)) * np.ldexp(1.0, rng.integers(-20, 20, size=(m, 1)))
    Bt = rng.normal(size=(n, k)) * np.ldexp(1.0, rng.integers(-20, 20, size=(n, 1)))
    got = _run(ctx, A, Bt)
    worst = _check(A, Bt, got, kappa)
    print(f"kappa={kappa}: worst error / bound = {worst:.3f}", flush=True)
    assert worst <= 1.0
    # the error shrinks with kappa: kappa = 6 reaches FP64-class accuracy
    rel = np.max(np.abs(got - A @ Bt.T)) / np.max(np.abs(A @ Bt.T))
    if kappa >= 6:
        assert rel < 1e-13


@pytest.mark.parametrize("m,n,k,ta,tb", [
    (1, 1, 1, False, True), (64, 64, 64, False, True), (65, 63, 15, True, False),
    (200, 129, 1000, False, False), (17, 300, 640, True, True), (128, 64, 2048, False, True)])
def test_ozaki_gemm_shapes_and_storage(ctx, m, n, k, ta, tb):
    rng = np.random.default_rng(m * 7 + n + k)
    A = rng.normal(size=(m, k))
    Bt = rng.normal(size=(n, k))
    got = _run(ctx, A, Bt, trans_a=ta, trans_b=tb)
    assert _check(A, Bt, got, 6) <= 1.0


def test_ozaki_gemm_scale_beta_and_zero_rows(ctx):
    rng = np.random.default_rng(3)
    m, n, k = 96, 80, 77
    A = rng.normal(size=(m, k)) * np.ldexp(1.0, rng.integers(-300, 300, size=(m, 1)))
    A[5] = 0.0
    A[:, 40:] *= 1e-9  # dynamic range inside rows
    Bt = rng.normal(size=(n, k)) * np.ldexp(1.0, rng.integers(-300, 300, size=(n, 1)))
    Bt[7] = 0.0
    C0 = rng.normal(size=(m, n))
    got = _run(ctx, A, Bt, alpha=-0.37, beta=1, C0=C0)
    assert _check(A, Bt, got, 6, alpha=-0.37, C0=C0) <= 1.0
    assert np.all(got[5] == C0[5]) and np.all(got[:, 7] == C0[:, 7])


@pytest.mark.parametrize("K,N,tsz,D,i", [(4, 4, 0, 100, 1), (6, 6, 0, 12, 2), (6, 7, -1, 10, 4),
                                         (8, 8, 0, 20, 3), (8, 6, 2, 30, 5), (10, 10, 0, 200, 4)])
def test_ozaki_sigma_matches_fp64(ctx, K, N, tsz, D, i):
    print(f"ozaki sigma vs FP64: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    lib_load(ctx, h, eri, m)
    psi = pack_psi(m.bonds, m.window, m.psi)
    s64 = lib_sigma_flat(ctx, psi, "fp64")
    soz = lib_sigma_flat(ctx, psi, "ozaki")
    soz2 = lib_sigma_flat(ctx, psi, "ozaki")
    rel = np.linalg.norm(soz - s64) / np.linalg.norm(s64)
    print(f"  relative error {rel:.2e}", flush=True)
    assert rel < 1e-12
    assert np.array_equal(soz, soz2)  # deterministic, operator slices reused


def test_ozaki_sigma_at_16_orbitals(ctx):
    print("ozaki sigma vs FP64: K=16 N=16 D=512 window=7", flush=True)
    h, eri, m = case(16, 16, 0, 512, 7)
    lib_load(ctx, h, eri, m)
    psi = pack_psi(m.bonds, m.window, m.psi)
    s64 = lib_sigma_flat(ctx, psi, "fp64")
    soz = lib_sigma_flat(ctx, psi, "ozaki")
    rel = np.linalg.norm(soz - s64) / np.linalg.norm(s64)
    e64 = float(psi @ s64) / float(psi @ psi)
    eoz = float(psi @ soz) / float(psi @ psi)
    print(f"  relative error {rel:.2e}, Rayleigh quotient difference {abs(eoz - e64):.2e}", flush=True)
    assert rel < 1e-12
    assert abs(eoz - e64) < 1e-10


def test_ozaki_ladder_stage_in_davidson(ctx):
    """An Ozaki stage in the Davidson ladder: same converged energy as FP64."""
    import torch
    print("davidson ladder ozaki -> fp64: K=8 N=8 D=20 window=3", flush=True)
    h, eri, m = case(8, 8, 0, 20, 3)
    lib_load(ctx, h, eri, m)
    psi0 = torch.from_numpy(pack_psi(m.bonds, m.window, m.psi)).cuda()
    x64 = psi0.clone()
    r64 = ctx.davidson(x64, tol=1e-9, max_iter=200)
    xoz = psi0.clone()
    roz = ctx.davidson(xoz, tol=1e-9, max_iter=200, ladder=(("ozaki", 1e-7), ("fp64", None)))
    torch.cuda.synchronize()
    print(f"  E_fp64={r64['energy']:.12f} E_ladder={roz['energy']:.12f} sigma calls {roz['n_sigma']}", flush=True)
    assert roz["n_sigma"]["ozaki"] > 0
    assert abs(roz["energy"] - r64["energy"]) < 1e-10
