"""dmrg_sigma_backward (GPU) against the oracle's RDMs, FCI and finite differences.

f = <lam, H_eff psi> is linear in the integrals, so its gradient is the
transition 1-RDM gamma (dh) and half the transition 2-RDM (deri) of the
full-space states P lam and P psi.

* small windows (every position, both edges): element-wise against
  oracle.fock.rdm12 of the Fock vectors (FP64 bar 1e-10 of max|.|);
* exact bond spaces at 10 orbitals / 10 electrons: the FCI RDMs;
* 16 orbitals / 16 electrons, D = 512, middle window: properties that hold at
  any size (contraction with the integrals equals <psi, sigma>, particle-number
  traces, permutation symmetries) and central finite differences with psi
  and the MPS held fixed (the integrals perturbed, operators rebuilt).
"""
import numpy as np
import pytest

from synthetic import pack_psi
from tests.helpers import case, lib_load

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _backward(ctx, psi, lam=None):
    import torch
    dh, deri = ctx.sigma_backward(_dev(psi), None if lam is None else _dev(lam))
    torch.cuda.synchronize()
    return dh.cpu().numpy(), deri.cpu().numpy()


def _sigma(ctx, psi):
    import torch
    x = _dev(psi)
    out = torch.empty_like(x)
    ctx.sigma(x, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _fock_sector(m, blocks):
    from oracle.fock import DetSpace
    from oracle.projection import psi_to_fock
    space = DetSpace.sector(m.n_orb, m.n_elec, m.two_sz)
    return space, psi_to_fock(m, blocks)[space.dets]


def _blocks(m, flat):
    from synthetic import unpack_psi
    return unpack_psi(m.bonds, m.window, flat)


SMALL = [  # K, N, 2Sz, D, window
    (4, 4, 0, 100, 0), (4, 4, 0, 100, 1), (4, 4, 0, 100, 2),
    (5, 5, 1, 8, 1), (5, 4, -2, 12, 3),
    (6, 6, 0, 12, 2), (6, 5, 1, 10, 0), (6, 7, -1, 10, 4), (6, 6, 2, 12, 3),
    (7, 7, 1, 16, 2), (8, 8, 0, 20, 3), (8, 6, 2, 30, 5),
]


@pytest.mark.parametrize("K,N,tsz,D,i", SMALL)
def test_backward_matches_oracle_rdms(ctx, K, N, tsz, D, i):
    from oracle.fock import rdm12
    print(f"backward vs transition RDMs: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    n = lib_load(ctx, h, eri, m)
    rng = np.random.default_rng(K * 100 + i)
    psi, lam = rng.normal(size=n), rng.normal(size=n)
    dh, deri = _backward(ctx, psi, lam)
    space, vk = _fock_sector(m, _blocks(m, psi))
    _, vb = _fock_sector(m, _blocks(m, lam))
    g, G = rdm12(space, vb, vk)
    sg = max(1.0, float(np.max(np.abs(g))))
    sG = max(1.0, float(np.max(np.abs(G))))
    assert np.max(np.abs(dh - g)) <= TOL * sg
    assert np.max(np.abs(deri - 0.5 * G)) <= TOL * sG
    # sigma_bar = NULL means psi
    dh2, deri2 = _backward(ctx, psi)
    g2, G2 = rdm12(space, vk, vk)
    assert np.max(np.abs(dh2 - g2)) <= TOL * max(1.0, float(np.max(np.abs(g2))))
    assert np.max(np.abs(deri2 - 0.5 * G2)) <= TOL * max(1.0, float(np.max(np.abs(G2))))


def test_backward_equals_fci_rdms_with_exact_bonds(ctx):
    """10 orbitals, 10 electrons, bond spaces complete at the middle window:
    the Davidson vector is the FCI state and gamma, Gamma are its RDMs."""
    import torch
    from oracle.fock import fci, rdm12
    print("backward vs FCI RDMs: K=10 N=10 D=1024 window=4", flush=True)
    h, eri, m = case(10, 10, 0, 1024, 4)
    n = lib_load(ctx, h, eri, m)
    psi = _dev(pack_psi(m.bonds, m.window, m.psi))
    r = ctx.davidson(psi, tol=1e-10, max_iter=400)
    torch.cuda.synchronize()
    e = r["energy"]
    w, v, space = fci(10, 10, 0, h, eri)
    print(f"  E_dmrg={e:.12f} E_fci={w[0]:.12f} residual={r['residual']:.2e}", flush=True)
    assert abs(e - w[0]) < 1e-9
    dh, deri = _backward(ctx, psi.cpu().numpy())
    g, G = rdm12(space, v[:, 0], v[:, 0])
    err_g = float(np.max(np.abs(dh - g)))
    err_G = float(np.max(np.abs(2 * deri - G)))
    print(f"  max|gamma - gamma_FCI| = {err_g:.2e}, max|Gamma - Gamma_FCI| = {err_G:.2e}", flush=True)
    assert err_g < 1e-8
    assert err_G < 1e-8
    # total spin of the GPU state from its 2-RDM: <S^2> = -N(N-4)/4 - 1/2 sum_pq Gamma_pqqp,
    # against the oracle's S_- S_+ + S_z(S_z + 1) on the FCI vector; an eigenstate, S(S+1)
    from oracle.fock import s_squared
    N = 10
    s2 = -N * (N - 4) / 4 - 0.5 * float(np.einsum("pqqp->", 2 * deri))
    s2_fci = s_squared(space, v[:, 0])
    S = (-1 + np.sqrt(1 + 4 * max(s2, 0.0))) / 2
    print(f"  <S^2> from the GPU 2-RDM {s2:.3e}, FCI {s2_fci:.3e}, S = {S:.6f}", flush=True)
    assert abs(s2 - s2_fci) < 1e-7
    assert abs(S - round(S)) < 1e-6


def _c4(ctx):
    h, eri, m = case(16, 16, 0, 512, 7)
    n = lib_load(ctx, h, eri, m)
    psi = pack_psi(m.bonds, m.window, m.psi)
    psi = psi / np.linalg.norm(psi)
    return h, eri, m, psi


def test_backward_identities_at_16_orbitals(ctx):
    print("backward identities: K=16 N=16 D=512 window=7", flush=True)
    h, eri, m, psi = _c4(ctx)
    N = m.n_elec
    dh, deri = _backward(ctx, psi)
    E = float(psi @ _sigma(ctx, psi))
    contr = float(np.sum(h * dh) + np.sum(eri * deri))
    print(f"  <psi,H psi> = {E:.15f}, contraction = {contr:.15f}", flush=True)
    assert abs(contr - E) <= 1e-12 * abs(E) + 1e-12
    assert abs(np.trace(dh) - N) < 1e-11
    assert abs(np.einsum("pprr->", deri) - 0.5 * N * (N - 1)) < 1e-10
    assert np.allclose(np.einsum("pqrr->pq", deri), 0.5 * (N - 1) * dh, atol=1e-11)
    assert np.allclose(dh, dh.T, atol=1e-12)
    assert np.allclose(deri, deri.transpose(2, 3, 0, 1), atol=1e-12)
    assert np.allclose(deri, deri.transpose(1, 0, 3, 2), atol=1e-12)


def _orbit(p, q, r, s):
    """The 8 index tuples that real 8-fold symmetry ties to (pq|rs)."""
    return {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}


def test_backward_matches_finite_differences_at_16_orbitals(ctx):
    """Central differences of E = <psi, H_eff psi> at fixed psi and MPS, the
    integrals perturbed symmetrically (h: the (p,q),(q,p) pair; eri: the
    whole 8-fold orbit) and the operators rebuilt: bar 1e-6 relative."""
    print("backward vs finite differences: K=16 N=16 D=512 window=7", flush=True)
    h, eri, m, psi = _c4(ctx)
    dh, deri = _backward(ctx, psi)
    d = 1e-5
    from synthetic import mps_arrays

    def energy(hh, ee):
        ctx.build_ops(m.window, h=hh, eri=ee, n_elec=m.n_elec, two_sz=m.two_sz,
                      mps_arrays=mps_arrays(m))
        return float(psi @ _sigma(ctx, psi))

    rng = np.random.default_rng(5)
    worst = 0.0
    for (p, q) in [(0, 0), (3, 11), (7, 8), (15, 2)]:
        hp, hm = h.copy(), h.copy()
        for (a, b) in {(p, q), (q, p)}:
            hp[a, b] += d
            hm[a, b] -= d
        fd = (energy(hp, eri) - energy(hm, eri)) / (2 * d)
        an = sum(dh[a, b] for (a, b) in {(p, q), (q, p)})
        rel = abs(fd - an) / max(abs(an), 1e-3)
        worst = max(worst, rel)
        print(f"  h[{p},{q}]: fd={fd:.10f} analytic={an:.10f} rel={rel:.1e}", flush=True)
        assert rel < 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 4), (7, 8, 7, 8), (6, 7, 8, 9), tuple(rng.integers(0, 16, 4))]:
        orb = _orbit(*[int(x) for x in idx])
        ep, em = eri.copy(), eri.copy()
        for t in orb:
            ep[t] += d
            em[t] -= d
        fd = (energy(h, ep) - energy(h, em)) / (2 * d)
        an = sum(deri[t] for t in orb)
        rel = abs(fd - an) / max(abs(an), 1e-3)
        worst = max(worst, rel)
        print(f"  eri{idx}: fd={fd:.10f} analytic={an:.10f} rel={rel:.1e}", flush=True)
        assert rel < 1e-6
    print(f"  worst relative FD error {worst:.1e}", flush=True)


def test_autograd_function(ctx):
    """DMRGEnergy: E and its gradients with respect to (h, eri, psi)."""
    import torch
    from paper_2603_28648_amd import DMRGEnergy
    print("DMRGEnergy autograd: K=6 N=6 D=12 window=2", flush=True)
    h, eri, m = case(6, 6, 0, 12, 2)
    lib_load(ctx, h, eri, m)
    psi0 = pack_psi(m.bonds, m.window, m.psi)
    ht = _dev(h).requires_grad_()
    et = _dev(eri).requires_grad_()
    pt = _dev(psi0).requires_grad_()
    E = DMRGEnergy.apply(ht, et, pt, ctx)
    E.backward()
    dh, deri = _backward(ctx, psi0)
    sig = _sigma(ctx, psi0)
    assert abs(E.item() - psi0 @ sig) < 1e-12 * max(1.0, abs(E.item()))
    assert np.allclose(ht.grad.cpu().numpy(), dh, atol=1e-13)
    assert np.allclose(et.grad.cpu().numpy(), deri, atol=1e-13)
    assert np.allclose(pt.grad.cpu().numpy(), 2 * sig, atol=1e-12)


# Mixed variant: the adjoint contractions on the BF16 kernel, FP64
# accumulation of the gradient.  Tolerance from the arithmetic: a split-BF16x3
# product carries a relative error of about 2^-16 per operand pair (hi/lo
# representation, dropped lo*lo), FP32 accumulation adds up to k * 2^-24 over
# a block contraction (k <= a few hundred), and the chain composes K/2 such
# steps; 1e-4 of max|.| covers that with margin.  Plain BF16 (2^-8 per
# operand) gets 3e-2.
MIXED_TOL = {"bf16x3": 1e-4, "bf16": 3e-2}


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("K,N,tsz,D,i", [(4, 4, 0, 100, 2), (6, 7, -1, 10, 4), (8, 6, 2, 30, 5), (8, 8, 0, 20, 3)])
def test_mixed_backward_matches_fp64(ctx, prec, K, N, tsz, D, i):
    import torch
    print(f"{prec} backward vs FP64: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    n = lib_load(ctx, h, eri, m)
    rng = np.random.default_rng(K * 100 + i)
    psi, lam = rng.normal(size=n), rng.normal(size=n)
    dh, deri = _backward(ctx, psi, lam)
    mh, me = ctx.sigma_backward(_dev(psi), _dev(lam), precision=prec)
    torch.cuda.synchronize()
    mh, me = mh.cpu().numpy(), me.cpu().numpy()
    eh = np.max(np.abs(mh - dh)) / max(1.0, float(np.max(np.abs(dh))))
    ee = np.max(np.abs(me - deri)) / max(1.0, float(np.max(np.abs(deri))))
    print(f"  relative error: dh {eh:.2e}, deri {ee:.2e}", flush=True)
    assert eh <= MIXED_TOL[prec] and ee <= MIXED_TOL[prec]
    assert eh > 0 or ee > 0  # the BF16 kernel did run


def test_mixed_backward_at_16_orbitals(ctx):
    """16o/16e D=512: split-BF16x3 backward against the FP64 one, the Euler
    identity and central differences (the FP64 bar of 1e-6 does not apply:
    the stated bar is MIXED_TOL)."""
    import time
    import torch
    print("bf16x3 backward at K=16 N=16 D=512 window=7", flush=True)
    h, eri, m, psi = _c4(ctx)
    t0 = time.perf_counter()
    dh, deri = _backward(ctx, psi)
    t1 = time.perf_counter()
    mh, me = ctx.sigma_backward(_dev(psi), None, precision="bf16x3")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mh, me = mh.cpu().numpy(), me.cpu().numpy()
    eh = np.max(np.abs(mh - dh)) / float(np.max(np.abs(dh)))
    ee = np.max(np.abs(me - deri)) / float(np.max(np.abs(deri)))
    E = float(psi @ _sigma(ctx, psi))
    contr = float(np.sum(h * mh) + np.sum(eri * me))
    print(f"  FP64 {1e3 * (t1 - t0):.0f} ms, bf16x3 {1e3 * (t2 - t1):.0f} ms; relative error dh {eh:.2e}, "
          f"deri {ee:.2e}; Euler identity {abs(contr - E) / abs(E):.2e}", flush=True)
    assert eh <= MIXED_TOL["bf16x3"] and ee <= MIXED_TOL["bf16x3"]
    assert abs(contr - E) <= MIXED_TOL["bf16x3"] * abs(E)
    assert abs(np.trace(mh) - m.n_elec) <= MIXED_TOL["bf16x3"] * m.n_elec
