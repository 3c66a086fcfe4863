"""dmrg_orbital_gradient (GPU): the DMRG-SCF orbital gradient from the
backward's RDMs, against the oracle and against rotated-integral energies.

* small windows: the library's F and g from its own dh, deri against
  oracle.orbital on the oracle's RDMs of the Fock vectors (FP64 bar 1e-10 of
  max|.|);
* 16 orbitals / 16 electrons, D = 512, middle window: the same contraction on
  the library's RDMs (bar 1e-12) and central differences of
  E(kappa) = <psi, H_eff(U^T h U, (pq|rs)') psi> with psi and the MPS held
  fixed, the operators rebuilt from the rotated integrals (bar 1e-6).
"""
import numpy as np
import pytest

from synthetic import pack_psi
from tests.helpers import case, lib_load

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _lib_grad(ctx, psi):
    import torch
    dh, deri = ctx.sigma_backward(_dev(psi), None)
    F, g = ctx.orbital_gradient(dh, deri)
    torch.cuda.synchronize()
    return dh.cpu().numpy(), deri.cpu().numpy(), F.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("K,N,tsz,D,i", [(4, 4, 0, 100, 1), (6, 6, 0, 12, 2), (7, 7, 1, 16, 2),
                                         (8, 6, 2, 30, 5), (8, 8, 0, 20, 0)])
def test_orbital_gradient_matches_oracle(ctx, K, N, tsz, D, i):
    from oracle.fock import DetSpace, rdm12
    from oracle.orbital import generalized_fock, orbital_gradient
    from oracle.projection import psi_to_fock
    from synthetic import unpack_psi
    print(f"orbital gradient vs oracle: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    n = lib_load(ctx, h, eri, m)
    psi = np.random.default_rng(K * 10 + i).normal(size=n)
    _, _, F, g = _lib_grad(ctx, psi)
    space = DetSpace.sector(K, N, tsz)
    v = psi_to_fock(m, unpack_psi(m.bonds, m.window, psi))[space.dets]
    gam, Gam = rdm12(space, v, v)
    Fr = generalized_fock(h, eri, gam, Gam)
    gr = orbital_gradient(h, eri, gam, Gam)
    assert np.max(np.abs(F - Fr)) <= 1e-10 * max(1.0, float(np.max(np.abs(Fr))))
    assert np.max(np.abs(g - gr)) <= 1e-10 * max(1.0, float(np.max(np.abs(gr))))
    assert np.allclose(g, -g.T, atol=1e-12)


def test_orbital_gradient_matches_rotated_energies_at_16_orbitals(ctx):
    from oracle.orbital import orbital_gradient, rotate_integrals
    from synthetic import mps_arrays
    print("orbital gradient vs finite differences: K=16 N=16 D=512 window=7", flush=True)
    h, eri, m = case(16, 16, 0, 512, 7)
    lib_load(ctx, h, eri, m)
    psi = pack_psi(m.bonds, m.window, m.psi)
    psi = psi / np.linalg.norm(psi)
    dh, deri, F, g = _lib_grad(ctx, psi)
    gr = orbital_gradient(h, eri, dh, 2.0 * deri)
    assert np.max(np.abs(g - gr)) <= 1e-12 * max(1.0, float(np.max(np.abs(gr))))

    def energy(kappa):
        import torch
        h2, e2 = rotate_integrals(h, eri, kappa)
        ctx.build_ops(m.window, h=h2, eri=e2, n_elec=m.n_elec, two_sz=m.two_sz,
                      mps_arrays=mps_arrays(m))
        x = _dev(psi)
        out = torch.empty_like(x)
        ctx.sigma(x, out)
        torch.cuda.synchronize()
        return float(psi @ out.cpu().numpy())

    d = 1e-5
    for (p, q) in [(1, 0), (9, 3), (15, 7)]:
        kap = np.zeros((16, 16))
        kap[p, q], kap[q, p] = d, -d
        fd = (energy(kap) - energy(-kap)) / (2 * d)
        rel = abs(fd - g[p, q]) / max(abs(g[p, q]), 1e-3)
        print(f"  kappa[{p},{q}]: fd={fd:.10f} analytic={g[p, q]:.10f} rel={rel:.1e}", flush=True)
        assert rel < 1e-6
