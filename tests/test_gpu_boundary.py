"""The boundary calls beyond the sigma (GPU): MPS out, energy, error states.

* dmrg_get_bond / dmrg_get_site return the MPS the context holds in the
  dmrg_mps layout: after loading, exactly the tensors passed in.
* dmrg_energy: psi^T H_eff psi + e_core psi^T psi and its psi gradient
  2 (sigma + e_core psi), against the oracle's P^T H P; it refuses integrals
  that differ from the ones the operators were built from, and DMRGEnergy
  (the autograd function) goes through it.
* Calls made in the wrong state return DMRG_ERR_STATE, calls with bad
  arguments DMRG_ERR_INVALID_ARG, on a live context.
"""
import numpy as np
import pytest

from synthetic import mps_arrays, pack_psi
from tests.helpers import case, lib_load

pytestmark = pytest.mark.gpu

INVALID_ARG, STATE = -1, -7


def test_get_bond_and_site_return_the_loaded_mps(ctx):
    print("get_bond / get_site round trip: K=8 N=8 D=30 window 3", flush=True)
    h, eri, m = case(8, 8, 0, 30, 3)
    lib_load(ctx, h, eri, m)
    a = mps_arrays(m)
    for b in range(9):
        assert ctx.get_bond(b) == [tuple(s) for s in m.bonds[b]]
    for s in range(8):
        if s in (3, 4):
            continue
        assert np.array_equal(ctx.get_site(s), a["sites"][s])


def test_energy_matches_projection_and_checks_integrals(ctx):
    import torch
    from oracle.projection import ProjectedHamiltonian
    from paper_2603_28648_amd import DMRGError
    print("dmrg_energy vs P^T H P: K=6 N=6 D=12 window 2, e_core 1.5", flush=True)
    h, eri, m = case(6, 6, 0, 12, 2)
    ctx.build_ops(2, h=h, eri=eri, n_elec=6, two_sz=0, mps_arrays=mps_arrays(m), e_core=1.5)
    flat = pack_psi(m.bonds, 2, m.psi) * 0.7
    ref_sig = pack_psi(m.bonds, 2, ProjectedHamiltonian(m, h, eri).apply(
        {k: 0.7 * v for k, v in m.psi.items()}))
    psi = torch.from_numpy(flat).cuda()
    sig = torch.empty_like(psi)
    grad = torch.empty_like(psi)
    e, n2 = ctx.energy(psi, h=h, eri=eri, sigma=sig, grad=grad)
    want = flat @ ref_sig + 1.5 * (flat @ flat)
    print(f"  energy {e:.14f} oracle {want:.14f}", flush=True)
    assert abs(e - want) <= 1e-12 * abs(want)
    assert abs(n2 - flat @ flat) <= 1e-14 * (flat @ flat)
    assert np.max(np.abs(sig.cpu().numpy() - ref_sig)) <= 1e-12 * np.max(np.abs(ref_sig))
    g = 2 * (ref_sig + 1.5 * flat)
    assert np.max(np.abs(grad.cpu().numpy() - g)) <= 1e-12 * np.max(np.abs(g))
    h2 = h.copy()
    h2[1, 2] += 1e-6
    h2[2, 1] += 1e-6
    with pytest.raises(DMRGError) as err:
        ctx.energy(psi, h=h2, eri=eri)
    assert err.value.status == INVALID_ARG and "differ" in str(err.value)
    e2 = eri.copy()
    e2 *= 1 + 1e-9
    with pytest.raises(DMRGError):
        ctx.energy(psi, h=h, eri=e2)


def test_dmrg_energy_autograd_refuses_other_integrals(ctx):
    import torch
    from paper_2603_28648_amd import DMRGEnergy, DMRGError
    print("DMRGEnergy with integrals other than the built ones", flush=True)
    h, eri, m = case(6, 6, 0, 12, 2)
    lib_load(ctx, h, eri, m)
    psi = torch.from_numpy(pack_psi(m.bonds, 2, m.psi)).cuda().requires_grad_()
    ht = torch.from_numpy(h + 0.01 * np.eye(6)).cuda().requires_grad_()
    et = torch.from_numpy(eri).cuda().requires_grad_()
    with pytest.raises(DMRGError):
        DMRGEnergy.apply(ht, et, psi, ctx)


def test_wrong_state_and_bad_arguments_on_a_live_context():
    import ctypes
    import torch
    from paper_2603_28648_amd import Context, DMRGError
    print("error states on a fresh context", flush=True)
    c = Context(0)
    try:
        x = torch.zeros(8, dtype=torch.float64, device="cuda")
        for f in (lambda: c.sigma(x, x), lambda: c.psi_size(), lambda: c.get_psi(x),
                  lambda: c.debug_diag(x), lambda: c.get_bond(0), lambda: c.get_site(0)):
            with pytest.raises(DMRGError) as e:
                f()
            assert e.value.status == STATE, str(e.value)
        h, eri, m = case(6, 6, 0, 12, 2)
        lib_load(c, h, eri, m)
        for f in (lambda: c.get_site(2), lambda: c.get_site(3), lambda: c.get_psi(x)):
            with pytest.raises(DMRGError) as e:
                f()
            assert e.value.status == STATE, str(e.value)
        lib = c.lib
        for st in (lib.dmrg_sigma(c.h, None, None, 0),
                   lib.dmrg_sigma(c.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 7),
                   lib.dmrg_truncate(c.h, ctypes.c_void_p(x.data_ptr()), 2, 4, 0.0, None, None),
                   lib.dmrg_truncate(c.h, ctypes.c_void_p(x.data_ptr()), 1, 0, 0.0, None, None),
                   lib.dmrg_get_bond(c.h, 99, 0, ctypes.byref(ctypes.c_int32()), None, None, None),
                   lib.dmrg_sigma_graphs(c.h, 5)):
            assert st == INVALID_ARG
        torch.cuda.synchronize()
    finally:
        c.close()
