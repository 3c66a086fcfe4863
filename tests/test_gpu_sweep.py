"""Two-site DMRG sweeps on the GPU against full CI (8 orbitals, 8 electrons).

At D = 256 every bond space is complete, so the sweeps must reach the FCI
energy; at D = 64 the energy must stay variational (>= E_FCI) and decrease
from half-sweep to half-sweep (GPU)."""
import numpy as np
import pytest

from synthetic import make_integrals, make_mps, mps_arrays, pack_psi

pytestmark = pytest.mark.gpu


def _run(ctx, D, D_init, n_sweeps):
    import torch
    h, eri = make_integrals(8, 8)
    m = make_mps(8, 8, 0, D_init, 0, 1008)
    ctx.build_ops(0, h=h, eri=eri, n_elec=8, two_sz=0, mps_arrays=mps_arrays(m))
    psi = torch.from_numpy(pack_psi(m.bonds, 0, m.psi)).cuda()
    E, eps, _ = ctx.sweep(psi, n_sweeps, D, tol=1e-8)
    # every window's eigensolver reached its tolerance
    assert all(hs["unconverged"] == 0 for hs in ctx.last_halves), ctx.last_halves
    return h, eri, E, eps


def test_sweeps_reach_fci_at_complete_bond_dimension(ctx):
    from oracle.fock import fci
    print("sweeps K=8 D=256 vs FCI", flush=True)
    h, eri, E, eps = _run(ctx, 256, 256, 3)
    e_fci = fci(8, 8, 0, h, eri)[0][0]
    print(f"  E per half-sweep {[round(e, 12) for e in E]} FCI {e_fci:.12f}", flush=True)
    assert abs(E[-1] - e_fci) < 1e-9
    assert max(eps[-2:]) < 1e-12


def test_sweeps_at_d64_are_variational_and_monotone(ctx):
    from oracle.fock import fci
    print("sweeps K=8 D=64 x10", flush=True)
    h, eri, E, eps = _run(ctx, 64, 64, 10)
    e_fci = fci(8, 8, 0, h, eri)[0][0]
    print(f"  E per half-sweep {[round(e, 10) for e in E]} FCI {e_fci:.10f} eps {eps[-1]:.2e}", flush=True)
    assert E[-1] >= e_fci - 1e-10
    assert all(E[k + 1] <= E[k] + 1e-9 for k in range(len(E) - 1))
    assert E[-1] - e_fci < 5e-3


def test_refined_sweeps_reach_fci_at_complete_bond_dimension(ctx):
    """Sweeps whose window solves run split-BF16x3 and then residual
    refinement (FP64 residuals, corrections on split-BF16x3) reach full CI."""
    import torch
    from oracle.fock import fci
    print("sweeps K=8 D=256, split-BF16x3 + refinement, vs FCI", flush=True)
    h, eri = make_integrals(8, 8)
    m = make_mps(8, 8, 0, 256, 0, 1008)
    ctx.build_ops(0, h=h, eri=eri, n_elec=8, two_sz=0, mps_arrays=mps_arrays(m))
    psi = torch.from_numpy(pack_psi(m.bonds, 0, m.psi)).cuda()
    E, eps, _ = ctx.sweep(psi, 3, 256, tol=1e-8, ladder=(("bf16x3", 1e-4), ("fp64", None)), refine=True)
    assert all(hs["unconverged"] == 0 for hs in ctx.last_halves)
    e_fci = fci(8, 8, 0, h, eri)[0][0]
    print(f"  E per half-sweep {[round(e, 12) for e in E]} FCI {e_fci:.12f}", flush=True)
    assert abs(E[-1] - e_fci) < 1e-9
