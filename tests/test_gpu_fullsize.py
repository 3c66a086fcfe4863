"""The sigma at the full benchmark shapes, in the launch configuration the
benchmark times (autotuned BF16 tiles, graph replay):
* CAS(54,36) (36 orbitals, 54 electrons), bond dimension 4096, middle window
  (17, 18), at 2S_z = 0 (the headline) and 2S_z = 4 (the S_z = 2 state);
* CAS(22,22) (22 orbitals and electrons, 2S_z = 0), bond dimension 1024,
  middle window (10, 11).

The oracle cannot build environments at D = 4096 in reasonable time, so
these tests check properties that hold at any size:

* a number-operator Hamiltonian, h = c 1 and (pq|rs) = u d_pq d_rs, gives
  H = c N + u N (N - 1) / 2 exactly (the two-body sum over all spin orbitals
  of a+_p a+_q a_q a_p is N^2 - N), so sigma = lambda psi element by element;
* H_eff is symmetric: <x|H y> = <H x|y> for random x, y (a transposed or
  mis-signed operand in one stage breaks it);
* the mixed and emulated precisions against the FP64 sigma, within the
  accuracy each one is built for, and the Rayleigh quotient within that
  relative accuracy of |E| (1e-6 Eh for the Ozaki sigma);
* graph replays are bit-identical to launch-by-launch execution.
"""
import numpy as np
import pytest

from synthetic import make_integrals, make_mps, mps_arrays, pack_psi

pytestmark = pytest.mark.gpu

# K, N, 2Sz, D, window, integral seed, MPS seed
CONFIGS = {"cas54_36": (36, 54, 0, 4096, 17, 36, 1036),
           "cas54_36_sz2": (36, 54, 4, 4096, 17, 36, 1036),
           "cas22_22": (22, 22, 0, 1024, 10, 22, 1022)}

# number-operator Hamiltonian: h = NUMBER_C 1, (pq|rs) = NUMBER_U d_pq d_rs
NUMBER_C, NUMBER_U = 0.3, 0.01
# relative tolerances against the FP64 sigma (norm-wise)
# (split-BF16x3: the 3e-6 relative error the Davidson ladder assumes for it)
REL_TOL = {"bf16": 3e-3, "bf16x3": 3e-6, "ozaki": 1e-12}


@pytest.fixture(scope="module", params=list(CONFIGS))
def big(request):
    """A context of its own (freed after the configuration's tests) with the
    operators of one benchmark workload."""
    import torch
    from paper_2603_28648_amd import Context
    K, N, TSZ, D, WINDOW, ISEED, MSEED = CONFIGS[request.param]
    print(f"full-size sigma: K={K} N={N} 2Sz={TSZ} D={D} window={WINDOW}", flush=True)
    m = make_mps(K, N, TSZ, D, WINDOW, MSEED)
    c = Context(0)
    state = {"ctx": c, "mps": m, "ops": None, "cfg": CONFIGS[request.param]}
    yield state
    torch.cuda.synchronize()
    c.close()


def _load(state, name):
    """Build the window's operators for the synthetic integrals ("real") or
    the number-operator Hamiltonian ("number"), unless they are loaded."""
    if state["ops"] == name:
        return
    K, N, TSZ, D, WINDOW, ISEED, MSEED = state["cfg"]
    if name == "real":
        h, eri = make_integrals(K, ISEED)
    else:
        h, eri = NUMBER_C * np.eye(K), np.zeros((K, K, K, K))
        idx = np.arange(K)
        eri[idx[:, None], idx[:, None], idx[None, :], idx[None, :]] = NUMBER_U
    c, m = state["ctx"], state["mps"]
    c.build_ops(WINDOW, h=h, eri=eri, n_elec=N, two_sz=TSZ, mps_arrays=mps_arrays(m))
    assert c.psi_size() == m.psi_size()
    state["ops"] = name


def _sigma(c, x, prec):
    import torch
    out = torch.empty_like(x)
    c.sigma(x, out, prec)
    torch.cuda.synchronize()
    return out


def test_fullsize_number_operator_closed_form(big):
    import torch
    _load(big, "number")
    c, m = big["ctx"], big["mps"]
    K, N, TSZ, D, WINDOW = big["cfg"][:5]
    lam = NUMBER_C * N + 0.5 * NUMBER_U * N * (N - 1)
    psi = torch.from_numpy(pack_psi(m.bonds, WINDOW, m.psi)).cuda()
    psi /= torch.linalg.norm(psi)
    want = lam * psi
    for prec, tol in (("fp64", 1e-12), ("ozaki", 1e-12), ("bf16x3", REL_TOL["bf16x3"])):
        got = _sigma(c, psi, prec)
        rel = float(torch.linalg.norm(got - want) / torch.linalg.norm(want))
        worst = float(torch.max(torch.abs(got - want)) / torch.max(torch.abs(want)))
        print(f"  number operator, {prec}: |sigma - lambda psi| / |lambda psi| = {rel:.2e}, "
              f"max element error / max |lambda psi| = {worst:.2e}", flush=True)
        assert rel < tol
        assert worst < 10 * tol


def test_fullsize_symmetry_and_precisions(big):
    import torch
    _load(big, "real")
    c, m = big["ctx"], big["mps"]
    WINDOW = big["cfg"][4]
    psi = torch.from_numpy(pack_psi(m.bonds, WINDOW, m.psi)).cuda()
    psi /= torch.linalg.norm(psi)
    s64 = _sigma(c, psi, "fp64")
    e64 = float(psi @ s64)
    # H_eff symmetric: <x|H y> = <H x|y>
    g = torch.Generator(device="cpu").manual_seed(17)
    x = torch.randn(psi.numel(), generator=g, dtype=torch.float64).cuda()
    y = torch.randn(psi.numel(), generator=g, dtype=torch.float64).cuda()
    for prec, tol in (("fp64", 1e-12), ("bf16x3", 1e-5)):
        hx, hy = _sigma(c, x, prec), _sigma(c, y, prec)
        a, b = float(x @ hy), float(hx @ y)
        scale = float(torch.linalg.norm(x) * torch.linalg.norm(hy))
        print(f"  symmetry, {prec}: <x|Hy> = {a:.12e}, <Hx|y> = {b:.12e}, "
              f"difference / (|x||Hy|) = {abs(a - b) / scale:.2e}", flush=True)
        assert abs(a - b) <= tol * scale
    # the mixed and emulated precisions against FP64
    for prec in ("bf16x3", "bf16", "ozaki"):
        s = _sigma(c, psi, prec)
        rel = float(torch.linalg.norm(s - s64) / torch.linalg.norm(s64))
        de = abs(float(psi @ s) - e64)
        print(f"  {prec} against FP64: relative {rel:.2e}, Rayleigh quotient difference {de:.2e} Eh",
              flush=True)
        assert rel < REL_TOL[prec]
        # the Rayleigh quotient carries at most the precision's relative error
        # (the FP64 energy itself comes from the FP64 stage of the ladder; a
        # single split-BF16x3 quotient moves by ~1e-6 Eh at |E| ~ 440 Eh)
        assert de <= REL_TOL[prec] * abs(e64)
        if prec == "ozaki":
            assert de < 1e-6


def test_fullsize_graph_replay_bitwise(big):
    import torch
    _load(big, "real")
    c, m = big["ctx"], big["mps"]
    WINDOW = big["cfg"][4]
    psi = torch.from_numpy(pack_psi(m.bonds, WINDOW, m.psi)).cuda()
    for prec in ("bf16x3", "fp64"):
        c.sigma_graphs(False)
        eager = _sigma(c, psi, prec).clone()
        c.sigma_graphs(True)
        r1 = _sigma(c, psi, prec).clone()
        r2 = _sigma(c, psi, prec)
        c.sigma_graphs(False)
        print(f"  graph replays, {prec}: identical to eager: {bool(torch.equal(r1, eager))}, "
              f"{bool(torch.equal(r2, eager))}", flush=True)
        assert torch.equal(r1, eager) and torch.equal(r2, eager)
