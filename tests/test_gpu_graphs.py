"""Graph replay of the sigma (dmrg_sigma_graphs) against launches made one by one.

Every replay is compared bitwise with the eager result of the same input;
between replays there is other eager device work and a synchronisation, and
the input and output buffers change from call to call (the graph reads its
copy-task lists from device memory, rebound on the host between calls).
"""
import numpy as np
import pytest

from synthetic import pack_psi
from tests.helpers import case, lib_load, lib_sigma_flat

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager(ctx):
    import torch
    print("sigma graph replay K=12 D=256 window=5", flush=True)
    h, eri, m = case(12, 12, 0, 256, 5)
    n = lib_load(ctx, h, eri, m)
    rng = np.random.default_rng(8)
    xs = [rng.normal(size=n) for _ in range(3)]
    precs = ("fp64", "bf16", "bf16x3")
    eager = {p: [lib_sigma_flat(ctx, x, p) for x in xs] for p in precs}
    ctx.sigma_graphs(True)
    try:
        for rep in range(3):
            for p in precs:
                for k, x in enumerate(xs):
                    got = lib_sigma_flat(ctx, x, p)
                    assert np.array_equal(got, eager[p][k]), (rep, p, k)
                    # eager work of the program and a synchronisation between replays
                    assert torch.ones(4096, device="cuda").sum().item() == 4096.0
    finally:
        ctx.sigma_graphs(False)
    # back to launches one by one
    assert np.array_equal(lib_sigma_flat(ctx, xs[0], "fp64"), eager["fp64"][0])


def test_davidson_with_graphs(ctx):
    """The Davidson solver's sigmas replay the graphs: same energy."""
    import torch
    print("davidson with graphs K=10 D=128 window=4", flush=True)
    h, eri, m = case(10, 10, 0, 128, 4)
    lib_load(ctx, h, eri, m)
    psi0 = pack_psi(m.bonds, m.window, m.psi)
    a = torch.from_numpy(psi0.copy()).cuda()
    r0 = ctx.davidson(a, tol=1e-8, ladder=(("bf16x3", 1e-4), ("fp64", None)))
    ctx.sigma_graphs(True)
    try:
        b = torch.from_numpy(psi0.copy()).cuda()
        r1 = ctx.davidson(b, tol=1e-8, ladder=(("bf16x3", 1e-4), ("fp64", None)))
    finally:
        ctx.sigma_graphs(False)
    torch.cuda.synchronize()
    print(f"  E eager {r0['energy']:.12f} graphs {r1['energy']:.12f}", flush=True)
    assert r0["iterations"] == r1["iterations"]
    assert abs(r0["energy"] - r1["energy"]) < 1e-12
