"""dmrg_sigma_noalloc against dmrg_sigma (GPU).

The no-allocation entry point runs the FP64 sigma with its stage-1 workspace
in the library's fixed per-GPU scratch array.  It must give the result of
dmrg_sigma (same kernels and order, so the bar is FP64 parity: 1e-12
relative, and in practice bit-identical) on two calls in a row, the second
on a smaller window (the scratch then holds the first call's data), and
refuse a window whose workspace exceeds the scratch.
"""
import os

import numpy as np
import pytest

from synthetic import pack_psi
from tests.helpers import case, lib_load, lib_sigma_flat

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module")
def small_ws():
    """A context whose stage-1 workspace is chunked to 16 MiB (below the scratch)."""
    import torch
    from paper_2603_28648_amd import Context
    old = os.environ.get("DMRG_WS_BUDGET_MB")
    os.environ["DMRG_WS_BUDGET_MB"] = "16"
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


def _noalloc(ctx, flat):
    import torch
    psi = torch.from_numpy(np.ascontiguousarray(flat)).cuda()
    out = torch.full_like(psi, np.nan)
    ctx.sigma_noalloc(psi, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _check(ctx, K, N, tsz, D, i):
    print(f"sigma_noalloc vs sigma: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    lib_load(ctx, h, eri, m)
    info = ctx.sigma_info()
    print(f"  workspace {info['workspace_bytes'] / 2**20:.1f} MiB per chunk, {info['n_chunks']} chunks",
          flush=True)
    assert info["workspace_bytes"] <= SCRATCH_BYTES
    flat = pack_psi(m.bonds, i, m.psi)
    ref = lib_sigma_flat(ctx, flat, "fp64")
    got = _noalloc(ctx, flat)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"  relative difference {rel:.2e}, bit-identical {np.array_equal(got, ref)}", flush=True)
    assert rel <= 1e-12
    # a second vector on the same buffers' window
    x = np.random.default_rng(K).normal(size=flat.size)
    rx = lib_sigma_flat(ctx, x)
    assert np.linalg.norm(_noalloc(ctx, x) - rx) <= 1e-12 * np.linalg.norm(rx)
    return info


def test_noalloc_sigma_equals_sigma_then_smaller_window(small_ws):
    """Two calls in a row, the second on a smaller window: the scratch then
    still holds the first window's intermediates."""
    a = _check(small_ws, 12, 12, 0, 256, 5)
    b = _check(small_ws, 8, 6, 2, 30, 5)
    assert a["n_chunks"] >= 2
    assert b["workspace_bytes"] < a["workspace_bytes"]


def test_noalloc_refuses_a_workspace_above_the_scratch(ctx):
    from paper_2603_28648_amd import DMRGError
    print("sigma_noalloc beyond the scratch: K=12 D=256 window 5, default workspace budget", flush=True)
    h, eri, m = case(12, 12, 0, 256, 5)
    lib_load(ctx, h, eri, m)
    info = ctx.sigma_info()
    print(f"  workspace {info['workspace_bytes'] / 2**20:.1f} MiB", flush=True)
    assert info["workspace_bytes"] > SCRATCH_BYTES
    with pytest.raises(DMRGError) as e:
        _noalloc(ctx, pack_psi(m.bonds, 5, m.psi))
    assert e.value.status == -2 and "scratch" in str(e.value)
