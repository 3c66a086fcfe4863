"""Grouped-GEMM kernel against a plain PyTorch reference (GPU)."""
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (16, 16, 4), (64, 64, 16), (65, 63, 17), (130, 70, 33), (7, 300, 129),
          (257, 9, 400)]


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_f64_matches_reference(ctx, m, n, k, ta, tb):
    import torch
    print(f"gemm_f64 m={m} n={n} k={k} ta={ta} tb={tb}", flush=True)
    g = torch.Generator().manual_seed(m * 1000 + n * 10 + k)
    A = torch.randn(m, k, generator=g, dtype=torch.float64)
    B = torch.randn(k, n, generator=g, dtype=torch.float64)
    C0 = torch.randn(m, n, generator=g, dtype=torch.float64)
    a = (A.t().contiguous() if ta else A).cuda()
    b = (B.t().contiguous() if tb else B).cuda()
    c = C0.clone().cuda()
    ctx.debug_gemm(a, b, c, trans_a=ta, trans_b=tb, alpha=0.75, beta=1)
    torch.cuda.synchronize()
    ref = 0.75 * (A @ B) + C0
    err = (c.cpu() - ref).abs().max().item()
    scale = (A.abs() @ B.abs()).max().item() + 1.0
    assert err <= 1e-14 * k * scale, err


# BF16: each operand rounded to 8 mantissa bits -> |err| <~ 2^-7 |A||B|;
# split BF16x3 drops only lo*lo and the residual of the split -> ~2^-15.
BF_TOL = {"bf16": 1.6e-2, "bf16x3": 1.5e-4}


@pytest.mark.parametrize("m,n,k", SHAPES)
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("tile", ["0", "1", "2", "3", "4", "5"])  # 128x64, 64x64, 64x128, 128x128 (2 or 3 LDS stages), 256x256
def test_gemm_bf16_matches_reference(ctx, monkeypatch, m, n, k, ta, tb, prec, tile):
    import torch
    monkeypatch.setenv("DMRG_BF16_SHAPE", tile)
    print(f"gemm_{prec} tile={tile} m={m} n={n} k={k} ta={ta} tb={tb}", flush=True)
    g = torch.Generator().manual_seed(7 + m * 1000 + n * 10 + k)
    A = torch.randn(m, k, generator=g, dtype=torch.float64)
    B = torch.randn(k, n, generator=g, dtype=torch.float64)
    C0 = torch.randn(m, n, generator=g, dtype=torch.float64)
    a = (A.t().contiguous() if ta else A).cuda()
    b = (B.t().contiguous() if tb else B).cuda()
    c = C0.clone().cuda()
    ctx.debug_gemm(a, b, c, trans_a=ta, trans_b=tb, alpha=-1.25, beta=1, precision=prec)
    torch.cuda.synchronize()
    ref = -1.25 * (A.float() @ B.float()).double() + C0
    bound = 1.25 * (A.abs() @ B.abs())
    err = ((c.cpu() - ref).abs() / (bound + 1e-30)).max().item()
    assert err <= BF_TOL[prec], err
