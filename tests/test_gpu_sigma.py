"""FP64 sigma of the HIP library against the CPU oracle (GPU).

Small windows are checked against the plain definition P^T H P psi
(oracle.projection); larger ones against the oracle's block-sparse
normal/complementary sigma, which is itself pinned to the definition on the
CPU.  Bar: ||d sigma|| / ||sigma|| <= 1e-10 and every element within
1e-10 * max|sigma| (FP64 arithmetic, rounding only).
"""
import numpy as np
import pytest

from tests.helpers import case, lib_sigma, rel_err, max_abs, lib_load, lib_sigma_flat

pytestmark = pytest.mark.gpu

TOL = 1e-10

SMALL = [  # K, N, 2Sz, D, window
    (2, 2, 0, 16, 0),
    (4, 4, 0, 100, 0), (4, 4, 0, 100, 1), (4, 4, 0, 100, 2),
    (5, 5, 1, 8, 1), (5, 4, -2, 12, 3),
    (6, 6, 0, 12, 2), (6, 5, 1, 10, 0), (6, 7, -1, 10, 4), (6, 6, 2, 12, 3),
    (8, 8, 0, 64, 3), (8, 8, 0, 20, 1), (8, 6, 2, 30, 5),
]


@pytest.mark.parametrize("K,N,tsz,D,i", SMALL)
def test_sigma_matches_projection(ctx, K, N, tsz, D, i):
    from oracle.projection import ProjectedHamiltonian
    print(f"sigma vs P^T H P: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = ProjectedHamiltonian(m, h, eri).apply(m.psi)
    got = lib_sigma(ctx, h, eri, m)
    scale = max(float(np.max(np.abs(v))) for v in ref.values())
    assert rel_err(got, ref) <= TOL
    assert max_abs(got, ref) <= TOL * scale


MID = [(12, 12, 0, 256, 5), (10, 9, 1, 200, 2), (12, 14, 2, 150, 7)]


@pytest.mark.parametrize("K,N,tsz,D,i", MID)
def test_sigma_matches_blocksparse_oracle(ctx, K, N, tsz, D, i):
    from oracle.blocksparse import BlockSparseSigma
    print(f"sigma vs block-sparse oracle: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = BlockSparseSigma(m, h, eri).apply(m.psi)
    got = lib_sigma(ctx, h, eri, m)
    scale = max(float(np.max(np.abs(v))) for v in ref.values())
    assert rel_err(got, ref) <= TOL
    assert max_abs(got, ref) <= TOL * scale


def test_sigma_is_symmetric_and_linear(ctx):
    """<x|H y> = <H x|y> and H(a x + y) = a Hx + Hy at a mid size."""
    print("sigma symmetry/linearity K=12 D=256", flush=True)
    h, eri, m = case(12, 12, 0, 256, 5)
    n = lib_load(ctx, h, eri, m)
    rng = np.random.default_rng(3)
    x, y = rng.normal(size=n), rng.normal(size=n)
    hx, hy = lib_sigma_flat(ctx, x), lib_sigma_flat(ctx, y)
    h2 = lib_sigma_flat(ctx, 0.3 * x + y)
    s = np.linalg.norm(hx) * np.linalg.norm(y)
    assert abs(x @ hy - hx @ y) <= 1e-12 * s
    assert np.linalg.norm(h2 - (0.3 * hx + hy)) <= 1e-12 * np.linalg.norm(h2)


def test_sigma_repeat_is_bitwise_deterministic(ctx):
    print("sigma determinism K=10 D=200", flush=True)
    h, eri, m = case(10, 9, 1, 200, 2)
    n = lib_load(ctx, h, eri, m)
    x = np.random.default_rng(4).normal(size=n)
    a, b = lib_sigma_flat(ctx, x), lib_sigma_flat(ctx, x)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("K,N,tsz,D,i", [(8, 8, 0, 64, 3), (12, 12, 0, 256, 5), (10, 9, 1, 200, 2)])
# 128x64, 64x64, 64x128, 128x128 (2 or 3 LDS stages), 256x256 (stage 2), per problem, 128x128 with
# 64-wide edge tiles
@pytest.mark.parametrize("tile", ["0", "1", "2", "3", "4", "5", "6", "7"])
def test_mixed_sigma_error_vs_fp64(ctx, monkeypatch, K, N, tsz, D, i, tile):
    """BF16 and split-BF16x3 sigma against the FP64 sigma of the same plan."""
    monkeypatch.setenv("DMRG_BF16_SHAPE", tile)
    print(f"mixed sigma K={K} D={D} window={i} tile={tile}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    n = lib_load(ctx, h, eri, m)
    x = np.random.default_rng(5).normal(size=n)
    x /= np.linalg.norm(x)
    s64 = lib_sigma_flat(ctx, x, "fp64")
    s16 = lib_sigma_flat(ctx, x, "bf16")
    s48 = lib_sigma_flat(ctx, x, "bf16x3")
    e16 = np.linalg.norm(s16 - s64) / np.linalg.norm(s64)
    e48 = np.linalg.norm(s48 - s64) / np.linalg.norm(s64)
    print(f"  rel err bf16 {e16:.2e} bf16x3 {e48:.2e}", flush=True)
    assert e16 < 2e-2
    assert e48 < 1e-4
    assert e48 < e16 / 20


def test_autotuned_mixed_sigma(ctx, monkeypatch):
    """The autotuner times every candidate launch configuration on the plan's
    own launches (which write the real buffers) and keeps the fastest; the
    sigma afterwards is still correct and bitwise repeatable."""
    monkeypatch.delenv("DMRG_BF16_SHAPE", raising=False)
    monkeypatch.setenv("DMRG_AUTOTUNE", "1")
    print("autotuned mixed sigma K=14 D=300 window=6", flush=True)
    h, eri, m = case(14, 14, 0, 300, 6)
    n = lib_load(ctx, h, eri, m)
    x = np.random.default_rng(6).normal(size=n)
    x /= np.linalg.norm(x)
    s64 = lib_sigma_flat(ctx, x, "fp64")
    s48 = lib_sigma_flat(ctx, x, "bf16x3")
    info = ctx.sigma_info("bf16x3")
    print(f"  tuned in {info['tune_ms']:.1f} ms: stage1 config {info['bf_config_stage1']}, "
          f"stage2 config {info['bf_config_stage2']}", flush=True)
    assert info["tune_ms"] > 0
    e48 = np.linalg.norm(s48 - s64) / np.linalg.norm(s64)
    assert e48 < 1e-4
    assert np.array_equal(s48, lib_sigma_flat(ctx, x, "bf16x3"))


# The Davidson ladder ends a split-BF16x3 stage at 3x the floor that a
# relative sigma error of 3e-6 allows (csrc/davidson.cpp, sigma_rel_error).
# Whatever launch configuration the autotuner picks, the split-BF16x3 sigma
# must stay below that error, including the 128x128 tiles that accumulate a
# whole segment list in FP32 without FP64 flushes: checked here on every tile
# shape at the largest window of this file, with the most segments per tile.
BF16X3_FLOOR = 3e-6


@pytest.mark.parametrize("tile", ["0", "1", "2", "3", "4", "5", "6", "7"])
def test_bf16x3_error_below_the_ladder_floor_for_every_tile(ctx, monkeypatch, tile):
    monkeypatch.setenv("DMRG_BF16_SHAPE", tile)
    print(f"bf16x3 error vs the ladder floor: K=14 D=300 window 6, tile {tile}", flush=True)
    h, eri, m = case(14, 14, 0, 300, 6)
    n = lib_load(ctx, h, eri, m)
    x = np.random.default_rng(7).normal(size=n)
    x /= np.linalg.norm(x)
    s64 = lib_sigma_flat(ctx, x, "fp64")
    s48 = lib_sigma_flat(ctx, x, "bf16x3")
    e48 = np.linalg.norm(s48 - s64) / np.linalg.norm(s64)
    print(f"  relative error {e48:.2e} (floor constant {BF16X3_FLOOR:.0e})", flush=True)
    assert e48 < BF16X3_FLOOR


# FP64 sigma stages run on 64 x 64 (four waves), 128 x 128, 128 x 64 or
# 64 x 128 (eight waves) tiles, chosen per stage (DMRG_F64_TILE); each shape
# in each stage against the oracle.
@pytest.mark.parametrize("tiles", ["64,64", "128,128", "64,128", "128,64", "128x64,64x128", "64x128,128x64"])
@pytest.mark.parametrize("K,N,tsz,D,i", [(12, 12, 0, 256, 5), (12, 14, 2, 150, 7)])
def test_fp64_tiles_match_blocksparse_oracle(ctx, monkeypatch, tiles, K, N, tsz, D, i):
    from oracle.blocksparse import BlockSparseSigma
    monkeypatch.setenv("DMRG_F64_TILE", tiles)
    print(f"FP64 tiles {tiles} vs oracle: K={K} N={N} 2Sz={tsz} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    ref = BlockSparseSigma(m, h, eri).apply(m.psi)
    got = lib_sigma(ctx, h, eri, m)
    scale = max(float(np.max(np.abs(v))) for v in ref.values())
    assert rel_err(got, ref) <= TOL
    assert max_abs(got, ref) <= TOL * scale


# The FP64 stages run on a direct-to-LDS kernel when every segment of a launch
# has NT operands with even leading dimensions and 16-byte aligned bases
# (else, or with DMRG_F64_LDS=0, on the register-staged kernel).  Both issue
# the same MFMA sequence, so the sigma must agree bit for bit, for each tile
# shape.
@pytest.mark.parametrize("tiles", ["128,128x64", "64,64", "64x128,128"])
@pytest.mark.parametrize("K,N,tsz,D,i", [(12, 12, 0, 256, 5), (10, 9, 1, 200, 2)])
def test_fp64_lds_kernel_is_bitwise_the_register_kernel(ctx, monkeypatch, tiles, K, N, tsz, D, i):
    monkeypatch.setenv("DMRG_F64_TILE", tiles)
    print(f"FP64 direct-to-LDS vs register-staged kernel, tiles {tiles}: K={K} D={D} window={i}", flush=True)
    h, eri, m = case(K, N, tsz, D, i)
    x = None
    out = {}
    for lds in ("1", "0"):
        monkeypatch.setenv("DMRG_F64_LDS", lds)
        n = lib_load(ctx, h, eri, m)
        if x is None:
            x = np.random.default_rng(8).normal(size=n)
        out[lds] = lib_sigma_flat(ctx, x, "fp64")
    assert np.array_equal(out["1"], out["0"])
