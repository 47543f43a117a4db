"""The split dense products of the mixed build (SNK_MIXED with a density screen and basis
screening): per tile, the functions whose largest |Phi| on the tile is below 1e-3 enter
F = P Phi (Eq. fmat) and K~ = G Phi^T (Eq. usym_k) through the FP32 matrix cores.

With the rigorous screen at a zero skip budget only blocks whose rigorous bound is zero are
skipped, so the FP64 and the split builds differ only by the FP32 products: |dE_x| must stay within the build's own rigorous
bound (stats lowprec_bound).  Real-shape systems on a subset of their grid points (K is a sum
over points, so a subset is a complete, smaller workload of the same shape)."""
import os
import sys

import numpy as np
import pytest

from paper_2303_14280_amd import snk, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg,stride", [(3, 8), (5, 64)])
def test_split_products_within_their_bound(cfg, stride):
    s = synth.make_system(cfg)
    s = s.subset_points(np.arange(0, s.npts, stride))
    kw = dict(eps_basis=1e-9, screen=snk.SNK_SCREEN_BOUND, eps_skip_energy=0.0)
    say("config %d / %d: %d points, %d functions" % (cfg, stride, s.npts, s.nbf))
    K0, st0 = snk.sn_k_build(s, **kw)
    ctx = snk.Context(s, precision=snk.SNK_MIXED, **kw)
    K1, st1 = ctx.build(s.P)
    K2, _ = ctx.build(s.P)
    dE = abs(st1["ex"] - st0["ex"])
    dK = float(np.max(np.abs(K1 - K0)))
    f32 = st1["gemm_flops_fp32"] / (st1["gemm_flops_fp32"] + st1["gemm_flops_fp64"])
    say("  FP32 share of the dense products %.3f; |dE_x| %.3e (bound %.3e); max|dK| %.3e (max|K| %.3e)" %
        (f32, dE, st1["lowprec_bound"], dK, np.max(np.abs(K0))))
    assert np.array_equal(K1, K2) and np.array_equal(K1, K1.T)
    assert st0["gemm_flops_fp32"] == 0 and st0["lowprec_bound"] == 0
    assert f32 > 0.3
    # a zero skip budget drops only blocks whose rigorous bound is zero (both builds)
    assert st1["skipped_bound"] == 0 and st0["skipped_bound"] == 0
    assert dE <= st1["lowprec_bound"]
    assert dK <= 1e-7 * np.max(np.abs(K0))


def test_split_with_learned_screen_within_budget():
    """config 3 (150 atoms) on every 4th point, the learned screen at the default budgets:
    |dE_x| <= 1e-6 Eh against the plain FP64 build."""
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        pytest.skip("no trained screener weights")
    m = snk.load_screener()
    s = synth.make_system(3)
    s = s.subset_points(np.arange(1, s.npts, 4))
    K0, st0 = snk.sn_k_build(s, eps_basis=1e-9)
    K1, st1 = snk.sn_k_build(s, eps_basis=1e-9, precision=snk.SNK_MIXED, screen=snk.SNK_SCREEN_LEARNED,
                             screener=m)
    dE = abs(st1["ex"] - st0["ex"])
    say("config 3/4 mixed+learned vs plain FP64: |dE_x| %.3e, FP32 product share %.3f, bound %.3e" %
        (dE, st1["gemm_flops_fp32"] / (st1["gemm_flops_fp32"] + st1["gemm_flops_fp64"]), st1["lowprec_bound"]))
    assert dE <= 1e-6


def test_output_tiles_give_identical_products():
    """Every output tile of the grouped products (64 x 64, 128 x 128, 64 x 128, 128 x 256) sums each
    element over k in the same order, so a mixed split build (FP64 and FP32 matrix-core
    products, F and K) is bitwise the same whichever tile every launch is forced to."""
    s = synth.make_system(3)
    s = s.subset_points(np.arange(0, s.npts, 16))
    kw = dict(eps_basis=1e-9, screen=snk.SNK_SCREEN_BOUND, eps_skip_energy=1e-6, precision=snk.SNK_MIXED)
    ctx = snk.Context(s, **kw)
    out = {}
    try:
        for tile in (0, 64, 128, 192, 384):
            snk.debug_force_tile(tile)
            out[tile] = ctx.build(s.P)
    finally:
        snk.debug_force_tile(0)
    K0, st0 = out[0]
    say("forced tiles: E_x %.12f, FP32 product share %.3f" %
        (st0["ex"], st0["gemm_flops_fp32"] / (st0["gemm_flops_fp32"] + st0["gemm_flops_fp64"])))
    assert st0["gemm_flops_fp32"] > 0
    for tile in (64, 128, 192, 384):
        assert np.array_equal(out[tile][0], K0), tile
    with pytest.raises(snk.SnkError):
        snk.debug_force_tile(96)
