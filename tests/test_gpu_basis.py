"""Basis-function screening (Eq. basis_screen) on the GPU.

With eps_basis > 0 the batches are ordered spatially into tiles (runs of at most 16
batches inside a batch group) and tile t collocates only the functions B_t whose sphere of
radius r_cut (beyond which |phi_mu| < eps_basis) reaches the box of the tile's points.
Checks:
  * B_t contains every function that reaches eps_basis at some point of the tile, by direct
    evaluation with the oracle's collocation (the defining property of Eq. basis_screen);
  * at eps_basis = 1e-13 the dropped collocation values are below 1e-13, so K and E_x keep
    the FP64 parity bar against the unscreened oracle while most groups drop functions;
  * at the paper's operating tolerance (1e-9) |dE_x| stays below 1e-6 Eh;
  * the FP64 build, the mixed build and the screens agree on the same
    B_t, including tiles that collocate nothing, and with several tiles per group.
"""
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import snk, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def group_bytes(s, batches):
    """Device budget that makes groups of about `batches` batches (Phi, F, G in FP64)."""
    return batches * s.nbf * 256 * 24


def group_points(ctx, s, b0, b1):
    cols = ctx.point_order()[b0 * 256:b1 * 256]
    return s.grid_xyz[cols[cols >= 0]]


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_basis_sets_contain_significant_functions(eps):
    s = synth.make_system(1)
    ctx = snk.Context(s, eps_basis=eps, max_device_bytes=group_bytes(s, 6))
    tiles = ctx.tiles()
    assert sum(b1 - b0 for _, b0, b1, _ in tiles) == ctx.nbatches
    sizes, needed = [], []
    for _, b0, b1, fn in tiles:
        phi = O.collocate(s, group_points(ctx, s, b0, b1))
        need = np.nonzero(np.max(np.abs(phi), axis=1) >= eps)[0]
        missing = np.setdiff1d(need, fn)
        assert missing.size == 0, "tile %d-%d misses functions %s" % (b0, b1, missing[:10])
        assert np.all(np.diff(fn) > 0)
        sizes.append(fn.size)
        needed.append(need.size)
    say("eps_basis %.0e: %d tiles, |B_t| mean %.1f min %d (functions reaching eps: mean %.1f) of N_b %d" %
        (eps, len(tiles), np.mean(sizes), np.min(sizes), np.mean(needed), s.nbf))
    if eps >= 1e-6:
        assert np.min(sizes) < s.nbf


def test_tight_basis_screen_keeps_fp64_parity():
    g = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    s = synth.make_system(1, with_density=False).with_density(g["P"])
    flags = 0
    ctx = snk.Context(s, eps_basis=1e-13, max_device_bytes=group_bytes(s, 6), flags=flags)
    sizes = [fn.size for _, _, _, fn in ctx.tiles()]
    K, st = ctx.build(s.P)
    dE = abs(st["ex"] - float(g["ex"][0]))
    dK = float(np.max(np.abs(K - g["K"])))
    say("config1 eps_basis 1e-13 (%s): %d tiles, |B_t| mean %.1f of %d; |dE| %.2e max|dK| %.2e" %
        ("native", len(sizes), np.mean(sizes), s.nbf, dE, dK))
    assert min(sizes) < s.nbf
    assert np.array_equal(K, K.T)
    assert dE <= 1e-10
    assert dK <= 1e-11 * max(1.0, float(np.max(np.abs(g["K"]))))


def test_paper_basis_tolerance_config2():
    g = np.load(os.path.join(GOLDEN, "oracle_config2.npz"))
    s = synth.make_system(2, with_density=False).with_density(g["P"])
    ctx = snk.Context(s, eps_basis=1e-9)
    sizes = [fn.size for _, _, _, fn in ctx.tiles()]
    K, st = ctx.build(s.P)
    dE = abs(st["ex"] - float(g["ex"][0]))
    dK = float(np.max(np.abs(K - g["K"])))
    say("config2 eps_basis 1e-9: %d groups, %d tiles, |B_t| mean %.1f of %d; |dE| %.2e max|dK| %.2e" %
        (ctx.ngroups, len(sizes), np.mean(sizes), s.nbf, dE, dK))
    assert len(sizes) > ctx.ngroups
    assert np.array_equal(K, K.T)
    assert dE <= 1e-6


def test_paths_agree_with_empty_groups():
    """Two grid centres 30 bohr apart, all basis functions (compact, exponents >= 1) on the
    first: at eps_basis = 1e-6 the groups around the second centre, and the outer groups of
    the first, collocate nothing.  Two FP64 contexts and the mixed FP32-GEMM build agree, and a tolerance above every function's peak gives K = 0 exactly."""
    shells = [[(0, [3.0, 1.0], [0.5, 0.5]), (1, [2.0], [1.0]), (2, [1.5], [1.0])], []]
    s = synth.make_custom([8, 1], [[0.0, 0.0, 0.0], [0.0, 0.0, 30.0]], shells, grid=(20, 50), n_occ=2)
    kw = dict(eps_basis=1e-6, max_device_bytes=group_bytes(s, 1))
    ctx = snk.Context(s, **kw)
    sizes = np.array([fn.size for _, _, _, fn in ctx.tiles()])
    K0, st0 = ctx.build(s.P)
    K1, st1 = snk.Context(s, **kw).build(s.P)
    K2, st2 = snk.Context(s, precision=snk.SNK_MIXED, flags=snk.SNK_FP32_GEMM, **kw).build(s.P)
    Kr, exr, _ = O.snk(s)
    say("eps_basis 1e-6: %d tiles, %d empty, |B_t| max %d of %d; E_x %.12f / %.12f / %.12f, oracle %.12f" %
        (sizes.size, int(np.sum(sizes == 0)), sizes.max(), s.nbf, st0["ex"], st1["ex"], st2["ex"], exr))
    assert np.sum(sizes == 0) > 0 and sizes.max() == s.nbf
    assert np.all(np.isfinite(K0)) and np.array_equal(K0, K0.T)
    scale = float(np.max(np.abs(K0)))
    assert np.max(np.abs(K1 - K0)) <= 1e-12 * scale
    assert np.max(np.abs(K2 - K0)) <= 1e-6 * scale
    assert abs(st0["ex"] - exr) <= 1e-6
    K3, st3 = snk.sn_k_build(s, eps_basis=1e6, max_device_bytes=group_bytes(s, 1))
    assert st3["ex"] == 0.0 and not np.any(K3)


def test_mixed_and_screens_with_basis_screen():
    """config 2 (1/7 of the points, one group of several tiles) at eps_basis = 1e-9: the mixed
    FP32-GEMM build and the bound-screened build against the FP64 build on the same B_t."""
    s = synth.make_system(2)
    s = s.subset_points(np.arange(0, s.npts, 7))
    kw = dict(eps_basis=1e-9)
    K0, st0 = snk.sn_k_build(s, **kw)
    K1, st1 = snk.sn_k_build(s, precision=snk.SNK_MIXED, flags=snk.SNK_FP32_GEMM, **kw)
    K2, st2 = snk.sn_k_build(s, screen=snk.SNK_SCREEN_BOUND, eps_skip_energy=5e-7, **kw)
    e1 = abs(st1["ex"] - st0["ex"])
    e2 = abs(st2["ex"] - st0["ex"])
    say("config2/7 eps_basis 1e-9: %d groups; mixed |dE| %.2e; bound screen |dE| %.2e (bound %.2e)" %
        (st0["n_groups"], e1, e2, st2["skipped_bound"]))
    assert e1 <= 2e-7 * abs(st0["ex"])
    assert e2 <= st2["skipped_bound"] + 1e-12


def test_learned_screen_with_basis_screen():
    """config 2 with the learned screen (5e-7 Eh skip budget) and eps_basis = 1e-9: the K
    GEMM of each tile runs over the rows of its kept blocks only; |dE_x| <= 1e-6 Eh against
    the FP64 build on the same tiles."""
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        pytest.skip("no trained screener weights")
    m = snk.load_screener()
    s = synth.make_system(2)
    K0, st0 = snk.sn_k_build(s, eps_basis=1e-9)
    for flags in (0,):
        ctx = snk.Context(s, eps_basis=1e-9, screen=snk.SNK_SCREEN_LEARNED, screener=m, flags=flags)
        K1, st1 = ctx.build(s.P)
        K2, _ = ctx.build(s.P)
        assert np.array_equal(K1, K2)   # tile products run on several streams; reductions stay ordered
        dE = abs(st1["ex"] - st0["ex"])
        skipped = st1["pair_points_skipped"] / max(1, st1["pair_points_skipped"] + sum(st1["pair_points"]))
        say("config2 learned + eps_basis 1e-9 (flags %d): skipped %.3f |dE| %.2e max|dK| %.2e, kgemm %.2f ms "
            "(unscreened %.2f); per tile |B_t| %.1f, F rows %.1f, G rows %.1f" %
            (flags, skipped, dE, np.max(np.abs(K1 - K0)), st1["t_kgemm_ms"], st0["t_kgemm_ms"],
             st1["tile_functions"], st1["tile_frows"], st1["tile_grows"]))
        assert np.array_equal(K1, K1.T)
        assert dE <= 1e-6


@pytest.mark.parametrize("screen", [snk.SNK_SCREEN_NONE, snk.SNK_SCREEN_BOUND])
def test_f_rows_bound(screen):
    """Rows of F restricted per tile: F = P Phi_t on the rows L_t, and every dropped element
    (rows whose bound sum_nu |P_lam,nu| max|phi_nu| < eps_basis) is below eps_basis.  Phi and
    F of the first group from the debug hook (full rows, zeros outside B_t and L_t)."""
    s = synth.make_system(1, grid=(30, 110))
    eps = 1e-4
    ctx = snk.Context(s, eps_basis=eps, screen=screen, eps_skip_energy=1e-8, max_device_bytes=group_bytes(s, 4))
    Phi, F, G = ctx.debug_intermediates(s.P)
    ref = s.P @ Phi
    kept = np.any(F != 0.0, axis=1)
    dropped = ~kept
    say("screen %d: %d of %d rows of F computed in the first group; max dropped |P Phi| %.2e; max |dF| kept %.2e" %
        (screen, int(kept.sum()), s.nbf, np.max(np.abs(ref[dropped])) if dropped.any() else 0.0,
         np.max(np.abs(F[kept] - ref[kept]))))
    assert np.max(np.abs(F - ref)) <= eps
    assert np.max(np.abs(F[kept] - ref[kept])) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("cfg,stride,precision", [(5, 64, snk.SNK_MIXED), (5, 64, snk.SNK_FP64), (3, 16, snk.SNK_MIXED)])
def test_f_row_prefilter_is_exact(cfg, stride, precision):
    """The block prefilter of the F-row restriction (a function of centre a is tested only when
    sum_b max|P_ab| sum_{nu in B_t on b} max|phi_nu| reaches eps_basis, an upper bound of its
    own test sum) rules out only functions whose exact test fails, so the kept rows, K and E_x
    are bit for bit those of testing every function: the 1000-atom cluster with its
    molecule-local density (most blocks ruled out) and the 150-atom one with a delocalised
    density, FP64 and mixed builds, on subsets of their points."""
    s = synth.make_system(cfg)
    s = s.subset_points(np.arange(0, s.npts, stride))
    kw = dict(eps_basis=1e-9, screen=snk.SNK_SCREEN_BOUND, eps_skip_energy=1e-6, precision=precision)
    ctx = snk.Context(s, **kw)
    try:
        snk.debug_frow_prefilter(False)
        K0, st0 = ctx.build(s.P)
        snk.debug_frow_prefilter(True)
        K1, st1 = ctx.build(s.P)
    finally:
        snk.debug_frow_prefilter(True)
    say("config %d / %d, precision %d: mean F rows per tile %.1f (every function tested) and %.1f "
        "(prefiltered), E_x %.12f" % (cfg, stride, precision, st0["tile_frows"], st1["tile_frows"], st1["ex"]))
    assert st0["tile_frows"] == st1["tile_frows"]
    assert st0["gemm_flops_fp64"] == st1["gemm_flops_fp64"] and st0["gemm_flops_fp32"] == st1["gemm_flops_fp32"]
    assert st0["ex"] == st1["ex"]
    assert np.array_equal(K0, K1)
    with pytest.raises(snk.SnkError):
        snk.debug_frow_prefilter(2)
