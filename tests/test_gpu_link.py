"""The paper's pair selection (SNK_SCREEN_LINK, Eq. sp_set) on the GPU.

A block (A, B) of batch j is kept when the energy estimate Ft_A Ft_B At_AB or the
exchange-matrix estimate max(Ft_A, Ft_B) phit_j At_AB reaches the threshold (the paper uses
1e-9 for both).  These are estimates, not bounds: the screen also reports the rigorous bound
on the energy of the blocks it drops (sum of c_AB U_A U_B, U from Cauchy-Schwarz with A(r)
positive semi-definite), which holds but is loose for distant pairs.  Checks against the
FP64 oracle (configs 1 and 2) or the FP64 GPU build:
  * threshold 0 keeps every block: the FP64 parity bar;
  * the paper's threshold 1e-9: |dE_x| <= 1e-6 Eh (the bar of the reduced forms), K symmetric;
  * larger thresholds skip more; every change stays within the reported bound;
  * the kept pair set of every batch equals the oracle's Eq. sp_set selection (F-tilde from
    |D| Phi-tilde, Eq. exx_fmat_approx), apart from decisions within rounding of the threshold.
"""
import os
import sys

import numpy as np
import pytest

from oracle import link_ref as LR
from paper_2303_14280_amd import snk, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def skipped_fraction(st):
    return st["pair_points_skipped"] / max(1, st["pair_points_skipped"] + sum(st["pair_points"]))


@pytest.mark.parametrize("cfg,eps", [(1, 0.0), (1, 1e-9), (1, 1e-6), (2, 0.0), (2, 1e-9), (2, 1e-7)])
def test_link_against_oracle(cfg, eps):
    g = np.load(os.path.join(GOLDEN, "oracle_config%d.npz" % cfg))
    s = synth.make_system(cfg, with_density=False).with_density(g["P"])
    K, st = snk.sn_k_build(s, screen=snk.SNK_SCREEN_LINK, eps_skip_energy=eps)
    dE = abs(st["ex"] - float(g["ex"][0]))
    say("config %d link eps %.0e: skipped %.4f, |dE| %.2e, reported bound %.2e, max|dK| %.2e, afg %.2f ms" %
        (cfg, eps, skipped_fraction(st), dE, st["skipped_bound"], np.max(np.abs(K - g["K"])), st["t_afg_ms"]))
    assert np.array_equal(K, K.T)
    assert dE <= st["skipped_bound"] + 1e-10
    if eps == 0.0:
        assert st["pair_points_skipped"] == 0 and dE <= 1e-10
    if eps <= 1e-9:
        assert dE <= 1e-6


def test_link_mixed_basis_screened():
    """config 2 (1/7 of the points) with basis screening and the mixed build: the reported
    bound, plus the FP32 share, covers the change against the FP64 build on the same tiles."""
    s = synth.make_system(2)
    s = s.subset_points(np.arange(0, s.npts, 7))
    K0, st0 = snk.sn_k_build(s, eps_basis=1e-9)
    for prec in (snk.SNK_FP64, snk.SNK_MIXED):
        K1, st1 = snk.sn_k_build(s, eps_basis=1e-9, screen=snk.SNK_SCREEN_LINK, eps_skip_energy=1e-8,
                                 precision=prec, eps_lowprec_energy=5e-7)
        dE = abs(st1["ex"] - st0["ex"])
        say("config2/7 link 1e-8 precision %d: skipped %.4f, FP32 %d units, |dE| %.2e, bound %.2e" %
            (prec, skipped_fraction(st1), st1["pair_points_lowprec"], dE, st1["skipped_bound"]))
        assert np.array_equal(K1, K1.T)
        assert dE <= st1["skipped_bound"] + (5e-7 if prec == snk.SNK_MIXED else 1e-10)


@pytest.mark.parametrize("cfg,eps", [(1, 1e-9), (1, 1e-6), (2, 1e-9)])
def test_link_kept_set_matches_oracle(cfg, eps):
    """The batches Q_j (the library's partition of the grid, checked to be one) are the input
    of Eq. sp_set; for each batch of the first group the oracle selects the pairs from its own
    collocation, |D| and A-tilde, and the screen must keep exactly those.  Decisions whose
    estimate lies within 1e-9 (relative) of the threshold may go either way."""
    g = np.load(os.path.join(GOLDEN, "oracle_config%d.npz" % cfg))
    s = synth.make_system(cfg, with_density=False).with_density(g["P"])
    ctx = snk.Context(s, screen=snk.SNK_SCREEN_LINK, eps_skip_energy=eps)
    order = ctx.point_order()
    real = order[order >= 0]
    assert np.array_equal(np.sort(real), np.arange(s.npts))      # every point in exactly one batch
    kept = ctx.debug_kept(s.P)
    nb0 = int(kept[:, 0].max()) + 1 if len(kept) else 0
    tiles = ctx.tiles()
    nb0 = max(nb0, max(b1 for gr, b0, b1, _ in tiles if gr == 0))
    got = {}
    for b, A, B in kept:
        got.setdefault(int(b), set()).add((max(int(A), int(B)), min(int(A), int(B))))
    at = LR.a_tilde(s)
    n_cmp = n_tie = 0
    for b in range(nb0):
        pts = order[b * 256:(b + 1) * 256]
        pts = pts[pts >= 0]
        ref, margin = LR.kept_pairs(s, pts, eps, at=at)
        tie = np.abs(margin - 1.0) <= 1e-9
        mine = np.zeros_like(ref)
        for A, B in got.get(b, ()):
            mine[A, B] = True
        low = np.tril(np.ones_like(ref, dtype=bool))
        diff = (mine != ref) & low & ~tie
        assert not diff.any(), (b, np.argwhere(diff)[:5], np.argwhere(mine & ~ref)[:5])
        n_cmp += int(low.sum())
        n_tie += int((tie & low).sum())
    say("config %d link eps %.0e: %d batches, %d pair decisions compared (%d ties), %d kept" %
        (cfg, eps, nb0, n_cmp, n_tie, len(kept)))
    assert len(kept) > 0
