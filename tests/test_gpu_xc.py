"""The exchange-correlation potential matrix (Sec. II.C) on the GPU, through the C ABI, against
the XC oracle (oracle/xc_oracle.py, pinned in test_oracle_xc.py).

Tolerance: every step is FP64; V^xc sums O(10^5) grid points of O(1) terms, so rounding
order alone moves elements by ~1e-13 of max |V|.  The bar is 1e-11 max |V| element by element
and 1e-10 (relative to max(1, |E_xc|)) for E_xc and N_el.
"""
import os
import sys

import numpy as np
import pytest

from oracle import xc_oracle as X
from paper_2303_14280_amd import snk, synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FUNCTIONALS = [snk.SNK_XC_SLATER, snk.SNK_XC_LDA, snk.SNK_XC_PBE]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare(V, exc, nel, s, functional, tag):
    Vr, er, nr = X.vxc(s, functional)
    scale = float(np.max(np.abs(Vr)))
    dV = float(np.max(np.abs(V - Vr)))
    say("%s functional %d: E_xc %.12f (oracle %.12f), N_el %.10f (oracle %.10f), max|dV| %.2e of %.2e" %
        (tag, functional, exc, er, nel, nr, dV, scale))
    assert np.array_equal(V, V.T)
    assert dV <= 1e-11 * scale
    assert abs(exc - er) <= 1e-10 * max(1.0, abs(er))
    assert abs(nel - nr) <= 1e-10 * max(1.0, abs(nr))


@pytest.mark.parametrize("functional", FUNCTIONALS)
def test_config1_matches_oracle(functional):
    s = synth.make_system(1)
    ctx = snk.Context(s)
    V, exc, nel = ctx.vxc(s.P, functional)
    compare(V, exc, nel, s, functional, "config1")


@pytest.mark.parametrize("functional", [snk.SNK_XC_LDA, snk.SNK_XC_PBE])
def test_config2_subset_matches_oracle(functional):
    """config 2 (290 functions) on every 7th grid point."""
    s = synth.make_system(2)
    s = s.subset_points(np.arange(3, s.npts, 7))
    ctx = snk.Context(s)
    V, exc, nel = ctx.vxc(s.P, functional)
    compare(V, exc, nel, s, functional, "config2/7")


def test_chunks_paths_and_determinism():
    """A small device budget (several chunks of batches) and one chunk, two calls in a row: same V
    to rounding, bitwise equal per call."""
    s = synth.make_system(1)
    # split partial products (256 x nbf^2) plus three FP64 rows per column: ten batches a chunk
    budget = 256 * 38 * 38 * 8 + (3 * 38 * 8 + 16) * 2560
    a = snk.Context(s, max_device_bytes=budget)
    b = snk.Context(s)
    Va, ea, na = a.vxc(s.P, snk.SNK_XC_PBE)
    Va2, ea2, _ = a.vxc(s.P, snk.SNK_XC_PBE)
    Vb, eb, nb = b.vxc(s.P, snk.SNK_XC_PBE)
    say("chunked vs one chunk: |dE| %.2e max|dV| %.2e" %
        (abs(ea - eb), np.max(np.abs(Va - Vb))))
    assert np.array_equal(Va, Va2) and ea == ea2
    assert np.max(np.abs(Va - Vb)) <= 1e-12 * np.max(np.abs(Vb))
    assert abs(ea - eb) <= 1e-12 * abs(eb) and abs(na - nb) <= 1e-12 * abs(nb)


def test_device_pointers_and_sn_k_on_one_context():
    """Device-pointer mode on a torch stream, interleaved with sn-K builds on the same context."""
    import torch
    s = synth.make_system(1)
    stream = torch.cuda.Stream()
    ctx = snk.Context(s, flags=snk.SNK_DEVICE_PTRS, stream=stream.cuda_stream, device=0)
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    V = torch.empty_like(P)
    K = torch.empty_like(P)
    ctx.build_device(P.data_ptr(), K.data_ptr())
    exc, nel = ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_LDA, scalars=True)
    ctx.build_device(P.data_ptr(), K.data_ptr())
    torch.cuda.synchronize()
    Vh, eh, nh = snk.Context(s).vxc(s.P, snk.SNK_XC_LDA)
    K0, _ = snk.Context(s).build(s.P)
    assert np.array_equal(V.cpu().numpy(), Vh) and exc == eh and nel == nh
    assert np.array_equal(K.cpu().numpy(), K0)


def test_empty_and_negligible_density():
    """A grid far from every basis function: every point is below the density threshold, so V,
    E_xc and N_el are exactly zero; arguments are checked."""
    shells = [[(0, [2.0, 0.5], [0.5, 0.5]), (1, [1.0], [1.0])], []]
    s = synth.make_custom([8, 1], [[0.0, 0.0, 0.0], [0.0, 0.0, 80.0]], shells, grid=None, n_occ=1)
    pts = np.array([[0.0, 0.0, 80.0 + 0.1 * k] for k in range(300)])
    s = s.with_grid(pts, np.full(300, 0.01))
    ctx = snk.Context(s)
    V, exc, nel = ctx.vxc(s.P, snk.SNK_XC_PBE)
    assert not np.any(V) and exc == 0.0 and nel == 0.0
    with pytest.raises(snk.SnkError):
        ctx.vxc(s.P, 7)
    bad = s.P.copy()
    bad[0, 0] = np.nan
    with pytest.raises(snk.SnkError):
        ctx.vxc(bad, snk.SNK_XC_LDA)
    asym = s.P.copy()
    asym[0, 1] += 1.0
    with pytest.raises(snk.SnkError):
        snk.Context(s, flags=snk.SNK_VALIDATE).vxc(asym, snk.SNK_XC_LDA)


def test_basis_screened_tight_matches_oracle():
    """eps_basis = 1e-13 (tiles of at most 16 batches, each over its functions B_t; small
    groups so that tiles drop functions): the dropped basis values are below 1e-13, so V^xc and
    E_xc keep the unscreened parity bar against the oracle."""
    s = synth.make_system(1)
    ctx = snk.Context(s, eps_basis=1e-13, max_device_bytes=6 * s.nbf * 256 * 24)
    sizes = [fn.size for _, _, _, fn in ctx.tiles()]
    assert min(sizes) < s.nbf
    for functional in (snk.SNK_XC_LDA, snk.SNK_XC_PBE):
        V, exc, nel = ctx.vxc(s.P, functional)
        V2, _, _ = ctx.vxc(s.P, functional)
        assert np.array_equal(V, V2)
        compare(V, exc, nel, s, functional, "config1 eps_basis 1e-13 (|B_t| mean %.1f of %d)" %
                (np.mean(sizes), s.nbf))


@pytest.mark.parametrize("cfg,stride", [(3, 256), (4, 4096)])
def test_basis_screened_sampled_large(cfg, stride):
    """The 150- and 500-atom clusters at their real basis size, on a seeded subset of their grid
    points, basis-screened at the paper's tolerance (1e-9), against the unscreened oracle on
    the same points: |dE_xc| <= 1e-6 Eh and max|dV| <= 1e-6 max|V|."""
    s = synth.make_system(cfg)
    off = int(np.random.default_rng([cfg, 91]).integers(stride))
    s = s.subset_points(np.arange(off, s.npts, stride))
    ctx = snk.Context(s, eps_basis=1e-9)
    sizes = [fn.size for _, _, _, fn in ctx.tiles()]
    V, exc, nel = ctx.vxc(s.P, snk.SNK_XC_PBE)
    V2, exc2, _ = ctx.vxc(s.P, snk.SNK_XC_PBE)
    assert np.array_equal(V, V2) and exc == exc2   # tile products on several streams, reductions in order
    Vr, er, nr = X.vxc(s, X.PBE, chunk=4000)
    dV = float(np.max(np.abs(V - Vr)))
    say("config %d / %d points, |B_t| mean %.1f of %d: E_xc %.10f (oracle %.10f) |dE| %.2e, N_el %.8f (oracle %.8f), "
        "max|dV| %.2e of %.2e" % (cfg, s.npts, np.mean(sizes), s.nbf, exc, er, abs(exc - er), nel, nr, dV,
                                  np.max(np.abs(Vr))))
    assert np.array_equal(V, V.T)
    assert abs(exc - er) <= 1e-6 and abs(nel - nr) <= 1e-6
    assert dV <= 1e-6 * float(np.max(np.abs(Vr)))


def test_xc_ignores_sn_k_modes_and_leaves_k_unchanged():
    """The XC build on contexts made for the other sn-K modes (mixed precision with the learned
    screen, the paper's pair selection, two overlapped groups) gives the plain context's V^xc,
    and sn-K builds on the same context before and after an XC call agree bitwise."""
    s = synth.make_system(2)
    s = s.subset_points(np.arange(0, s.npts, 5))
    V0, e0, _ = snk.Context(s).vxc(s.P, snk.SNK_XC_PBE)
    kws = [dict(screen=snk.SNK_SCREEN_LINK, eps_skip_energy=1e-9),
           dict(flags=snk.SNK_OVERLAP_GROUPS, max_device_bytes=64 * s.nbf * 256 * 24)]
    if os.path.exists(snk.SCREENER_WEIGHTS):
        kws.append(dict(precision=snk.SNK_MIXED, screen=snk.SNK_SCREEN_LEARNED, screener=snk.load_screener()))
    for kw in kws:
        ctx = snk.Context(s, **kw)
        K1, st1 = ctx.build(s.P)
        V, e, _ = ctx.vxc(s.P, snk.SNK_XC_PBE)
        K2, st2 = ctx.build(s.P)
        say("context %s: max|dV| %.2e, |dE_xc| %.2e, K unchanged %s" %
            (sorted(kw), np.max(np.abs(V - V0)), abs(e - e0), np.array_equal(K1, K2)))
        assert np.max(np.abs(V - V0)) <= 1e-12 * np.max(np.abs(V0)) and abs(e - e0) <= 1e-11 * abs(e0)
        assert np.array_equal(K1, K2) and st1["ex"] == st2["ex"]


@pytest.mark.parametrize("kw", [dict(), dict(screen=snk.SNK_SCREEN_LINK, eps_skip_energy=1e-9),
                                dict(eps_basis=1e-9), dict(max_device_bytes=40 * 290 * 256 * 24)])
def test_combined_build_matches_separate_calls(kw):
    """snk_ctx_build_kxc (Phi and F shared between sn-K and XC where the context allows it) gives
    the K of snk_ctx_build bitwise and the V^xc of snk_vxc_build to rounding order; V^xc
    also against the XC oracle.  The last case splits the grid into several batch groups, whose
    XC contributions accumulate across groups."""
    s = synth.make_system(2)
    s = s.subset_points(np.arange(1, s.npts, 9))
    ctx = snk.Context(s, **kw)
    if "max_device_bytes" in kw:
        assert ctx.ngroups > 1
    K0, st0 = ctx.build(s.P)
    V0, e0, n0 = ctx.vxc(s.P, snk.SNK_XC_PBE)
    K1, V1, e1, n1, st1 = ctx.build_kxc(s.P, snk.SNK_XC_PBE)
    K2, V2, e2, _, _ = ctx.build_kxc(s.P, snk.SNK_XC_PBE)
    say("combined %s: K equal %s, max|dV| %.2e, |dE_xc| %.2e, repeat equal %s" %
        (sorted(kw), np.array_equal(K0, K1), np.max(np.abs(V1 - V0)), abs(e1 - e0),
         np.array_equal(V1, V2) and np.array_equal(K1, K2)))
    assert np.array_equal(K0, K1) and st0["ex"] == st1["ex"]
    assert np.array_equal(V1, V2) and np.array_equal(K1, K2) and e1 == e2
    assert np.max(np.abs(V1 - V0)) <= 1e-13 * np.max(np.abs(V0))
    assert abs(e1 - e0) <= 1e-12 * abs(e0) and abs(n1 - n0) <= 1e-12 * abs(n0)
    if not kw:
        compare(V1, e1, n1, s, snk.SNK_XC_PBE, "config2/9 combined")
        # the other order on a fresh context: combined first, then the XC build alone
        c2 = snk.Context(s, **kw)
        K3, V3, e3, _, _ = c2.build_kxc(s.P, snk.SNK_XC_PBE)
        V4, e4, _ = c2.vxc(s.P, snk.SNK_XC_PBE)
        assert np.array_equal(K3, K1) and np.array_equal(V3, V1) and np.array_equal(V4, V0) and e4 == e0
