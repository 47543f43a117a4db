"""Pins of the oracle's sn-LinK selection (Sec. II.E, Eqs. sp_set and exx_fmat_approx) against
what the definitions fix independently of the oracle's own formulas: the triangle inequality
that makes F~ bound the weighted F = D Phi, its equality case, the closed form of A~ for a
one-primitive s-s pair (checked against the oracle's three-centre integral routine), the bound
A~ puts on every s-s integral, and the limits of the threshold."""
import math

import numpy as np
import pytest

from oracle import link_ref as LR
from oracle import oracle as O
from paper_2303_14280_amd import synth


def small_system():
    s = synth.make_system(1)
    rng = np.random.default_rng(5)
    return s, [np.sort(rng.choice(s.npts, size=48, replace=False)) for _ in range(4)]


def s_only_system(grid=(8, 26)):
    xyz = [[0.0, 0.0, 0.0], [0.9, 0.3, -0.2], [2.5, -1.0, 0.8]]
    shells = [[(0, [3.0, 0.7], [0.6, 0.5]), (0, [1.2], [1.0])],
              [(0, [2.2, 0.4], [0.3, 0.8])],
              [(0, [0.9], [1.0])]]
    return synth.make_custom([8, 1, 1], xyz, shells, grid=grid, n_occ=2)


def test_ftilde_bounds_weighted_F():
    """|F_mu,i| = |sum_nu D_mu,nu Phi_nu,i| <= sum_nu |D_mu,nu| |Phi_nu,i|, so F~_mu bounds
    sqrt(w_i) |F_mu,i| at every point of the batch, and F~ of a shell bounds each function."""
    s, batches = small_system()
    off = LR.shell_offsets(s)
    for pts in batches:
        Ft, Fs, phit = LR.batch_estimates(s, pts)
        F = s.P @ O.collocate(s, s.grid_xyz[pts])
        wF = np.max(np.abs(F) * np.sqrt(s.grid_w[pts])[None, :], axis=1)
        assert np.all(Ft >= wF * (1 - 1e-13))
        assert np.any(Ft > 1.5 * wF)      # signs in D and Phi make the bound loose somewhere
        for k in range(len(off) - 1):
            assert Fs[k] == np.max(Ft[off[k]:off[k + 1]])
        phi = O.collocate(s, s.grid_xyz[pts])
        assert phit >= np.max(np.abs(phi.sum(axis=0)) * np.sqrt(s.grid_w[pts])) * (1 - 1e-13)


def test_ftilde_equality_for_nonnegative_density_and_functions():
    """s Gaussians with positive coefficients are positive everywhere; with D >= 0 elementwise
    and a one-point batch every absolute value in Eq. exx_fmat_approx is inert, so
    F~ = sqrt(w) D Phi and phi~ = sqrt(w) sum_mu Phi_mu exactly."""
    s = s_only_system()
    P = np.abs(s.P) + 0.1
    for i in (0, 17, s.npts // 2, s.npts - 1):
        Ft, _, phit = LR.batch_estimates(s, [i], P=P)
        phi = O.collocate(s, s.grid_xyz[[i]])[:, 0]
        assert np.all(phi > 0)
        sw = math.sqrt(s.grid_w[i])
        np.testing.assert_allclose(Ft, sw * (P @ phi), rtol=1e-14, atol=0)
        assert abs(phit - sw * phi.sum()) <= 1e-14 * phit


def test_atilde_closed_form_one_primitive_ss():
    """For one-primitive s shells closer than 1 bohr, A~ = (2 pi / zeta_p) exp(-zeta_a zeta_b
    |AB|^2 / zeta_p) |c_a c_b|, which is A_ab at the Gaussian product centre (F_0(0) = 1):
    compared with the oracle's three-centre integral there."""
    xyz = [[0.0, 0.0, 0.0], [0.5, 0.4, -0.3]]
    shells = [[(0, [1.3], [1.0])], [(0, [0.45], [1.0])]]
    s = synth.make_custom([1, 1], xyz, shells, grid=None, n_occ=1)
    at = LR.a_tilde(s)
    za, zb = s.exps[0], s.exps[1]
    RA, RB = np.asarray(xyz[0]), np.asarray(xyz[1])
    Pc = (za * RA + zb * RB) / (za + zb)
    A = O.a3c(s, Pc)
    assert abs(at[1, 0] - abs(A[1, 0])) <= 1e-13 * at[1, 0]
    A0 = O.a3c(s, RA)      # a same-centre pair peaks at its centre
    assert abs(at[0, 0] - A0[0, 0]) <= 1e-13 * at[0, 0]


def test_atilde_bounds_every_ss_integral():
    """F_0 <= 1, so |A_ab(r)| <= sum over primitive pairs of |prefactor| <= A~_AB for s shells."""
    s = s_only_system()
    at = LR.a_tilde(s)
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.normal(scale=2.0, size=(40, 3)), np.asarray(s.shell_center)])
    worst = 0.0
    for C in pts:
        A = O.a3c(s, C)      # one function per s shell: A is nshell x nshell here
        assert np.all(np.abs(A) <= at * (1 + 1e-13))
        worst = max(worst, float(np.max(np.abs(A) / at)))
    assert worst > 0.5       # the bound is attained closely at the centres


def test_selection_limits_and_monotonicity():
    s, batches = small_system()
    at = LR.a_tilde(s)
    low = np.tril(np.ones_like(at, dtype=bool))
    for pts in batches[:2]:
        k0, _ = LR.kept_pairs(s, pts, 0.0, at=at)
        assert np.array_equal(k0, (at > 0) & low)
        kinf, _ = LR.kept_pairs(s, pts, 1e300, at=at)
        assert not kinf.any()
        prev = k0
        for eps in (1e-12, 1e-9, 1e-6, 1e-3):
            k, m = LR.kept_pairs(s, pts, eps, at=at)
            assert np.all(prev | ~k)                     # a larger threshold keeps a subset
            assert np.array_equal(k, (m >= 1.0) & (at > 0) & low)
            prev = k
        assert prev.sum() < k0.sum()


@pytest.mark.parametrize("bad", ["no_abs", "max_over_shell_min"])
def test_pins_catch_planted_mistakes(bad, monkeypatch):
    """The pins above fail for plausible mistakes planted in the oracle (on the CPU)."""
    s = s_only_system()
    P = s.P.copy()
    P[0, 1] = P[1, 0] = -abs(P[0, 1]) - 0.2       # a negative coupling
    orig = LR.batch_estimates

    def planted(sy, pts, P=None, funcs=None):
        Ft, Fs, phit = orig(sy, pts, P, funcs)
        Pm = np.asarray(sy.P if P is None else P)
        if bad == "no_abs":
            sw = np.sqrt(sy.grid_w[pts])
            phi = O.collocate(sy, sy.grid_xyz[pts])
            Ft = Pm @ np.max(np.abs(phi) * sw[None, :], axis=1)
        else:
            off = LR.shell_offsets(sy)
            Fs = np.array([np.min(Ft[off[k]:off[k + 1]]) for k in range(len(off) - 1)])
        return Ft, Fs, phit

    monkeypatch.setattr(LR, "batch_estimates", planted)
    s2 = s.with_density(P)
    failed = False
    try:
        if bad == "no_abs":
            Ft, _, _ = LR.batch_estimates(s2, [3])
            F = s2.P @ O.collocate(s2, s2.grid_xyz[[3]])[:, 0]
            assert np.all(Ft >= math.sqrt(s2.grid_w[3]) * np.abs(F) * (1 - 1e-13))
            # the equality case with a nonnegative density must also hold
            Pn = np.abs(s2.P) + 0.1
            Ft, _, _ = LR.batch_estimates(s2, [3], P=Pn)
            phi = O.collocate(s2, s2.grid_xyz[[3]])[:, 0]
            np.testing.assert_allclose(Ft, math.sqrt(s2.grid_w[3]) * (Pn @ phi), rtol=1e-14)
            # and the bound over a batch with the negative coupling
            pts = np.arange(0, s2.npts, 7)
            Ft, _, _ = LR.batch_estimates(s2, pts)
            F = s2.P @ O.collocate(s2, s2.grid_xyz[pts])
            assert np.all(Ft >= np.max(np.abs(F) * np.sqrt(s2.grid_w[pts]), axis=1) * (1 - 1e-13))
        else:
            s3, batches = small_system()
            off = LR.shell_offsets(s3)
            Ft, Fs, _ = LR.batch_estimates(s3, batches[0])
            for k in range(len(off) - 1):
                assert Fs[k] == np.max(Ft[off[k]:off[k + 1]])
    except AssertionError:
        failed = True
    assert failed
