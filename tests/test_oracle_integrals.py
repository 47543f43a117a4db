"""Pins of the oracle's basis, collocation and 3c-CP integrals (Eqs. collocation, 3c_grid).

The 3c-CP integral A_ab(C) = int phi_a phi_b / |r - C| is pinned by two facts
that together determine it uniquely: Poisson's equation in C,
    nabla_C^2 A_ab(C) = -4 pi phi_a(C) phi_b(C),
and its decay at infinity, R * A_ab(C) -> S_ab as |C| = R grows (a function
that is harmonic everywhere and vanishes at infinity is zero).  A brute-force
spherical quadrature of the defining integral on soft functions, positive
semi-definiteness, symmetry, translation invariance and rotation covariance of
p components add independent checks.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import synth


def soft_system(grid=None):
    """Three atoms, s/p/d shells with moderate exponents (smooth integrands)."""
    xyz = [[0.0, 0.0, 0.0], [1.3, 0.4, -0.2], [-0.5, 1.1, 0.7]]
    shells = [
        [(0, [2.1, 0.6], [0.5, 0.6]), (1, [1.4, 0.45], [0.7, 0.4]), (2, [0.9], [1.0])],
        [(0, [1.7, 0.5], [0.4, 0.7]), (1, [0.8], [1.0])],
        [(0, [1.1], [1.0]), (2, [1.3, 0.5], [0.5, 0.5])],
    ]
    return synth.make_custom([8, 1, 1], xyz, shells, grid=grid, n_occ=3)


def test_overlap_unit_diagonal_and_generator_agreement():
    s = synth.make_system(1)
    S = O.overlap(s)
    assert np.allclose(np.diag(S), 1.0, atol=2e-15, rtol=0)
    # the generator computes S by Obara-Saika, the oracle by McMurchie-Davidson
    assert np.max(np.abs(S - synth.overlap_matrix(s))) < 5e-15
    sd = soft_system()
    assert np.allclose(np.diag(O.overlap(sd)), 1.0, atol=2e-15, rtol=0)
    assert np.max(np.abs(O.overlap(sd) - synth.overlap_matrix(sd))) < 5e-15


def test_grid_integrates_overlap_and_density():
    # sum_i w_i Phi_mu,i Phi_nu,i -> S_mu,nu  and  sum_i w_i rho(r_i) -> tr(PS) = 2 N_occ
    s = synth.make_system(1, grid=(99, 590))
    Phi = O.collocate(s)
    S = O.overlap(s)
    Sg = (Phi * s.grid_w) @ Phi.T
    assert np.max(np.abs(Sg - S)) < 2e-5
    rho = np.einsum("mi,mn,ni->i", Phi, s.P, Phi)
    assert abs(np.dot(s.grid_w, rho) - 2 * s.n_occ) < 2e-4
    assert abs(np.trace(s.P @ S) - 2 * s.n_occ) < 1e-12


def test_lebedev_and_partition_of_unity():
    u, w = synth.lebedev(302)
    assert abs(w.sum() - 4 * math.pi) < 1e-13
    atoms = synth.make_system(1, with_density=False).atom_xyz
    rng = np.random.default_rng(5)
    pts = rng.normal(scale=3.0, size=(500, 3))
    tot = np.zeros(len(pts))
    for a in range(len(atoms)):
        wa = synth.becke_partition(pts, a, atoms, np.arange(len(atoms)))
        assert np.all(wa >= 0) and np.all(wa <= 1)
        tot += wa
    assert np.max(np.abs(tot - 1.0)) < 1e-13


def test_collocation_component_order():
    # p components transform like x, y, z; d like xx, xy, xz, yy, yz, zz
    s = synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(1, [1.0], [1.0]), (2, [1.0], [1.0])]], grid=None, n_occ=1)
    r = np.array([[0.3, 0.0, 0.0], [0.0, 0.3, 0.0], [0.0, 0.0, 0.3], [0.2, 0.3, 0.5]])
    Phi = O.collocate(s, r)
    p = Phi[:3]
    assert p[0, 0] > 0 and abs(p[1, 0]) == 0 and abs(p[2, 0]) == 0
    assert p[1, 1] > 0 and abs(p[0, 1]) == 0 and abs(p[2, 1]) == 0
    assert p[2, 2] > 0 and abs(p[0, 2]) == 0 and abs(p[1, 2]) == 0
    d = Phi[3:, 3]
    x, y, z = r[3]
    mono = np.array([x * x, x * y, x * z, y * y, y * z, z * z])
    ratio = d / mono
    # unit-normalised components: cross terms carry sqrt(3) relative to squares
    assert np.allclose(ratio / ratio[0], [1, math.sqrt(3), math.sqrt(3), 1, math.sqrt(3), 1], rtol=1e-13)


def _fd_laplacian(f, C, h):
    """Fourth-order central differences."""
    acc = 0.0
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        acc = acc + (-f(C + 2 * e) + 16 * f(C + e) - 30 * f(C) + 16 * f(C - e) - f(C - 2 * e)) / (12 * h * h)
    return acc


@pytest.mark.parametrize("C", [[0.2, -0.3, 0.1], [0.9, 0.5, 0.3], [-1.0, 0.2, 1.4], [2.5, -1.5, 0.5]])
def test_a3c_poisson_equation(C):
    s = soft_system()
    C = np.array(C)
    lap = _fd_laplacian(lambda c: O.a3c(s, c), C, 2e-2)
    phi = O.collocate(s, C[None, :])[:, 0]
    rhs = -4 * math.pi * np.outer(phi, phi)
    scale = np.max(np.abs(rhs))
    assert np.max(np.abs(lap - rhs)) < 2e-5 * scale


def test_a3c_far_field_limit():
    s = soft_system()
    S = O.overlap(s)
    u = np.array([0.36, -0.48, 0.8])
    errs = []
    for R in (1e3, 1e4):
        A = O.a3c(s, R * u)
        errs.append(np.max(np.abs(R * A - S)))
    # R A - S = O(1/R): the dipole term
    assert errs[1] < 0.2 * errs[0] and errs[1] < 1e-3


def _brute_a3c(s, C, nrad=160, nang=974):
    # int phi_a phi_b / |r - C| = int_0^inf r dr int dOmega phi_a phi_b (C + r u), radial map r = t/(1-t)
    t, wt = np.polynomial.legendre.leggauss(nrad)
    t = 0.5 * (t + 1.0)
    wt = 0.5 * wt
    r = 3.0 * t / (1.0 - t)
    dr = 3.0 / (1.0 - t) ** 2
    u, wa = synth.lebedev(nang)
    pts = C + (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    wq = ((wt * dr * r)[:, None] * wa[None, :]).reshape(-1)
    Phi = O.collocate(s, pts)
    return (Phi * wq) @ Phi.T


@pytest.mark.parametrize("C", [[0.1, 0.2, 0.3], [1.0, -0.6, 0.4]])
def test_a3c_brute_force_quadrature(C):
    s = soft_system()
    C = np.array(C)
    A = O.a3c(s, C)
    B = _brute_a3c(s, C)
    assert np.max(np.abs(A - B)) < 1e-6 * np.max(np.abs(A))


def test_a3c_symmetric_psd_translation_rotation():
    s = synth.make_system(1, with_density=False)
    C = np.array([0.7, -0.2, 1.1])
    A = O.a3c(s, C)
    assert np.max(np.abs(A - A.T)) < 1e-15 * np.max(np.abs(A))
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > -1e-12 * ev.max()
    # translation invariance
    t = np.array([3.0, -7.0, 2.5])
    st = synth.System(**{**s.__dict__, "shell_center": s.shell_center + t})
    At = O.a3c(st, C + t)
    assert np.max(np.abs(At - A)) < 1e-13 * np.max(np.abs(A))
    # rotation covariance of (p, s) blocks
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    sr = synth.System(**{**s.__dict__, "shell_center": s.shell_center @ Q.T})
    Ar = O.a3c(sr, Q @ C)
    offs = s.shell_offsets()
    for sp in np.nonzero(s.shell_l == 1)[0][:3]:
        for ss in np.nonzero(s.shell_l == 0)[0][:4]:
            blk = A[offs[sp]:offs[sp] + 3, offs[ss]]
            blkr = Ar[offs[sp]:offs[sp] + 3, offs[ss]]
            assert np.allclose(blkr, Q @ blk, rtol=0, atol=1e-13 * max(1.0, np.abs(blk).max()))


def test_a3c_single_s_primitive_closed_form():
    # a lone normalised s primitive: A(C) = erf(sqrt(2 zeta) d) / d at distance d from its centre
    z = 1.7
    s = synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(0, [z], [1.0])]], grid=None, n_occ=1)
    for d in [0.05, 0.4, 1.3, 4.0]:
        A = O.a3c(s, np.array([0.0, d, 0.0]))[0, 0]
        assert abs(A - math.erf(math.sqrt(2 * z) * d) / d) < 2e-15 * A


def test_eri_closed_forms_and_symmetry():
    z = 1.3
    s = synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(0, [z], [1.0])]], grid=None, n_occ=1)
    # (ss|ss) for one normalised s primitive = 2 sqrt(zeta/pi)
    assert abs(O.eri_shells(s, 0, 0, 0, 0)[0, 0, 0, 0] - 2 * math.sqrt(z / math.pi)) < 1e-15
    sd = soft_system()
    e = O.eri_shells(sd, 1, 4, 2, 3)
    assert np.allclose(e, O.eri_shells(sd, 4, 1, 2, 3).transpose(1, 0, 2, 3), atol=1e-15)
    assert np.allclose(e, O.eri_shells(sd, 2, 3, 1, 4).transpose(2, 3, 0, 1), atol=1e-15)
    assert np.allclose(e, O.eri_shells(sd, 1, 4, 3, 2).transpose(0, 1, 3, 2), atol=1e-15)
    # Schwarz: |(ab|cd)| <= sqrt((ab|ab)(cd|cd))
    ab = O.eri_shells(sd, 1, 4, 1, 4)
    cd = O.eri_shells(sd, 2, 3, 2, 3)
    dab = np.einsum("ijij->ij", ab)
    dcd = np.einsum("ijij->ij", cd)
    assert np.all(np.abs(e) <= np.sqrt(dab[:, :, None, None] * dcd[None, None, :, :]) * (1 + 1e-12))


def test_eri_against_collocated_potential():
    # (mu lam | nu kap) = int phi_nu phi_kap A_mu,lam (Eq. sn_eri): the grid quadrature
    # with the oracle's A and collocation converges to the analytic four-centre integral
    s = soft_system(grid=(80, 590))
    Phi = O.collocate(s)
    offs = s.shell_offsets()
    for (sa, sb) in [(0, 3), (1, 6), (2, 2)]:
        mu, lam = offs[sa], offs[sb]
        Aw = np.array([O.a3c(s, s.grid_xyz[i])[mu, lam] for i in range(s.npts)]) * s.grid_w
        approx = np.einsum("i,ni,ki->nk", Aw, Phi, Phi)
        exact = np.zeros_like(approx)
        for c in range(s.nshell):
            for d in range(s.nshell):
                exact[offs[c]:offs[c + 1], offs[d]:offs[d + 1]] = O.eri_shells(s, sa, sb, c, d)[0, 0]
        assert np.max(np.abs(approx - exact)) < 2e-5 * np.max(np.abs(exact))
