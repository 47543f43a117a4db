"""Pins of the oracle's density-fitted Coulomb matrix (Sec. II.B, Eqs. V_df, P_df, J_df)
against what the definitions fix independently of the oracle's own arithmetic:

  * the three-centre integral with an s auxiliary function equals the grid quadrature of
    phi_mu phi_nu against that function's closed-form potential (erf), a different route from
    the Hermite recursions;
  * the metric's diagonal for an s function is the closed-form self-repulsion of a Gaussian
    charge, and the metric is symmetric positive definite;
  * when the auxiliary basis holds every product phi_mu phi_nu of the orbital basis (one
    primitive per shell: the products are Gaussians at the product centre, s and p orbitals
    need s, p and d auxiliary functions there) the fit is exact: J equals the four-centre J;
  * the Coulomb-metric fit is variational: E_J(DF) = 1/2 v V^-1 v <= E_J(exact), on config 1;
  * J is symmetric and linear in the density; planted mistakes fail these pins.
"""
import math
import types

import numpy as np
import pytest
from scipy.special import erf

from oracle import dfj_ref as D
from oracle import oracle as O
from paper_2303_14280_amd import synth


def soft_system(grid=(40, 110)):
    xyz = [[0.0, 0.0, 0.0], [1.1, 0.4, -0.3]]
    shells = [[(0, [1.4, 0.5], [0.6, 0.5]), (1, [0.9], [1.0])], [(0, [0.8], [1.0])]]
    return synth.make_custom([8, 1], xyz, shells, grid=grid, n_occ=1)


def aux_of(centres, ls, exps, coefs=None):
    m = len(ls)
    return types.SimpleNamespace(shell_center=np.asarray(centres, np.float64).reshape(-1, 3),
                                 shell_l=np.asarray(ls, np.int32), shell_nprim=np.ones(m, np.int32),
                                 shell_prim_off=np.arange(m, dtype=np.int32), exps=np.asarray(exps, np.float64),
                                 coefs=np.ones(m) if coefs is None else np.asarray(coefs, np.float64))


def test_three_centre_matches_potential_quadrature():
    """(mu nu | K) = int phi_mu phi_nu(r) V_K(r) dr with V_K(r) = c (pi/z)^{3/2} erf(sqrt(z) R) / R
    for chi_K = c exp(-z |r - C|^2), R = |r - C|: the oracle's grid quadrature of it."""
    s = soft_system()
    C = np.array([0.3, -0.2, 0.5])
    z, c = 0.7, 1.3
    aux = aux_of([C], [0], [z], [c])
    T, _ = D.tensors(s, aux)
    R = np.linalg.norm(s.grid_xyz - C, axis=1)
    pot = c * (math.pi / z) ** 1.5 * erf(math.sqrt(z) * R) / R
    phi = O.collocate(s)
    ref = (phi * (s.grid_w * pot)[None, :]) @ phi.T
    # the grid integrates these smooth integrands to a few parts in 1e5
    assert np.max(np.abs(T[:, :, 0] - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_metric_closed_form_and_definite():
    """(K|K) of c exp(-z r^2) is the self-repulsion q^2 sqrt(2 z / pi) of a Gaussian charge
    q = c (pi/z)^{3/2}; the metric of a real auxiliary basis is symmetric positive definite."""
    z, c = 0.9, 0.7
    aux = aux_of([[0.0, 0.0, 0.0]], [0], [z], [c])
    s = soft_system(grid=None)
    _, V = D.tensors(s, aux)
    q = c * (math.pi / z) ** 1.5
    assert abs(V[0, 0] - q * q * math.sqrt(2 * z / math.pi)) <= 1e-13 * V[0, 0]
    s1 = synth.make_system(1, with_density=False)
    _, V1 = D.tensors(s1, synth.make_aux_basis(s1))
    assert np.max(np.abs(V1 - V1.T)) <= 1e-13 * np.max(np.abs(V1))
    assert np.linalg.eigvalsh(V1)[0] > 0.0


def product_aux(s, lmax):
    """Auxiliary shells l = 0..lmax at every product centre of the one-primitive orbital shells."""
    cen, ls, ex = [], [], []
    for a in range(s.nshell):
        for b in range(a + 1):
            za, zb = s.exps[s.shell_prim_off[a]], s.exps[s.shell_prim_off[b]]
            P = (za * s.shell_center[a] + zb * s.shell_center[b]) / (za + zb)
            for l in range(lmax + 1):
                cen.append(P)
                ls.append(l)
                ex.append(za + zb)
    return aux_of(cen, ls, ex)


@pytest.mark.parametrize("with_p", [False, True])
def test_fit_exact_for_product_gaussians(with_p):
    xyz = [[0.0, 0.0, 0.0], [1.2, 0.3, -0.4], [0.2, 1.5, 0.6]]
    shells = [[(0, [1.1], [1.0]), (0, [0.35], [1.0])], [(0, [0.8], [1.0])], [(0, [0.5], [1.0])]]
    if with_p:
        shells = [[(0, [1.1], [1.0]), (1, [0.6], [1.0])], [(0, [0.8], [1.0])], [(1, [0.5], [1.0])]]
    s = synth.make_custom([8, 1, 1], xyz, shells, grid=None, n_occ=2)
    aux = product_aux(s, 2 if with_p else 0)
    J, v, d, E = D.dfj(s, aux)
    Jx = O.eri_j(s)
    Ex = 0.5 * float(np.sum(s.P * Jx))
    assert abs(E - Ex) <= 1e-9 * Ex
    assert np.max(np.abs(J - Jx)) <= 1e-8 * np.max(np.abs(Jx))


def test_fit_is_variational_config1():
    s = synth.make_system(1)
    aux = synth.make_aux_basis(s)
    T, V = D.tensors(s, aux)
    J, v, d, E = D.dfj(s, aux, T=T, V=V)
    Jx = O.eri_j(s)
    Ex = 0.5 * float(np.sum(s.P * Jx))
    assert 0.0 < E <= Ex
    assert (Ex - E) <= 0.01 * Ex               # the auxiliary set spans the density well
    assert np.max(np.abs(J - J.T)) <= 1e-12 * np.max(np.abs(J))
    # linear in the density
    P2 = synth.random_symmetric(s.nbf, 1)
    J2, *_ = D.dfj(s, aux, P=P2, T=T, V=V)
    J3, *_ = D.dfj(s, aux, P=s.P + 0.5 * P2, T=T, V=V)
    assert np.max(np.abs(J3 - (J + 0.5 * J2))) <= 1e-10 * np.max(np.abs(J))
    # a smaller auxiliary set fits worse
    keep = np.asarray(aux.shell_l) == 0
    small = aux_of(np.asarray(aux.shell_center)[keep], np.asarray(aux.shell_l)[keep], np.asarray(aux.exps)[keep],
                   np.asarray(aux.coefs)[keep])
    _, _, _, Es = D.dfj(s, small)
    assert Es < E


@pytest.mark.parametrize("bad", ["no_solve", "mismatched_aux_index"])
def test_pins_catch_planted_mistakes(bad, monkeypatch):
    """Plausible mistakes planted in the oracle (on the CPU) fail the exactness pin."""
    def planted(s, aux, P=None, T=None, V=None):
        P = np.asarray(s.P if P is None else P, np.float64)
        if T is None or V is None:
            T, V = D.tensors(s, aux)
        v = np.einsum("mnk,mn->k", T, P)
        d = v / np.diag(V) if bad == "no_solve" else np.linalg.solve(V, v)
        J = T @ (d if bad == "no_solve" else d[::-1])
        return J, v, d, 0.5 * float(np.sum(P * J))

    monkeypatch.setattr(D, "dfj", planted)
    with pytest.raises(AssertionError):
        test_fit_exact_for_product_gaussians(False)
