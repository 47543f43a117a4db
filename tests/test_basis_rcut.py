"""Basis screening radius (Eq. basis_screen) of the library's host code, checked on the CPU
against direct evaluation of the basis functions by the oracle: beyond r_cut every Cartesian
component is below eps_basis (along the axes, the face and the body diagonals and random
directions, where the angular factors of p and d components peak), and for a single
positive s primitive the radius is exact (the function reaches eps just inside it)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import snk, synth


def one_shell(l, exps, raw):
    return synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(l, exps, raw)]], grid=None, n_occ=1)


def directions(rng, n=64):
    d = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [0, 1, 1], [1, 1, 1], [-1, 1, -1]]
    d = np.array(d, float)
    d = np.vstack([d, rng.normal(size=(n, 3))])
    return d / np.linalg.norm(d, axis=1, keepdims=True)


SHELLS = [(0, [5000.0, 120.0, 3.0], [0.3, 0.5, 0.4]),
          (0, [0.1], [1.0]),
          (1, [40.0, 2.0, 0.15], [0.2, 0.7, 0.5]),
          (1, [0.8], [1.0]),
          (2, [12.0, 0.9, 0.12], [0.4, 0.4, 0.6]),
          (2, [1.1], [1.0])]


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9, 1e-12])
@pytest.mark.parametrize("shell", range(len(SHELLS)))
def test_functions_below_eps_beyond_rcut(shell, eps):
    l, e, c = SHELLS[shell]
    s = one_shell(l, e, c)
    r = snk.shell_rcut(l, s.exps, s.coefs, eps)
    rng = np.random.default_rng([shell, int(-np.log10(eps))])
    if r < 0:
        # never significant: check a dense radial sweep
        radii = np.linspace(0.0, 20.0, 401)
    else:
        radii = r * np.array([1.0 + 1e-9, 1.001, 1.01, 1.1, 1.3, 1.7, 2.5, 4.0])
    d = directions(rng)
    pts = (radii[:, None, None] * d[None, :, :]).reshape(-1, 3)
    phi = O.collocate(s, pts)
    assert np.max(np.abs(phi)) < eps, (r, np.max(np.abs(phi)))


@pytest.mark.parametrize("eps", [1e-2, 1e-5, 1e-9, 1e-13])
@pytest.mark.parametrize("zeta", [0.1, 2.0, 300.0])
def test_single_s_primitive_radius_is_exact(zeta, eps):
    s = one_shell(0, [zeta], [1.0])
    r = snk.shell_rcut(0, s.exps, s.coefs, eps)
    c = s.coefs[0]
    if c < eps:
        assert r < 0
        return
    # exp(-zeta r^2) c = eps has the closed-form root
    r_exact = np.sqrt(np.log(c / eps) / zeta)
    assert abs(r - r_exact) <= 1e-9 * r_exact
    inside = O.collocate(s, np.array([[0.0, 0.0, r * (1 - 1e-6)]]))
    assert abs(inside[0, 0]) >= eps


def test_never_significant_and_errors():
    s = one_shell(2, [0.5], [1.0])
    assert snk.shell_rcut(2, s.exps, s.coefs, 1e6) == -1.0
    with pytest.raises(snk.SnkError):
        snk.shell_rcut(3, [1.0], [1.0], 1e-9)
    with pytest.raises(snk.SnkError):
        snk.shell_rcut(0, [1.0], [1.0], 0.0)
    with pytest.raises(snk.SnkError):
        snk.shell_rcut(1, [-1.0], [1.0], 1e-9)
