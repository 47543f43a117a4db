"""Pins of the exchange-correlation oracle (Sec. II.C, Eqs. vxc_num, zmat, exc_grid, den_grid).

Each check ties the oracle to something other than its own formulas:
  * basis values equal the C oracle's collocation; gradients equal central differences of it;
  * Dirac-Slater exchange of a single s Gaussian against its closed-form integral, and the
    electron count against tr(P S);
  * Perdew-Wang correlation against its published high-density (A ln rs - c1, c1 = 0.046644)
    and low-density (-d0 / rs, d0 = alpha1 / beta4 = 0.4335) limits;
  * PBE against its defining limits: no gradient reduces it to the local form; the exchange
    enhancement tends to 1 + kappa and grows as 1 + mu s^2; the correlation correction grows as
    beta t^2 and cancels the local correlation for large t;
  * complex-step derivatives against central differences;
  * V^xc against finite differences of E_xc with respect to the density matrix (the definition
    V_mu,nu = dE_xc / dD_mu,nu), which fixes the factors of Eq. zmat;
  * Euler's theorem for Slater exchange (degree 4/3 in D): tr(P V) = 4/3 E_x.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import xc_oracle as X
from paper_2303_14280_amd import synth


def small_system(grid=(30, 110)):
    shells = [[(0, [30.0, 4.0, 0.5], [0.3, 0.5, 0.4]), (1, [3.0, 0.4], [0.6, 0.5]), (2, [0.9], [1.0])],
              [(0, [5.0, 0.6], [0.5, 0.5]), (1, [0.7], [1.0])]]
    return synth.make_custom([8, 1], [[0.0, 0.0, 0.0], [0.3, -0.4, 1.7]], shells, grid=grid, n_occ=3)


def test_collocation_values_and_gradients():
    s = small_system(grid=None)
    rng = np.random.default_rng(5)
    pts = rng.normal(scale=1.2, size=(40, 3))
    phi, dphi = X.collocate_grad(s, pts)
    ref = O.collocate(s, pts)
    assert np.max(np.abs(phi - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref)))
    h = 1e-5
    for q in range(3):
        e = np.zeros(3)
        e[q] = h
        fd = (O.collocate(s, pts + e) - O.collocate(s, pts - e)) / (2 * h)
        assert np.max(np.abs(dphi[q] - fd)) <= 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_slater_exchange_of_a_gaussian():
    zeta = 1.3
    s = synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(0, [zeta], [1.0])]], grid=(120, 26), n_occ=1)
    P = np.array([[2.0]])
    V, ex, nel = X.vxc(s, X.SLATER, P=P)
    # rho = 2 N^2 exp(-2 zeta r^2), N^2 = (2 zeta / pi)^{3/2}
    n2 = (2 * zeta / np.pi) ** 1.5
    exact = -0.75 * (3 / np.pi) ** (1 / 3) * (2 * n2) ** (4 / 3) * (np.pi / (8 * zeta / 3)) ** 1.5
    assert abs(ex - exact) <= 1e-9 * abs(exact)
    assert abs(nel - 2.0) <= 1e-9
    # V_11 = dE/dP_11: eps is homogeneous of degree 4/3 in P, so V_11 P_11 = 4/3 E
    assert abs(V[0, 0] * 2.0 - 4.0 / 3.0 * exact) <= 1e-9 * abs(exact)


def test_electron_count_matches_trace():
    s = small_system(grid=(60, 194))
    _, _, nel = X.vxc(s, X.LDA)
    S = O.overlap(s)
    assert abs(nel - float(np.sum(s.P * S))) <= 1e-6 * abs(nel)


def test_pw92_limits():
    for rs in (1e-6, 1e-7, 1e-8):
        assert abs(X.pw92_eps(rs) - (X.PW_A * np.log(rs) - 0.046644)) <= 0.1 * np.sqrt(rs) + 2e-6
    for rs in (1e5, 1e6):
        assert abs(rs * X.pw92_eps(rs) + 0.4335) <= 2e-3 * 0.4335 + 10.0 / np.sqrt(rs)
    rs = np.array([0.5, 1.0, 2.0, 5.0])
    assert np.all(X.pw92_eps(rs) < 0) and np.all(np.diff(X.pw92_eps(rs)) > 0)


def test_pbe_limits():
    rho = np.array([1e-3, 0.1, 1.0, 30.0])
    assert np.allclose(X.pbe_x(rho, 0.0 * rho), X.slater_x(rho), rtol=1e-15, atol=0)
    assert np.allclose(X.pbe_c(rho, 0.0 * rho), rho * X.pw92_eps(X.wigner_rs(rho)), rtol=1e-15, atol=0)
    assert abs(X.pbe_fx(1e12) - 1.804) <= 1e-9
    s2 = 1e-7
    assert abs((X.pbe_fx(s2) - 1.0) / s2 - 0.2195149727645171) <= 1e-6
    for rs in (0.5, 2.0, 6.0):
        t2 = 1e-8
        assert abs(X.pbe_h(rs, t2) / t2 - 0.06672455060314922) <= 1e-6
        ec = X.pw92_eps(rs)
        assert abs(X.pbe_h(rs, 1e10) + ec) <= 1e-6 * abs(ec)


@pytest.mark.parametrize("functional", [X.SLATER, X.LDA, X.PBE])
def test_complex_step_matches_central_differences(functional):
    rng = np.random.default_rng(functional)
    rho = 10.0 ** rng.uniform(-6, 1, size=50)
    gamma = rho ** (8 / 3) * 10.0 ** rng.uniform(-3, 1.5, size=50)
    e, er, eg = X.eps_and_derivs(functional, rho, gamma)
    f = X.FUNCTIONALS[functional]
    h = 1e-6 * rho
    fd_r = (f(rho + h, gamma) - f(rho - h, gamma)) / (2 * h)
    assert np.allclose(er, fd_r, rtol=1e-6, atol=0)
    if functional == X.PBE:
        # exchange and correlation gradient terms nearly cancel at some points: difference
        # each part and bound the error by the size of the parts
        hg = 1e-4 * gamma
        parts = [(g(rho, gamma + hg) - g(rho, gamma - hg)) / (2 * hg) for g in (X.pbe_x, X.pbe_c)]
        assert np.all(np.abs(eg - parts[0] - parts[1]) <= 1e-6 * (np.abs(parts[0]) + np.abs(parts[1])))
    else:
        assert not np.any(eg)
    lo = X.eps_and_derivs(functional, np.array([0.5 * X.RHO_MIN]), np.array([0.0]))
    assert all(float(a[0]) == 0.0 for a in lo)


@pytest.mark.parametrize("functional", [X.SLATER, X.LDA, X.PBE])
def test_vxc_is_the_derivative_of_exc(functional):
    s = small_system(grid=(24, 50))
    V, exc, _ = X.vxc(s, functional)
    assert np.allclose(V, V.T, rtol=0, atol=1e-14 * np.max(np.abs(V)))
    assert abs(exc - X.exc_only(s, functional, s.P)) <= 1e-12 * abs(exc)
    rng = np.random.default_rng(10 + functional)
    n = s.nbf
    pairs = [(int(a), int(b)) for a, b in zip(rng.integers(n, size=8), rng.integers(n, size=8))] + [(0, 0), (3, 3)]
    h = 1e-5
    for a, b in pairs:
        E = np.zeros((n, n))
        E[a, b] += 1.0
        E[b, a] += 1.0 if a != b else 0.0
        d = (X.exc_only(s, functional, s.P + h * E) - X.exc_only(s, functional, s.P - h * E)) / (2 * h)
        want = d / (2.0 if a != b else 1.0)
        assert abs(V[a, b] - want) <= 1e-6 * max(1.0, np.max(np.abs(V))), (a, b, V[a, b], want)


def test_slater_euler_theorem():
    s = small_system(grid=(30, 110))
    V, ex, _ = X.vxc(s, X.SLATER)
    assert abs(float(np.sum(s.P * V)) - 4.0 / 3.0 * ex) <= 1e-10 * abs(ex)
