"""CPU FP64 oracle of the exchange-correlation potential matrix (Sec. II.C).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.  It shares no
code with the HIP library; systems are passed duck-typed (basis SoA, grid, weights, density).

What it computes, step by step in the paper's notation, for a spin-restricted density:
  * Phi_{mu i} = phi_mu(r_i) (Eq. collocation) and grad Phi_{mu i}, by direct evaluation of the
    contracted Cartesian Gaussians and their analytic first derivatives;
  * F = D Phi (Eq. fmat); rho_i = sum_mu F_{mu i} Phi_{mu i} and
    grad rho_i = 2 sum_mu F_{mu i} grad Phi_{mu i} (Eq. den_grid); gamma_i = |grad rho_i|^2;
  * the energy density eps(rho, gamma) per unit volume of the chosen functional and its
    partial derivatives E^rho, E^gamma (Eq. exc_grid), taken here by complex-step
    differentiation of eps itself (exact to rounding, and independent of any hand-derived
    derivative formula);
  * Z_{mu i} = w_i/2 (E^rho_i Phi_{mu i} + 4 E^gamma_i grad rho_i . grad Phi_{mu i}) (Eq. zmat);
  * V^xc = Phi Z^T + Z Phi^T (Eq. vxc_num), E_xc = sum_i w_i eps_i, N_el = sum_i w_i rho_i.

Points whose density is below RHO_MIN contribute nothing (the usual density threshold of
numerical XC integration; the paper does not state one).

Functionals (closed-shell forms, atomic units), written from their published definitions:
  1 SLATER  Dirac-Slater exchange, eps = -(3/4)(3/pi)^(1/3) rho^(4/3)
  2 LDA     Slater exchange + Perdew-Wang 1992 correlation (zeta = 0)
  3 PBE     Perdew-Burke-Ernzerhof exchange + correlation (phi = 1)
"""
from __future__ import annotations

import numpy as np

RHO_MIN = 1e-12

SLATER, LDA, PBE = 1, 2, 3

# Perdew-Wang 1992, paramagnetic correlation energy per particle
PW_A, PW_A1 = 0.031091, 0.21370
PW_B1, PW_B2, PW_B3, PW_B4 = 7.5957, 3.5876, 1.6382, 0.49294
# Perdew-Burke-Ernzerhof
PBE_KAPPA = 0.804
PBE_BETA = 0.06672455060314922
PBE_MU = PBE_BETA * np.pi ** 2 / 3.0
PBE_GAMMA = (1.0 - np.log(2.0)) / np.pi ** 2


# ---------------------------------------------------------------------------------------------
# basis functions and their gradients
# ---------------------------------------------------------------------------------------------

def _components(l):
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def _dfact(n):
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def collocate_grad(s, xyz=None):
    """Phi [nbf, n] and grad Phi [3, nbf, n] at the points (rows in shell order, Cartesian
    components lexicographic, each unit-normalised)."""
    xyz = np.asarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    n = xyz.shape[0]
    nbf = int(sum((int(l) + 1) * (int(l) + 2) // 2 for l in s.shell_l))
    phi = np.zeros((nbf, n))
    dphi = np.zeros((3, nbf, n))
    row = 0
    for sh in range(len(s.shell_l)):
        l = int(s.shell_l[sh])
        o, k = int(s.shell_prim_off[sh]), int(s.shell_nprim[sh])
        ex = np.asarray(s.exps[o:o + k])
        co = np.asarray(s.coefs[o:o + k])
        d = xyz - np.asarray(s.shell_center[sh])[None, :]
        r2 = np.sum(d * d, axis=1)
        g = np.exp(-np.outer(r2, ex))              # [n, k]
        R = g @ co                                 # sum_k c_k e^{-zeta_k r^2}
        dR = -2.0 * (g @ (co * ex))                # (1/r) dR/dr: d/dx R = x * dR
        for (ax, ay, az) in _components(l):
            nc = np.sqrt(_dfact(2 * l - 1) / (_dfact(2 * ax - 1) * _dfact(2 * ay - 1) * _dfact(2 * az - 1)))
            a = (ax, ay, az)
            mono = d[:, 0] ** ax * d[:, 1] ** ay * d[:, 2] ** az
            phi[row] = nc * mono * R
            for q in range(3):
                if a[q] > 0:
                    e = list(a)
                    e[q] -= 1
                    dmono = a[q] * d[:, 0] ** e[0] * d[:, 1] ** e[1] * d[:, 2] ** e[2]
                else:
                    dmono = np.zeros(n)
                dphi[q, row] = nc * (dmono * R + mono * d[:, q] * dR)
            row += 1
    return phi, dphi


# ---------------------------------------------------------------------------------------------
# functionals: energy per unit volume eps(rho, gamma); complex-safe (no abs, no branches)
# ---------------------------------------------------------------------------------------------

def slater_x(rho, gamma=None):
    return -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * rho ** (4.0 / 3.0)


def pw92_eps(rs):
    """Correlation energy per particle of the uniform gas, zeta = 0 (Perdew-Wang 1992)."""
    q0 = -2.0 * PW_A * (1.0 + PW_A1 * rs)
    q1 = 2.0 * PW_A * (PW_B1 * np.sqrt(rs) + PW_B2 * rs + PW_B3 * rs ** 1.5 + PW_B4 * rs ** 2)
    return q0 * np.log(1.0 + 1.0 / q1)


def wigner_rs(rho):
    return (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)


def lda_xc(rho, gamma=None):
    return slater_x(rho) + rho * pw92_eps(wigner_rs(rho))


def pbe_fx(s2):
    """PBE exchange enhancement factor as a function of s^2."""
    return 1.0 + PBE_KAPPA - PBE_KAPPA / (1.0 + PBE_MU * s2 / PBE_KAPPA)


def pbe_x(rho, gamma):
    kf = (3.0 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    s2 = gamma / (4.0 * kf ** 2 * rho ** 2)
    return slater_x(rho) * pbe_fx(s2)


def pbe_h(rs, t2):
    """PBE gradient correction H(rs, t^2) to the correlation energy per particle (phi = 1)."""
    ec = pw92_eps(rs)
    A = (PBE_BETA / PBE_GAMMA) / (np.exp(-ec / PBE_GAMMA) - 1.0)
    y = A * t2
    return PBE_GAMMA * np.log(1.0 + (PBE_BETA / PBE_GAMMA) * t2 * (1.0 + y) / (1.0 + y + y * y))


def pbe_c(rho, gamma):
    rs = wigner_rs(rho)
    kf = (3.0 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    ks2 = 4.0 * kf / np.pi
    t2 = gamma / (4.0 * ks2 * rho ** 2)
    return rho * (pw92_eps(rs) + pbe_h(rs, t2))


def pbe_xc(rho, gamma):
    return pbe_x(rho, gamma) + pbe_c(rho, gamma)


FUNCTIONALS = {SLATER: slater_x, LDA: lda_xc, PBE: pbe_xc}


def eps_and_derivs(functional, rho, gamma):
    """eps, E^rho = d eps / d rho, E^gamma = d eps / d gamma by complex steps; zero where
    rho < RHO_MIN."""
    f = FUNCTIONALS[functional]
    rho = np.asarray(rho, np.float64)
    gamma = np.asarray(gamma, np.float64)
    ok = rho >= RHO_MIN
    r, g = rho[ok], gamma[ok]
    hr = 1e-20 * r
    hg = 1e-20 * np.maximum(g, 1e-20)
    e = np.zeros_like(rho)
    er = np.zeros_like(rho)
    eg = np.zeros_like(rho)
    e[ok] = np.real(f(r.astype(complex), g.astype(complex)))
    er[ok] = np.imag(f(r + 1j * hr, g.astype(complex))) / hr
    if functional == PBE:
        eg[ok] = np.imag(f(r.astype(complex), g + 1j * hg)) / hg
    return e, er, eg


# ---------------------------------------------------------------------------------------------
# the potential matrix
# ---------------------------------------------------------------------------------------------

def vxc(s, functional, P=None, xyz=None, w=None, chunk=20000):
    """(V^xc [nbf, nbf], E_xc, N_el) on the system's grid."""
    P = np.asarray(s.P if P is None else P, np.float64)
    xyz = np.asarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    w = np.asarray(s.grid_w if w is None else w, np.float64)
    nbf = P.shape[0]
    V = np.zeros((nbf, nbf))
    exc = 0.0
    nel = 0.0
    for i0 in range(0, len(w), chunk):
        X = xyz[i0:i0 + chunk]
        wi = w[i0:i0 + chunk]
        phi, dphi = collocate_grad(s, X)
        F = P @ phi                                        # Eq. fmat
        rho = np.sum(F * phi, axis=0)                      # Eq. den_grid
        grad = 2.0 * np.einsum("mi,qmi->qi", F, dphi)
        gamma = np.sum(grad * grad, axis=0)
        e, er, eg = eps_and_derivs(functional, rho, gamma)  # Eq. exc_grid
        Z = 0.5 * wi[None, :] * (er[None, :] * phi + 4.0 * eg[None, :] * np.einsum("qi,qmi->mi", grad, dphi))
        V += phi @ Z.T + Z @ phi.T                         # Eq. vxc_num
        exc += float(np.sum(wi * e))
        nel += float(np.sum(wi * rho))
    return V, exc, nel


def exc_only(s, functional, P, xyz=None, w=None, chunk=20000):
    """E_xc for a density matrix P (the finite-difference pins of V^xc)."""
    xyz = np.asarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    w = np.asarray(s.grid_w if w is None else w, np.float64)
    exc = 0.0
    for i0 in range(0, len(w), chunk):
        phi, dphi = collocate_grad(s, xyz[i0:i0 + chunk])
        F = P @ phi
        rho = np.sum(F * phi, axis=0)
        grad = 2.0 * np.einsum("mi,qmi->qi", F, dphi)
        e, _, _ = eps_and_derivs(functional, rho, np.sum(grad * grad, axis=0))
        exc += float(np.sum(w[i0:i0 + chunk] * e))
    return exc
