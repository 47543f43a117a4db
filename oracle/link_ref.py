"""The sn-LinK pair selection of Sec. II.E (Eqs. sp_set and exx_fmat_approx), written out from
its definition with numpy, one batch at a time.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.  It imports
nothing from the HIP library's package; systems are passed duck-typed (shell arrays, grid and
density as in ``oracle.py``), and the collocation comes from the oracle's C code.

For one quadrature batch Q_j (points r_i with weights w_i) and the functions B_j that may
be non-negligible on it:

  Phi~_nu  = max_{i in Q_j} sqrt(w_i) |Phi_nu,i|
  F~_mu    = sum_{nu in B_j} |D_mu,nu| Phi~_nu                    (Eq. exx_fmat_approx, mu over the
                                                                   whole basis)
  phi~     = max_{i in Q_j} sqrt(w_i) sum_{mu in B_j} |Phi_mu,i|
  eps^E_AB = F~_A F~_B A~_AB
  eps^K_AB = max(F~_A, F~_B) phi~ A~_AB
  (A, B) is kept on Q_j when eps^E_AB >= eps_E or eps^K_AB >= eps_K   (Eq. sp_set)

Readings (the paper states the selection per function pair and takes A~ from a global
upper-bound estimate it does not print):
  * the selection is made per shell pair: F~ of a shell is the largest F~ of its functions;
  * A~_AB = max(1, |R_A - R_B|)^(l_A + l_B) sum |(2 pi / zeta_p) exp(-zeta_a zeta_b |AB|^2 / zeta_p) c_a c_b|
    over the primitive pairs (a, b) whose term is at least 1e-30 (zeta_p = zeta_a + zeta_b);
    a pair with no such primitive pair is never kept.  For two s shells this bounds
    |A_ab(r)| at every r, since F_0 <= 1;
  * eps_E = eps_K = eps.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def _ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def shell_offsets(s) -> np.ndarray:
    off = np.zeros(len(s.shell_l) + 1, np.int64)
    off[1:] = np.cumsum([_ncart(int(l)) for l in s.shell_l])
    return off


def a_tilde(s) -> np.ndarray:
    """A~[A, B] (symmetric, nshell x nshell): the global estimate of max_r |A_ab(r)|."""
    n = len(s.shell_l)
    out = np.zeros((n, n))
    for A in range(n):
        pa = slice(int(s.shell_prim_off[A]), int(s.shell_prim_off[A] + s.shell_nprim[A]))
        for B in range(A + 1):
            pb = slice(int(s.shell_prim_off[B]), int(s.shell_prim_off[B] + s.shell_nprim[B]))
            RA, RB = np.asarray(s.shell_center[A]), np.asarray(s.shell_center[B])
            ab2 = float(np.sum((RA - RB) ** 2))
            grow = max(1.0, math.sqrt(ab2)) ** (int(s.shell_l[A]) + int(s.shell_l[B]))
            total = 0.0
            for za, ca in zip(s.exps[pa], s.coefs[pa]):
                for zb, cb in zip(s.exps[pb], s.coefs[pb]):
                    zp = za + zb
                    term = abs(2.0 * math.pi / zp * math.exp(-za * zb / zp * ab2) * ca * cb) * grow
                    if term >= 1e-30:
                        total += term
            out[A, B] = out[B, A] = total
    return out


def batch_estimates(s, pts, P=None, funcs=None):
    """(F~ per function, F~ per shell, phi~) of the batch of input points `pts` (Eqs. exx_fmat_approx and the
    phi~ definition); `funcs`: the function indices B_j (default: the whole basis)."""
    P = np.asarray(s.P if P is None else P, np.float64)
    pts = np.asarray(pts, np.int64)
    nbf = P.shape[0]
    funcs = np.arange(nbf) if funcs is None else np.asarray(funcs, np.int64)
    sw = np.sqrt(np.asarray(s.grid_w, np.float64)[pts])
    phi = O.collocate(s, np.asarray(s.grid_xyz, np.float64)[pts])[funcs]     # |B_j| x |Q_j|
    phi_t = np.max(np.abs(phi) * sw[None, :], axis=1) if len(pts) else np.zeros(len(funcs))
    Ft = np.abs(P[:, funcs]) @ phi_t                                          # every mu of the basis
    phit = float(np.max(sw * np.sum(np.abs(phi), axis=0))) if len(pts) else 0.0
    off = shell_offsets(s)
    Fs = np.array([np.max(Ft[off[k]:off[k + 1]]) for k in range(len(off) - 1)])
    return Ft, Fs, phit


def kept_pairs(s, pts, eps: float, P=None, funcs=None, at=None):
    """Eq. sp_set for one batch.  Returns (kept, margin), both nshell x nshell lower-triangular
    (A >= B): kept[A, B] is the decision, margin[A, B] = max(eps^E, eps^K) / eps (NaN when eps
    is 0), from which a caller can tell decisions that rounding could turn."""
    at = a_tilde(s) if at is None else at
    _, Fs, phit = batch_estimates(s, pts, P, funcs)
    eE = np.outer(Fs, Fs) * at
    eK = np.maximum(Fs[:, None], Fs[None, :]) * phit * at
    kept = ((eE >= eps) | (eK >= eps)) & (at > 0.0)
    low = np.tril(np.ones_like(kept, dtype=bool))
    margin = np.maximum(eE, eK) / eps if eps > 0 else np.full(kept.shape, np.nan)
    return kept & low, np.where(low, margin, np.nan)
