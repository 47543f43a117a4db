"""The density-fitted Coulomb matrix of Sec. II.B (Eqs. V_df, P_df, J_df), written out from
its definition.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the product path.  It imports
nothing from the HIP library's package: the orbital system and the auxiliary basis are passed
duck-typed (shell arrays as in ``oracle.py``).

  (mu nu | K) = int int phi_mu(r) phi_nu(r) chi_K(r') / |r - r'|
  V_KL        = int int chi_K(r) chi_L(r') / |r - r'|
  v_L         = sum_{lam kap} (L | lam kap) D_lam kap                  (Eq. V_df)
  d_K         = sum_L (V^-1)_KL v_L                                   (Eq. P_df)
  J_mu nu     = sum_K (mu nu | K) d_K                                 (Eq. J_df)

The integrals come from the oracle's four-centre routine with the constant function 1 (an s
Gaussian of exponent 0) as the fourth function; V^-1 v is a dense solve in FP64.
"""
from __future__ import annotations

import types

import numpy as np

from . import oracle as O


def combined(s, aux):
    """Orbital shells, then auxiliary shells, then the constant function (one s shell)."""
    center = np.concatenate([np.asarray(s.shell_center, np.float64).reshape(-1, 3),
                             np.asarray(aux.shell_center, np.float64).reshape(-1, 3), np.zeros((1, 3))])
    l = np.concatenate([s.shell_l, aux.shell_l, [0]]).astype(np.int32)
    nprim = np.concatenate([s.shell_nprim, aux.shell_nprim, [1]]).astype(np.int32)
    nexp = len(s.exps)
    off = np.concatenate([s.shell_prim_off, np.asarray(aux.shell_prim_off) + nexp,
                          [nexp + len(aux.exps)]]).astype(np.int32)
    exps = np.concatenate([s.exps, aux.exps, [0.0]])
    coefs = np.concatenate([s.coefs, aux.coefs, [1.0]])
    return types.SimpleNamespace(shell_center=center, shell_l=l, shell_nprim=nprim, shell_prim_off=off,
                                 exps=exps, coefs=coefs)


def tensors(s, aux, nthreads: int = 0):
    """(T, V): T[mu, nu, K] = (mu nu | K), V[K, L] = (K | L)."""
    c = combined(s, aux)
    b = O._Basis(c)
    norb, naux = len(s.shell_l), len(aux.shell_l)
    nbf = int(sum((int(x) + 1) * (int(x) + 2) // 2 for x in s.shell_l))
    nauxf = int(sum((int(x) + 1) * (int(x) + 2) // 2 for x in aux.shell_l))
    T = np.zeros((nbf, nbf, nauxf))
    V = np.zeros((nauxf, nauxf))
    rc = O.lib().orc_df_tensors(*b.args(), norb, naux, O._dp(T), O._dp(V), int(nthreads))
    if rc != 0:
        raise ValueError("combined basis does not end with the constant function")
    return T, V


def dfj(s, aux, P=None, T=None, V=None):
    """(J, v, d, E_J) with E_J = 1/2 tr(P J)."""
    P = np.asarray(s.P if P is None else P, np.float64)
    if T is None or V is None:
        T, V = tensors(s, aux)
    v = np.einsum("mnk,mn->k", T, P)
    d = np.linalg.solve(V, v)
    J = T @ d
    return J, v, d, 0.5 * float(np.sum(P * J))
