"""Algorithmic work model of the 3c-CP digestion step (App. A, Eqs. vrr, hrr, gmat).

Counts the floating-point operations the recursions need as written, walking
them term by term (add/sub/mul = 1, fused multiply-add = 2):

per primitive pair and grid point
  - P - r_i and T = zeta_p |P - r_i|^2                                  9
  - Boys function F_0..F_L, charged at the cost of the evaluation the    2 + 22 (L + 1)
    kernels use for T < 50 (nearly every evaluation): a table node and
    offset, then an 11-term Taylor series in the offset for each order
    (10 fused multiply-adds)
  - base case Theta^n_0 = pref F_n                                      L + 1
  - each VRR term: PA_q Theta^n - PC_q Theta^{n+1}                      3
    plus, when a_q > 0, a_q/(2 zeta_p) (Theta^n_{a-1} - Theta^{n+1}_{a-1})  4 more
  - contraction of Theta^0 over primitives (one add per target)
per shell pair and grid point
  - each HRR term                                                        2
  - digestion G_a += A F_b and G_b += A^T F_a                           4 n_a n_b
  - weights and component norms on the updates                          2 (n_a + n_b)

The model is the unit of the reported FLOP rates; the kernels execute more
instructions than this (table-driven Boys branch, address arithmetic).
"""
from __future__ import annotations

from functools import lru_cache
from typing import Tuple


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def comps(l: int):
    out = []
    for x in range(l, -1, -1):
        for y in range(l - x, -1, -1):
            out.append((x, y, l - x - y))
    return out


def _dir(c) -> int:
    return 0 if c[0] > 0 else (1 if c[1] > 0 else 2)


@lru_cache(maxsize=None)
def per_prim_pair(la: int, lb: int) -> int:
    L = la + lb
    f = 9 + (2 + 22 * (L + 1)) + (L + 1)
    for l in range(1, L + 1):
        for c in comps(l):
            q = _dir(c)
            am = c[q] - 1
            for _n in range(0, L - l + 1):
                f += 3 + (4 if am > 0 else 0)
    f += sum(ncart(l) for l in range(la, L + 1))
    return f


@lru_cache(maxsize=None)
def per_shell_pair(la: int, lb: int) -> int:
    f = 0
    for lbp in range(1, lb + 1):
        for _cb in comps(lbp):
            for lap in range(la, la + lb - lbp + 1):
                f += 2 * ncart(lap)
    na, nb = ncart(la), ncart(lb)
    return f + 4 * na * nb + 2 * (na + nb)


CLASS_L: Tuple[Tuple[int, int], ...] = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2))


def class_flops(cls: int, pair_points: int, prim_pair_points: int) -> float:
    la, lb = CLASS_L[cls]
    return float(prim_pair_points) * per_prim_pair(la, lb) + float(pair_points) * per_shell_pair(la, lb)


def nherm(l: int) -> int:
    """Hermite components t + u + v <= l."""
    return (l + 1) * (l + 2) * (l + 3) // 6


@lru_cache(maxsize=None)
def dfj_pair_aux(lp: int, lc: int) -> int:
    """Flops of one (orbital primitive pair of total angular momentum lp, auxiliary shell lc)
    term of the Coulomb build's digestion (Sec. II.B, Eqs. pc, md1, cabP-jengine):
      - P - C, alpha = zeta_p zeta_c / (zeta_p + zeta_c), T = alpha |P - C|^2        12
      - Boys function F_0..F_N, N = lp + lc, as above                            2 + 22 (N + 1)
      - (-2 alpha)^n, n <= N                                                     N
      - Eq. md1: R^(n)_tuv for t + u + v <= N - n; the first of each level one
        multiply, the others a multiply plus, with a lower index > 1, one fused
        multiply-add                                                             1, 1 or 3
      - prefactor 2 pi^(5/2) / (zeta_p zeta_c sqrt(zeta_p + zeta_c))             4
      - digestion sum_c~ (p~|c~) D_c~ per p~ and its update with the prefactor    2 nherm(lc) + 2
    The same count serves the v pass (Eq. V_df), which digests the pair's Hermite density
    against the same integrals."""
    n_all = lp + lc
    f = 12 + 2 + 22 * (n_all + 1) + n_all + 4
    for n in range(n_all + 1):
        top = n_all - n
        for t in range(top + 1):
            for u in range(top + 1 - t):
                for v in range(top + 1 - t - u):
                    if t + u + v == 0:
                        f += 1
                    else:
                        k = t if t > 0 else (u if u > 0 else v)
                        f += 3 if k > 1 else 1
    return f + nherm(lp) * (2 * nherm(lc) + 2)


# MI355X (gfx950) peaks used for roofline fractions
PEAK_FP64_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6: 256 CU x 4 SIMD x 16 lanes x FMA x 2.4 GHz
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
