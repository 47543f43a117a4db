"""Pins of the oracle's sn-K build (Eqs. fmat, gmat, usym_k, sn_k) against invariants,
closed forms and brute-force exact exchange from four-centre integrals (Eq. full_k)."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_snk_invariants_config1():
    s = synth.make_system(1, grid=(30, 110))
    K, ex_tr, ex_fg = O.snk(s)
    assert np.array_equal(K, K.T)                      # Eq. sn_k symmetrises exactly
    assert ex_tr < 0                                   # tr(PK) = sum_i w_i F_i^T A(r_i) F_i >= 0
    assert abs(ex_tr - ex_fg) < 1e-12 * abs(ex_tr)     # -1/2 tr(PK) = -1/2 sum F*G
    # independent of the thread count (fixed chunking, pairwise sums)
    K1, e1, _ = O.snk(s, nthreads=1)
    assert np.array_equal(K1, K) and e1 == ex_tr


def test_snk_linear_in_density():
    s = synth.make_system(1, grid=(20, 50))
    P1 = s.P
    P2 = synth.random_symmetric(s.nbf, 1)
    K1 = O.snk(s, P=P1)[0]
    K2 = O.snk(s, P=P2)[0]
    K12 = O.snk(s, P=0.7 * P1 - 1.9 * P2)[0]
    assert np.max(np.abs(K12 - (0.7 * K1 - 1.9 * K2))) < 1e-12 * np.max(np.abs(K12))


def test_snk_single_s_primitive_closed_form():
    # one normalised s primitive, P = [p]:  K -> p (ss|ss) = p 2 sqrt(zeta/pi), E_x -> -p^2 sqrt(zeta/pi)
    z, p = 0.8, 1.7
    s = synth.make_custom([1], [[0.0, 0.0, 0.0]], [[(0, [z], [1.0])]], grid=(120, 302), n_occ=1)
    K, ex, _ = O.snk(s, P=np.array([[p]]))
    assert abs(K[0, 0] - p * 2 * math.sqrt(z / math.pi)) < 1e-9
    assert abs(ex + p * p * math.sqrt(z / math.pi)) < 1e-9


def test_snk_weights_enter_once():
    # doubling every weight doubles K (G carries w_i exactly once, Eq. gmat)
    s = synth.make_system(1, grid=(20, 50))
    K = O.snk(s)[0]
    K2 = O.snk(s, w=2.0 * s.grid_w)[0]
    assert np.max(np.abs(K2 - 2.0 * K)) < 1e-13 * np.max(np.abs(K))


def test_snk_point_partition_additivity():
    # K is a sum over grid points (Sec. II.E): two disjoint halves add up to the whole
    s = synth.make_system(1, grid=(20, 50))
    idx = np.arange(s.npts)
    a, b = idx[idx % 3 == 0], idx[idx % 3 != 0]
    K = O.snk(s)[0]
    Ka = O.snk(s.subset_points(a))[0]
    Kb = O.snk(s.subset_points(b))[0]
    assert np.max(np.abs(Ka + Kb - K)) < 1e-13 * np.max(np.abs(K))


def test_snk_converges_to_exact_exchange():
    """sn-K is a quadrature of the r' integral in the ERIs (Eq. sn_eri), so it converges to
    the four-centre exact exchange as the grid is refined."""
    g = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    Kx = g["K_exact"]
    base = synth.make_system(1)
    ex_exact = O.exchange_energy(base.P, Kx)
    assert ex_exact < 0
    errE, errK = [], []
    for grid in [(20, 50), (35, 86), (50, 110), (75, 194), (75, 302)]:
        s = synth.make_system(1, grid=grid)
        K, ex, _ = O.snk(s)
        errE.append(abs(ex - ex_exact))
        errK.append(np.max(np.abs(K - Kx)))
    drops = sum(1 for i in range(len(errE) - 1) if errE[i + 1] > errE[i])
    assert drops <= 1, errE
    assert errE[-1] < errE[0] / 100.0, errE
    assert errK[-1] < errK[0] / 30.0, errK


def test_exact_exchange_properties():
    g = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    Kx = g["K_exact"]
    assert np.max(np.abs(Kx - Kx.T)) < 1e-13 * np.max(np.abs(Kx))
    # exchange of a PSD density is PSD
    ev = np.linalg.eigvalsh(0.5 * (Kx + Kx.T))
    assert ev.min() > -1e-10 * ev.max()


def test_golden_config1_reproduces():
    g = np.load(os.path.join(GOLDEN, "oracle_config1.npz"))
    s = synth.make_system(1)
    # the generator reproduces the stored density to rounding
    assert np.max(np.abs(s.P - g["P"])) < 1e-12
    K, ex, _ = O.snk(s.with_density(g["P"]))
    assert abs(ex - g["ex"][0]) < 1e-12 * abs(ex)
    assert np.max(np.abs(K - g["K"])) < 1e-13 * np.max(np.abs(K))


@pytest.mark.parametrize("cfg", [1, 2])
def test_stored_inputs_fingerprint(cfg):
    import importlib.util
    path = os.path.join(GOLDEN, "oracle_config%d.npz" % cfg)
    if not os.path.exists(path):
        pytest.skip("no stored result")
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(GOLDEN, "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g = np.load(path)
    s = synth.make_system(cfg)
    assert np.allclose(mg.fingerprint(s), g["fingerprint"], rtol=1e-12, atol=0)
    assert np.max(np.abs(s.P - g["P"])) < 1e-12


@pytest.mark.parametrize("which", ["config1", "soft_spd"])
def test_rows_match_full_oracle(which):
    """orc_snk_rows (selected rows of the unsymmetrised matrix, for sampling large systems)
    against the full oracle: K[S][S] from the rows equals the full K on S x S."""
    if which == "config1":
        s = synth.make_system(1, grid=(20, 50))
    else:
        xyz = [[0.0, 0.0, 0.0], [1.3, 0.4, -0.2], [-0.5, 1.1, 0.7]]
        shells = [
            [(0, [2.1, 0.6], [0.5, 0.6]), (1, [1.4, 0.45], [0.7, 0.4]), (2, [0.9], [1.0])],
            [(0, [1.7, 0.5], [0.4, 0.7]), (1, [0.8], [1.0])],
            [(0, [1.1], [1.0]), (2, [1.3, 0.5], [0.5, 0.5]), (1, [30.0, 3.0, 0.3], [0.3, 0.5, 0.4])],
        ]
        s = synth.make_custom([8, 1, 1], xyz, shells, grid=(16, 50), n_occ=3)
    K, ex, _ = O.snk(s)
    rows = np.sort(np.random.default_rng(3).choice(s.nbf, size=min(9, s.nbf), replace=False))
    Kb = O.k_block(s, rows)
    assert np.max(np.abs(Kb - K[np.ix_(rows, rows)])) <= 1e-13 * np.max(np.abs(K))
    Kt = O.snk_rows(s, np.arange(s.nbf))
    assert np.max(np.abs(0.5 * (Kt + Kt.T) - K)) <= 1e-13 * np.max(np.abs(K))
