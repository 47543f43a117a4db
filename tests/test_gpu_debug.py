"""Step-by-step checks of the HIP path: matrix-core lane layout, the FP64 GEMM, and the
intermediates Phi (Eq. collocation), F (Eq. fmat) and G (Eq. gmat) against the oracle."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import snk, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_mfma_f64_layout():
    out = snk.debug_mfma_layout().reshape(64, 4)
    say("mfma probe lane0..3:", out[:4].tolist())
    for lane in range(64):
        for r in range(4):
            v = out[lane, r]
            j, i = int(v) // 100, int(v) % 100
            say_ok = (i == 4 * r + lane // 16) and (j == lane % 16)
            if not say_ok:
                say("lane", lane, "r", r, "holds D[%d][%d]" % (i, j))
            assert say_ok


@pytest.mark.parametrize("tile", [64, 128, 192, 384])
@pytest.mark.parametrize("bt", [False, True])
@pytest.mark.parametrize("shape", [(100, 130, 77), (300, 517, 333), (1, 1, 1), (129, 257, 16)])
def test_gemm_f64_vs_numpy(bt, shape, tile):
    """The grouped matrix-core product on one problem: ragged edges of the output tiles (64 x 64,
    128 x 128, 64 x 128, 128 x 256) and of the 16-wide k steps, several tiles in both directions."""
    import torch
    rng = np.random.default_rng(1)
    M, N, K = shape
    A = rng.normal(size=(M, K))
    B = rng.normal(size=(N, K)) if bt else rng.normal(size=(K, N))
    ref = A @ (B.T if bt else B)
    Ad = torch.tensor(A, device="cuda")
    Bd = torch.tensor(B, device="cuda")
    Cd = torch.full((M, N), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    say("gemm bt", bt, "shape", shape, "tile", tile)
    snk.debug_gemm_f64(M, N, K, Ad.data_ptr(), K, Bd.data_ptr(), K if bt else N, bt, Cd.data_ptr(), N, tile=tile)
    torch.cuda.synchronize()
    C = Cd.cpu().numpy()
    err = np.max(np.abs(C - ref))
    say("  max err", err)
    assert err < 1e-12


def test_intermediates_vs_oracle():
    s = synth.make_system(1, grid=(12, 26))
    ctx = snk.Context(s)
    order = ctx.point_order()
    say("intermediates: npts", s.npts, "cols", len(order))
    Phi, F, G = ctx.debug_intermediates(s.P)
    real = np.nonzero(order >= 0)[0]
    pts = order[real]
    PhiR = O.collocate(s, s.grid_xyz[pts])
    e_phi = np.max(np.abs(Phi[:, real] - PhiR))
    FR = s.P @ PhiR
    e_f = np.max(np.abs(F[:, real] - FR))
    say("  Phi err", e_phi, "F err", e_f)
    sel = real[:: max(1, len(real) // 40)]
    GR = np.zeros((s.nbf, len(sel)))
    for k, col in enumerate(sel):
        p = order[col]
        A = O.a3c(s, s.grid_xyz[p])
        GR[:, k] = s.grid_w[p] * (A @ (s.P @ O.collocate(s, s.grid_xyz[p:p + 1])[:, 0]))
    e_g = np.max(np.abs(G[:, sel] - GR)) / np.max(np.abs(GR))
    say("  G rel err", e_g)
    assert e_phi < 1e-13 and e_f < 1e-12 and e_g < 1e-12
