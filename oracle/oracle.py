"""Python access to the CPU FP64 oracle (``snk_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product path.  It imports
nothing from the HIP library's package; systems are passed duck-typed (any
object with the basis/grid/density fields of a generated system).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "snk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            basis = [ctypes.c_int, _D, _I, _I, _I, _D, _D]
            L.orc_boys.argtypes = [ctypes.c_int, ctypes.c_double]
            L.orc_boys.restype = ctypes.c_double
            L.orc_nbf.argtypes = [ctypes.c_int, _I]
            L.orc_nbf.restype = ctypes.c_int
            L.orc_collocate.argtypes = basis + [ctypes.c_long, _D, _D]
            L.orc_collocate.restype = None
            L.orc_overlap.argtypes = basis + [_D]
            L.orc_overlap.restype = None
            L.orc_a3c.argtypes = basis + [_D, _D]
            L.orc_a3c.restype = None
            L.orc_snk.argtypes = basis + [ctypes.c_long, _D, _D, _D, _D, _D, ctypes.c_int]
            L.orc_snk.restype = ctypes.c_int
            L.orc_snk_rows.argtypes = basis + [ctypes.c_long, _D, _D, _D, _I, ctypes.c_int, _D, ctypes.c_int]
            L.orc_snk_rows.restype = ctypes.c_int
            L.orc_eri_j.argtypes = basis + [_D, _D, ctypes.c_int]
            L.orc_eri_j.restype = ctypes.c_int
            L.orc_df_tensors.argtypes = basis + [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int]
            L.orc_df_tensors.restype = ctypes.c_int
            L.orc_eri_shells.argtypes = basis + [ctypes.c_int] * 4 + [_D]
            L.orc_eri_shells.restype = None
            L.orc_eri_k.argtypes = basis + [_D, _D, ctypes.c_int]
            L.orc_eri_k.restype = ctypes.c_int
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _ip(a):
    return a.ctypes.data_as(_I)


class _Basis:
    def __init__(self, s):
        self.center = np.ascontiguousarray(s.shell_center, np.float64).reshape(-1)
        self.l = np.ascontiguousarray(s.shell_l, np.int32)
        self.nprim = np.ascontiguousarray(s.shell_nprim, np.int32)
        self.prim_off = np.ascontiguousarray(s.shell_prim_off, np.int32)
        self.exps = np.ascontiguousarray(s.exps, np.float64)
        self.coefs = np.ascontiguousarray(s.coefs, np.float64)
        self.nshell = int(self.l.shape[0])
        self.nbf = int(sum((l + 1) * (l + 2) // 2 for l in self.l))

    def args(self):
        return [self.nshell, _dp(self.center), _ip(self.l), _ip(self.nprim), _ip(self.prim_off),
                _dp(self.exps), _dp(self.coefs)]


def boys(m: int, x: float) -> float:
    return lib().orc_boys(int(m), float(x))


def collocate(s, xyz=None) -> np.ndarray:
    """Phi[mu, i] = phi_mu(r_i)."""
    b = _Basis(s)
    xyz = np.ascontiguousarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    out = np.zeros((b.nbf, len(xyz)))
    lib().orc_collocate(*b.args(), len(xyz), _dp(xyz), _dp(out))
    return out


def overlap(s) -> np.ndarray:
    b = _Basis(s)
    out = np.zeros((b.nbf, b.nbf))
    lib().orc_overlap(*b.args(), _dp(out))
    return out


def a3c(s, C) -> np.ndarray:
    """A_{mu lam}(C) = int phi_mu phi_lam / |r - C| over all function pairs."""
    b = _Basis(s)
    C = np.ascontiguousarray(C, np.float64).reshape(3)
    out = np.zeros((b.nbf, b.nbf))
    lib().orc_a3c(*b.args(), _dp(C), _dp(out))
    return out


def snk(s, P=None, xyz=None, w=None, nthreads: int = 0):
    """Plain sn-K: returns (K, E_x = -1/2 tr(PK), E_x = -1/2 sum F*G)."""
    b = _Basis(s)
    P = np.ascontiguousarray(s.P if P is None else P, np.float64)
    xyz = np.ascontiguousarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(s.grid_w if w is None else w, np.float64)
    assert P.shape == (b.nbf, b.nbf) and len(w) == len(xyz)
    K = np.zeros((b.nbf, b.nbf))
    ex = np.zeros(2)
    rc = lib().orc_snk(*b.args(), len(w), _dp(xyz), _dp(w), _dp(P), _dp(K), _dp(ex), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle sn-K failed")
    return K, float(ex[0]), float(ex[1])


def snk_rows(s, rows, P=None, xyz=None, w=None, nthreads: int = 0) -> np.ndarray:
    """Rows `rows` of the unsymmetrised sn-K matrix Kt = G Phi^T (len(rows) x nbf)."""
    b = _Basis(s)
    P = np.ascontiguousarray(s.P if P is None else P, np.float64)
    xyz = np.ascontiguousarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(s.grid_w if w is None else w, np.float64)
    r = np.ascontiguousarray(rows, np.int32)
    assert P.shape == (b.nbf, b.nbf) and len(w) == len(xyz) and r.min() >= 0 and r.max() < b.nbf
    out = np.zeros((len(r), b.nbf))
    rc = lib().orc_snk_rows(*b.args(), len(w), _dp(xyz), _dp(w), _dp(P), _ip(r), len(r), _dp(out), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle sn-K rows failed")
    return out


def k_block(s, rows, **kw) -> np.ndarray:
    """K[rows][rows] = (Kt + Kt^T)/2 restricted to `rows` (Eq. sn_k), from snk_rows."""
    Kt = snk_rows(s, rows, **kw)
    sub = Kt[:, np.asarray(rows)]
    return 0.5 * (sub + sub.T)


def eri_shells(s, sa, sb, sc, sd) -> np.ndarray:
    b = _Basis(s)
    n = [(int(s.shell_l[x]) + 1) * (int(s.shell_l[x]) + 2) // 2 for x in (sa, sb, sc, sd)]
    out = np.zeros(int(np.prod(n)))
    lib().orc_eri_shells(*b.args(), int(sa), int(sb), int(sc), int(sd), _dp(out))
    return out.reshape(n)


def eri_k(s, P=None, nthreads: int = 0) -> np.ndarray:
    """Exact exchange K_{mu nu} = sum (mu lam|nu kap) P_{lam kap} from four-centre ERIs."""
    b = _Basis(s)
    P = np.ascontiguousarray(s.P if P is None else P, np.float64)
    K = np.zeros((b.nbf, b.nbf))
    lib().orc_eri_k(*b.args(), _dp(P), _dp(K), int(nthreads))
    return K


def eri_j(s, P=None, nthreads: int = 0) -> np.ndarray:
    """Coulomb matrix J_{mu nu} = sum (mu nu | lam kap) P_{lam kap} from all four-centre integrals."""
    b = _Basis(s)
    P = np.ascontiguousarray(s.P if P is None else P, np.float64)
    J = np.zeros((b.nbf, b.nbf))
    if lib().orc_eri_j(*b.args(), _dp(P), _dp(J), int(nthreads)) != 0:
        raise MemoryError("oracle J failed")
    return J


def exchange_energy(P: np.ndarray, K: np.ndarray) -> float:
    """E_x = -1/2 tr(P K)."""
    return -0.5 * float(np.sum(P * K.T))
