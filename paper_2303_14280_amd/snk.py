"""Thin ctypes binding of the sn-K C ABI (include/snk.h).

Argument marshalling only: every step of the build runs in the HIP library
``libsnk.so``.  Importing this module does not load the library; the first call
does, and it raises if the library has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnk.so")

SNK_OK, SNK_E_ARG, SNK_E_UNSUPPORTED, SNK_E_NOMEM, SNK_E_DEVICE, SNK_E_ASYM = range(6)
SNK_FP64, SNK_MIXED = 0, 1
SNK_SCREEN_NONE, SNK_SCREEN_BOUND, SNK_SCREEN_LEARNED = 0, 1, 2
SNK_DEVICE_PTRS = 0x1
SNK_VALIDATE = 0x2
CLASSES = ("ss", "ps", "pp", "ds", "dp", "dd")
CLASS_L = ((0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2))

_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)


class SnkBasis(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int32), ("center", _D), ("l", _I32), ("nprim", _I32),
                ("prim_off", _I32), ("exps", _D), ("coefs", _D)]


class SnkGrid(ctypes.Structure):
    _fields_ = [("npts", ctypes.c_int64), ("xyz", _D), ("atom_of_point", _I32)]


class SnkStats(ctypes.Structure):
    _fields_ = [("ex", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("t_collocate_ms", ctypes.c_double),
                ("t_fgemm_ms", ctypes.c_double), ("t_screen_ms", ctypes.c_double), ("t_afg_ms", ctypes.c_double),
                ("t_kgemm_ms", ctypes.c_double), ("t_finish_ms", ctypes.c_double),
                ("pair_points", ctypes.c_int64 * 6), ("pair_points_skipped", ctypes.c_int64),
                ("pair_points_lowprec", ctypes.c_int64), ("skipped_bound", ctypes.c_double),
                ("n_batches", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("prim_pair_points", ctypes.c_int64 * 6), ("t_afg_class_ms", ctypes.c_double * 6)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("pair_points", "prim_pair_points", "t_afg_class_ms"):
            d[k] = list(d[k])
        return d


class SnkOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("screen", ctypes.c_int32), ("screener", ctypes.c_void_p),
                ("eps_basis", ctypes.c_double), ("eps_skip_energy", ctypes.c_double),
                ("eps_lowprec_energy", ctypes.c_double), ("batch_points", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("max_device_bytes", ctypes.c_int64),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("stats", ctypes.POINTER(SnkStats))]


_lock = threading.Lock()
_lib = None


class SnkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("sn-K library error %d (%s): %s" % (status, STATUS.get(status, "?"), msg))
        self.status = status


STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "out of memory", 4: "device error", 5: "asymmetric P"}


def lib():
    """Load libsnk.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("HIP library %s is not built; run __graft_entry__.build() "
                                   "or python -m paper_2303_14280_amd.build" % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            L.snk_opts_default.argtypes = [ctypes.POINTER(SnkOpts)]
            L.snk_opts_default.restype = None
            L.sn_k_build.argtypes = [ctypes.POINTER(SnkBasis), ctypes.POINTER(SnkGrid), _D, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.POINTER(SnkOpts)]
            L.sn_k_build.restype = ctypes.c_int
            L.snk_ctx_create.argtypes = [ctypes.POINTER(SnkBasis), ctypes.POINTER(SnkGrid), _D,
                                         ctypes.POINTER(SnkOpts), ctypes.POINTER(ctypes.c_void_p)]
            L.snk_ctx_create.restype = ctypes.c_int
            L.snk_ctx_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SnkStats)]
            L.snk_ctx_build.restype = ctypes.c_int
            L.snk_ctx_destroy.argtypes = [ctypes.c_void_p]
            L.snk_ctx_destroy.restype = None
            L.snk_ctx_nbf.argtypes = [ctypes.c_void_p]
            L.snk_ctx_nbf.restype = ctypes.c_int
            L.snk_ctx_nbatches.argtypes = [ctypes.c_void_p]
            L.snk_ctx_nbatches.restype = ctypes.c_int
            L.snk_status_string.argtypes = [ctypes.c_int]
            L.snk_status_string.restype = ctypes.c_char_p
            L.snk_last_error.argtypes = [ctypes.c_void_p]
            L.snk_last_error.restype = ctypes.c_char_p
            L.snk_version.argtypes = []
            L.snk_version.restype = ctypes.c_int
            L.snk_boys_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]
            L.snk_boys_device.restype = ctypes.c_int
            L.snk_debug_gemm_f64.argtypes = [ctypes.c_int64] * 3 + [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                                                   ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                                                   ctypes.c_int64, ctypes.c_void_p]
            L.snk_debug_gemm_f64.restype = ctypes.c_int
            L.snk_debug_mfma_layout.argtypes = [ctypes.c_void_p]
            L.snk_debug_mfma_layout.restype = ctypes.c_int
            L.snk_ctx_point_order.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.snk_ctx_point_order.restype = ctypes.c_int
            L.snk_ctx_debug_intermediates.argtypes = [ctypes.c_void_p] * 5 + [ctypes.POINTER(ctypes.c_int64)]
            L.snk_ctx_debug_intermediates.restype = ctypes.c_int
            _lib = L
    return _lib


def last_error(ctx=None) -> str:
    r = lib().snk_last_error(ctx)
    return r.decode() if r else ""


def _check(rc: int, ctx=None):
    if rc != SNK_OK:
        raise SnkError(rc, last_error(ctx))


def default_opts(**kw) -> SnkOpts:
    o = SnkOpts()
    lib().snk_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class _Marshal:
    """Holds contiguous copies of a system's basis and grid for the duration of a call."""

    def __init__(self, s, xyz=None, w=None, atom=None, use_atoms=True):
        self.center = np.ascontiguousarray(s.shell_center, np.float64).reshape(-1)
        self.l = np.ascontiguousarray(s.shell_l, np.int32)
        self.nprim = np.ascontiguousarray(s.shell_nprim, np.int32)
        self.prim_off = np.ascontiguousarray(s.shell_prim_off, np.int32)
        self.exps = np.ascontiguousarray(s.exps, np.float64)
        self.coefs = np.ascontiguousarray(s.coefs, np.float64)
        self.xyz = np.ascontiguousarray(s.grid_xyz if xyz is None else xyz, np.float64).reshape(-1)
        self.w = np.ascontiguousarray(s.grid_w if w is None else w, np.float64)
        a = s.grid_atom if atom is None else atom
        self.atom = np.ascontiguousarray(a, np.int32) if (use_atoms and a is not None) else None
        self.basis = SnkBasis(int(self.l.shape[0]), self.center.ctypes.data_as(_D), self.l.ctypes.data_as(_I32),
                              self.nprim.ctypes.data_as(_I32), self.prim_off.ctypes.data_as(_I32),
                              self.exps.ctypes.data_as(_D), self.coefs.ctypes.data_as(_D))
        self.grid = SnkGrid(int(self.w.shape[0]), self.xyz.ctypes.data_as(_D),
                            self.atom.ctypes.data_as(_I32) if self.atom is not None else None)


def nbf_of(s) -> int:
    return int(sum((int(l) + 1) * (int(l) + 2) // 2 for l in s.shell_l))


def sn_k_build(s, P: Optional[np.ndarray] = None, **opts) -> Tuple[np.ndarray, dict]:
    """One-shot build with host arrays: returns (K, stats)."""
    m = _Marshal(s)
    P = np.ascontiguousarray(s.P if P is None else P, np.float64)
    nb = nbf_of(s)
    if P.shape != (nb, nb):
        raise ValueError("P has shape %s, expected %s" % (P.shape, (nb, nb)))
    K = np.zeros((nb, nb))
    st = SnkStats()
    o = default_opts(**opts)
    o.stats = ctypes.pointer(st)
    _check(lib().sn_k_build(ctypes.byref(m.basis), ctypes.byref(m.grid), m.w.ctypes.data_as(_D),
                            P.ctypes.data, K.ctypes.data, ctypes.byref(o)))
    return K, st.as_dict()


class Context:
    """Geometry set-up once, many builds (snk_ctx_*)."""

    def __init__(self, s, xyz=None, w=None, atom=None, use_atoms=True, **opts):
        self._m = _Marshal(s, xyz, w, atom, use_atoms)
        self.opts = default_opts(**opts)
        self.device_ptrs = bool(self.opts.flags & SNK_DEVICE_PTRS)
        h = ctypes.c_void_p()
        _check(lib().snk_ctx_create(ctypes.byref(self._m.basis), ctypes.byref(self._m.grid),
                                    self._m.w.ctypes.data_as(_D), ctypes.byref(self.opts), ctypes.byref(h)))
        self.handle = h
        self.nbf = lib().snk_ctx_nbf(h)
        self.nbatches = lib().snk_ctx_nbatches(h)

    def build(self, P: np.ndarray, stats: bool = True) -> Tuple[np.ndarray, dict]:
        """Host-pointer build: returns (K, stats)."""
        if self.device_ptrs:
            raise ValueError("context was created for device pointers; use build_device")
        P = np.ascontiguousarray(P, np.float64)
        if P.shape != (self.nbf, self.nbf):
            raise ValueError("P has shape %s, expected %s" % (P.shape, (self.nbf, self.nbf)))
        K = np.zeros_like(P)
        st = SnkStats()
        _check(lib().snk_ctx_build(self.handle, P.ctypes.data, K.ctypes.data, ctypes.byref(st) if stats else None),
               self.handle)
        return K, st.as_dict()

    def build_device(self, P_ptr: int, K_ptr: int, stats: bool = False) -> Optional[dict]:
        """Device-pointer build on the context's stream (asynchronous unless stats are asked for)."""
        if not self.device_ptrs:
            raise ValueError("context was created for host pointers")
        st = SnkStats()
        _check(lib().snk_ctx_build(self.handle, ctypes.c_void_p(P_ptr), ctypes.c_void_p(K_ptr),
                                   ctypes.byref(st) if stats else None), self.handle)
        return st.as_dict() if stats else None

    def point_order(self) -> np.ndarray:
        """Input point index of every batch column (-1 = padding slot)."""
        out = np.zeros(self.nbatches * 256, np.int64)
        _check(lib().snk_ctx_point_order(self.handle, out.ctypes.data), self.handle)
        return out

    def debug_intermediates(self, P: np.ndarray):
        """(Phi, F, G) of the first batch group, each nbf x ncols (host-pointer contexts)."""
        P = np.ascontiguousarray(P, np.float64)
        n = ctypes.c_int64(0)
        _check(lib().snk_ctx_debug_intermediates(self.handle, P.ctypes.data, None, None, None, ctypes.byref(n)),
               self.handle)
        Phi = np.zeros((self.nbf, n.value))
        F = np.zeros_like(Phi)
        G = np.zeros_like(Phi)
        _check(lib().snk_ctx_debug_intermediates(self.handle, P.ctypes.data, Phi.ctypes.data, F.ctypes.data,
                                                 G.ctypes.data, ctypes.byref(n)), self.handle)
        return Phi, F, G

    def close(self):
        if getattr(self, "handle", None):
            lib().snk_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def boys_device(T_ptr: int, n: int, mmax: int, F_ptr: int, stream: int = 0):
    """F_m(T[k]) for m = 0..mmax on the device (pointers to FP64 device memory)."""
    _check(lib().snk_boys_device(ctypes.c_void_p(T_ptr), int(n), int(mmax), ctypes.c_void_p(F_ptr),
                                 ctypes.c_void_p(stream) if stream else None))


def debug_gemm_f64(M, N, K, A_ptr, lda, B_ptr, ldb, bt, C_ptr, ldc, stream: int = 0):
    _check(lib().snk_debug_gemm_f64(M, N, K, ctypes.c_void_p(A_ptr), lda, ctypes.c_void_p(B_ptr), ldb, int(bt),
                                    ctypes.c_void_p(C_ptr), ldc, ctypes.c_void_p(stream) if stream else None))


def debug_mfma_layout() -> np.ndarray:
    out = np.zeros(256)
    _check(lib().snk_debug_mfma_layout(out.ctypes.data))
    return out
