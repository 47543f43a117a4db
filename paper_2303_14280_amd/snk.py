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
SNK_SCREEN_NONE, SNK_SCREEN_BOUND, SNK_SCREEN_LEARNED, SNK_SCREEN_LINK = 0, 1, 2, 3
SNK_DEVICE_PTRS = 0x1
SNK_VALIDATE = 0x2
SNK_FP32_GEMM = 0x8
SNK_OVERLAP_GROUPS = 0x10
SNK_XC_SLATER, SNK_XC_LDA, SNK_XC_PBE = 1, 2, 3
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
                ("prim_pair_points", ctypes.c_int64 * 6), ("t_afg_class_ms", ctypes.c_double * 6),
                ("tile_functions", ctypes.c_double), ("tile_frows", ctypes.c_double), ("tile_grows", ctypes.c_double),
                ("gemm_flops_fp64", ctypes.c_double), ("gemm_flops_fp32", ctypes.c_double),
                ("lowprec_bound", ctypes.c_double), ("t_gemm_ms", ctypes.c_double * 4),
                ("gemm_launches", ctypes.c_int64 * 4), ("gemm_kind_flops", (ctypes.c_double * 2) * 4)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("pair_points", "prim_pair_points", "t_afg_class_ms", "t_gemm_ms", "gemm_launches"):
            d[k] = list(d[k])
        d["gemm_kind_flops"] = [list(r) for r in self.gemm_kind_flops]
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
            L.snk_ctx_ngroups.argtypes = [ctypes.c_void_p]
            L.snk_ctx_ngroups.restype = ctypes.c_int
            L.snk_mlp_backward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_void_p]
            L.snk_mlp_backward.restype = ctypes.c_int
            L.snk_collect_block_norms.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
            L.snk_collect_block_norms.restype = ctypes.c_int
            L.snk_shell_rcut.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                         ctypes.POINTER(ctypes.c_double)]
            L.snk_shell_rcut.restype = ctypes.c_int
            L.snk_vxc_build.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
            L.snk_vxc_build.restype = ctypes.c_int
            L.snk_ctx_build_kxc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(SnkStats)]
            L.snk_ctx_build_kxc.restype = ctypes.c_int
            L.snk_ctx_ntiles.argtypes = [ctypes.c_void_p]
            L.snk_ctx_ntiles.restype = ctypes.c_int
            L.snk_ctx_tile_info.argtypes = [ctypes.c_void_p] * 5
            L.snk_ctx_tile_info.restype = ctypes.c_int
            L.snk_ctx_tile_functions.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
            L.snk_ctx_tile_functions.restype = ctypes.c_int
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
                                                                   ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
            L.snk_debug_gemm_f64.restype = ctypes.c_int
            L.snk_debug_force_tile.argtypes = [ctypes.c_int]
            L.snk_debug_force_tile.restype = ctypes.c_int
            L.snk_debug_frow_prefilter.argtypes = [ctypes.c_int]
            L.snk_debug_frow_prefilter.restype = ctypes.c_int
            L.snk_debug_mfma_layout.argtypes = [ctypes.c_void_p]
            L.snk_debug_mfma_layout.restype = ctypes.c_int
            L.snk_ctx_point_order.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.snk_ctx_point_order.restype = ctypes.c_int
            L.snk_ctx_debug_intermediates.argtypes = [ctypes.c_void_p] * 5 + [ctypes.POINTER(ctypes.c_int64)]
            L.snk_ctx_debug_intermediates.restype = ctypes.c_int
            L.snk_ctx_nblock_pairs.argtypes = [ctypes.c_void_p]
            L.snk_ctx_nblock_pairs.restype = ctypes.c_int64
            L.snk_ctx_block_data.argtypes = [ctypes.c_void_p] * 5
            L.snk_ctx_block_data.restype = ctypes.c_int
            L.snk_ctx_npair_index.argtypes = [ctypes.c_void_p]
            L.snk_ctx_npair_index.restype = ctypes.c_int64
            L.snk_ctx_debug_learned.argtypes = [ctypes.c_void_p] * 5 + [ctypes.POINTER(ctypes.c_int64)]
            L.snk_ctx_debug_learned.restype = ctypes.c_int
            L.snk_dfj_create.argtypes = [ctypes.POINTER(SnkBasis), ctypes.POINTER(SnkBasis), ctypes.c_int,
                                         ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
            L.snk_dfj_create.restype = ctypes.c_int
            L.snk_dfj_build.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_uint32]
            L.snk_dfj_build.restype = ctypes.c_int
            L.snk_dfj_naux.argtypes = [ctypes.c_void_p]
            L.snk_dfj_naux.restype = ctypes.c_int64
            L.snk_dfj_last_error.argtypes = [ctypes.c_void_p]
            L.snk_dfj_last_error.restype = ctypes.c_char_p
            L.snk_dfj_destroy.argtypes = [ctypes.c_void_p]
            L.snk_dfj_destroy.restype = None
            L.snk_ctx_debug_kept.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
            L.snk_ctx_debug_kept.restype = ctypes.c_int
            L.snk_debug_mfma_bf16.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int]
            L.snk_debug_mfma_bf16.restype = ctypes.c_int
            _F = ctypes.POINTER(ctypes.c_float)
            L.snk_mlp_nparams.argtypes = []
            L.snk_mlp_nparams.restype = ctypes.c_int
            L.snk_mlp_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
            L.snk_mlp_create.restype = ctypes.c_int
            L.snk_mlp_destroy.argtypes = [ctypes.c_void_p]
            L.snk_mlp_destroy.restype = None
            L.snk_mlp_set_params.argtypes = [ctypes.c_void_p, _F]
            L.snk_mlp_set_params.restype = ctypes.c_int
            L.snk_mlp_get_params.argtypes = [ctypes.c_void_p, _F]
            L.snk_mlp_get_params.restype = ctypes.c_int
            L.snk_mlp_set_normalisation.argtypes = [ctypes.c_void_p, _F, _F]
            L.snk_mlp_set_normalisation.restype = ctypes.c_int
            L.snk_mlp_set_range.argtypes = [ctypes.c_void_p, _F, _F, ctypes.c_float]
            L.snk_mlp_set_range.restype = ctypes.c_int
            L.snk_mlp_forward.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_void_p]
            L.snk_mlp_forward.restype = ctypes.c_int
            L.snk_mlp_loss_grad.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
            L.snk_mlp_loss_grad.restype = ctypes.c_int
            L.snk_mlp_loss_grad_noalloc.argtypes = L.snk_mlp_loss_grad.argtypes
            L.snk_mlp_loss_grad_noalloc.restype = ctypes.c_int
            L.snk_mlp_adam_step.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float, ctypes.c_int,
                                            ctypes.c_void_p]
            L.snk_mlp_adam_step.restype = ctypes.c_int
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
        if k == "screener" and hasattr(v, "handle"):
            v = v.handle
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


class _BasisOnly:
    """Contiguous copies of one basis (orbital or auxiliary shell arrays) for a call."""

    def __init__(self, b):
        self.center = np.ascontiguousarray(b.shell_center, np.float64).reshape(-1)
        self.l = np.ascontiguousarray(b.shell_l, np.int32)
        self.nprim = np.ascontiguousarray(b.shell_nprim, np.int32)
        self.prim_off = np.ascontiguousarray(b.shell_prim_off, np.int32)
        self.exps = np.ascontiguousarray(b.exps, np.float64)
        self.coefs = np.ascontiguousarray(b.coefs, np.float64)
        self.basis = SnkBasis(int(self.l.shape[0]), self.center.ctypes.data_as(_D), self.l.ctypes.data_as(_I32),
                              self.nprim.ctypes.data_as(_I32), self.prim_off.ctypes.data_as(_I32),
                              self.exps.ctypes.data_as(_D), self.coefs.ctypes.data_as(_D))


class DfJ:
    """Density-fitted Coulomb matrix context (snk_dfj_*): orbital basis of `system`, auxiliary
    basis `aux` (shell arrays as the orbital basis, one primitive per shell)."""

    def __init__(self, system, aux, device: int = 0, stream: int = 0):
        self.handle = None
        b, a = _BasisOnly(system), _BasisOnly(aux)
        h = ctypes.c_void_p()
        rc = lib().snk_dfj_create(ctypes.byref(b.basis), ctypes.byref(a.basis), int(device),
                                  ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if rc != SNK_OK:
            raise SnkError(rc, last_error(None))
        self.handle = h
        self.nbf = int(sum((int(x) + 1) * (int(x) + 2) // 2 for x in b.l))

    @property
    def naux(self) -> int:
        return int(lib().snk_dfj_naux(self.handle))

    def _check(self, rc):
        if rc != SNK_OK:
            raise SnkError(rc, lib().snk_dfj_last_error(self.handle).decode())

    def build(self, P):
        """(J, v, d, E_J) for a host density matrix."""
        P = np.ascontiguousarray(P, np.float64)
        J = np.zeros((self.nbf, self.nbf))
        v = np.zeros(self.naux)
        d = np.zeros(self.naux)
        ej = ctypes.c_double(0.0)
        self._check(lib().snk_dfj_build(self.handle, P.ctypes.data, J.ctypes.data, v.ctypes.data, d.ctypes.data,
                                        ctypes.byref(ej), 0))
        return J, v, d, ej.value

    def build_device(self, P_ptr: int, J_ptr: int, v_ptr: int = 0, d_ptr: int = 0, energy: bool = False):
        """Device-pointer build on the context's stream; returns E_J when energy is set."""
        ej = ctypes.c_double(0.0)
        self._check(lib().snk_dfj_build(self.handle, ctypes.c_void_p(P_ptr), ctypes.c_void_p(J_ptr),
                                        ctypes.c_void_p(v_ptr) if v_ptr else None,
                                        ctypes.c_void_p(d_ptr) if d_ptr else None,
                                        ctypes.byref(ej) if energy else None, SNK_DEVICE_PTRS))
        return ej.value if energy else None

    def close(self):
        if getattr(self, "handle", None):
            lib().snk_dfj_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shell_rcut(l: int, exps, coefs, eps: float) -> float:
    """Basis screening radius of one shell (snk_shell_rcut; host only, no GPU needed)."""
    e = np.ascontiguousarray(exps, np.float64)
    c = np.ascontiguousarray(coefs, np.float64)
    r = ctypes.c_double(0.0)
    _check(lib().snk_shell_rcut(int(l), e.ctypes.data, c.ctypes.data, int(e.shape[0]), float(eps), ctypes.byref(r)))
    return r.value


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
        self._screener = opts.get("screener")   # keeps the network alive while the context uses it
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

    def vxc(self, P: np.ndarray, functional: int = SNK_XC_LDA) -> Tuple[np.ndarray, float, float]:
        """Host-pointer XC potential (snk_vxc_build): returns (V^xc, E_xc, N_el)."""
        if self.device_ptrs:
            raise ValueError("context was created for device pointers; use vxc_device")
        P = np.ascontiguousarray(P, np.float64)
        if P.shape != (self.nbf, self.nbf):
            raise ValueError("P has shape %s, expected %s" % (P.shape, (self.nbf, self.nbf)))
        V = np.zeros_like(P)
        exc, nel = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(lib().snk_vxc_build(self.handle, P.ctypes.data, int(functional), V.ctypes.data, ctypes.byref(exc),
                                   ctypes.byref(nel)), self.handle)
        return V, exc.value, nel.value

    def build_kxc(self, P: np.ndarray, functional: int = SNK_XC_LDA, stats: bool = True):
        """Host-pointer sn-K and XC build of one density (snk_ctx_build_kxc): returns
        (K, V^xc, E_xc, N_el, stats)."""
        if self.device_ptrs:
            raise ValueError("context was created for device pointers")
        P = np.ascontiguousarray(P, np.float64)
        if P.shape != (self.nbf, self.nbf):
            raise ValueError("P has shape %s, expected %s" % (P.shape, (self.nbf, self.nbf)))
        K = np.zeros_like(P)
        V = np.zeros_like(P)
        exc, nel = ctypes.c_double(0.0), ctypes.c_double(0.0)
        st = SnkStats()
        _check(lib().snk_ctx_build_kxc(self.handle, P.ctypes.data, K.ctypes.data, int(functional), V.ctypes.data,
                                       ctypes.byref(exc), ctypes.byref(nel), ctypes.byref(st) if stats else None),
               self.handle)
        return K, V, exc.value, nel.value, st.as_dict()

    def build_kxc_device(self, P_ptr: int, K_ptr: int, V_ptr: int, functional: int = SNK_XC_LDA):
        """Device-pointer sn-K and XC build on the context's stream (asynchronous)."""
        if not self.device_ptrs:
            raise ValueError("context was created for host pointers")
        _check(lib().snk_ctx_build_kxc(self.handle, ctypes.c_void_p(P_ptr), ctypes.c_void_p(K_ptr), int(functional),
                                       ctypes.c_void_p(V_ptr), None, None, None), self.handle)

    def vxc_device(self, P_ptr: int, V_ptr: int, functional: int = SNK_XC_LDA, scalars: bool = False):
        """Device-pointer XC potential on the context's stream; (E_xc, N_el) when scalars is set
        (then the call waits for them), else None (asynchronous)."""
        if not self.device_ptrs:
            raise ValueError("context was created for host pointers")
        exc, nel = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(lib().snk_vxc_build(self.handle, ctypes.c_void_p(P_ptr), int(functional), ctypes.c_void_p(V_ptr),
                                   ctypes.byref(exc) if scalars else None, ctypes.byref(nel) if scalars else None),
               self.handle)
        return (exc.value, nel.value) if scalars else None

    @property
    def ngroups(self) -> int:
        return int(lib().snk_ctx_ngroups(self.handle))

    def tiles(self):
        """Tiles: list of (group, b0, b1, functions B_t) with batches [b0, b1) in batch order."""
        n = lib().snk_ctx_ntiles(self.handle)
        gr, b0, b1, nB = (np.zeros(n, np.int32) for _ in range(4))
        _check(lib().snk_ctx_tile_info(self.handle, gr.ctypes.data, b0.ctypes.data, b1.ctypes.data, nB.ctypes.data),
               self.handle)
        out = []
        for k in range(n):
            fn = np.zeros(max(1, int(nB[k])), np.int32)
            _check(lib().snk_ctx_tile_functions(self.handle, k, fn.ctypes.data), self.handle)
            out.append((int(gr[k]), int(b0[k]), int(b1[k]), fn[:int(nB[k])].copy()))
        return out

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

    @property
    def nblock_pairs(self) -> int:
        return int(lib().snk_ctx_nblock_pairs(self.handle))

    @property
    def npair_index(self) -> int:
        return int(lib().snk_ctx_npair_index(self.handle))

    def collect_block_norms(self, P, feats_ptr: int, target_ptr: int, cap: int) -> int:
        """Features and log10 targets of every block (snk_collect_block_norms); returns the count."""
        if self.device_ptrs:
            pp = ctypes.c_void_p(int(P))
        else:
            P = np.ascontiguousarray(P, np.float64)
            pp = ctypes.c_void_p(P.ctypes.data)
        n = ctypes.c_int64(0)
        _check(lib().snk_collect_block_norms(self.handle, pp, ctypes.c_void_p(feats_ptr), ctypes.c_void_p(target_ptr),
                                             int(cap), ctypes.byref(n)), self.handle)
        return int(n.value)

    def block_data(self, P, features_ptr: int = 0, energy_ptr: int = 0) -> np.ndarray:
        """Training data of the learned screener (device outputs, see snk_ctx_block_data).

        P is a host array, or a device pointer for device-pointer contexts.  Returns the
        (A, B) shells of every listed pair."""
        if self.device_ptrs:
            pp = ctypes.c_void_p(int(P))
        else:
            P = np.ascontiguousarray(P, np.float64)
            pp = ctypes.c_void_p(P.ctypes.data)
        shells = np.zeros((self.nblock_pairs, 2), np.int32)
        _check(lib().snk_ctx_block_data(self.handle, pp, ctypes.c_void_p(features_ptr) if features_ptr else None,
                                        ctypes.c_void_p(energy_ptr) if energy_ptr else None,
                                        ctypes.c_void_p(shells.ctypes.data)), self.handle)
        return shells

    def debug_learned(self, P: np.ndarray):
        """(yraw, log2 est, thr) of the first batch group's learned screen, [batches][pair index]."""
        P = np.ascontiguousarray(P, np.float64)
        n = ctypes.c_int64(0)
        npi = self.npair_index
        nb = self.nbatches
        y = np.zeros(nb * npi, np.float32)
        e = np.zeros(nb * npi, np.float32)
        t = np.zeros(nb, np.int32)
        _check(lib().snk_ctx_debug_learned(self.handle, P.ctypes.data, y.ctypes.data, e.ctypes.data, t.ctypes.data,
                                           ctypes.byref(n)), self.handle)
        k = n.value
        return y[:k * npi].reshape(k, npi), e[:k * npi].reshape(k, npi), t[:k]

    def debug_kept(self, P: np.ndarray) -> np.ndarray:
        """(batch, A, B) of every shell pair the density screen keeps in the first batch group."""
        P = np.ascontiguousarray(P, np.float64)
        n = ctypes.c_int64(0)
        _check(lib().snk_ctx_debug_kept(self.handle, P.ctypes.data, None, 0, ctypes.byref(n)), self.handle)
        out = np.zeros((max(1, n.value), 3), np.int32)
        _check(lib().snk_ctx_debug_kept(self.handle, P.ctypes.data, out.ctypes.data, n.value, ctypes.byref(n)),
               self.handle)
        return out[:n.value]

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


def debug_gemm_f64(M, N, K, A_ptr, lda, B_ptr, ldb, bt, C_ptr, ldc, stream: int = 0, tile: int = 0):
    _check(lib().snk_debug_gemm_f64(M, N, K, ctypes.c_void_p(A_ptr), lda, ctypes.c_void_p(B_ptr), ldb, int(bt),
                                    ctypes.c_void_p(C_ptr), ldc, int(tile), ctypes.c_void_p(stream) if stream else None))


def debug_force_tile(tile: int = 0):
    _check(lib().snk_debug_force_tile(int(tile)))


def debug_frow_prefilter(on: bool = True):
    _check(lib().snk_debug_frow_prefilter(int(on)))


def debug_mfma_layout() -> np.ndarray:
    out = np.zeros(256)
    _check(lib().snk_debug_mfma_layout(out.ctypes.data))
    return out


def _f32(a, n=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if n is not None and a.size != n:
        raise ValueError("expected %d values, got %d" % (n, a.size))
    return a


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


class Mlp:
    """The learned block screener's network on one device (FP32 parameters in device memory).

    forward / loss_grad / adam_step take device pointers (e.g. ``tensor.data_ptr()``)."""

    def __init__(self, device: int = 0):
        self.nparams = int(lib().snk_mlp_nparams())
        h = ctypes.c_void_p()
        _check(lib().snk_mlp_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = int(device)

    @property
    def handle(self) -> int:
        return self._h.value or 0

    def set_params(self, flat) -> None:
        a = _f32(flat, self.nparams)
        _check(lib().snk_mlp_set_params(self._h, _fptr(a)))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.nparams, np.float32)
        _check(lib().snk_mlp_get_params(self._h, _fptr(a)))
        return a

    def set_normalisation(self, mean, std) -> None:
        m, s = _f32(mean, 16), _f32(std, 16)
        _check(lib().snk_mlp_set_normalisation(self._h, _fptr(m), _fptr(s)))

    def set_range(self, lo, hi, margin: float) -> None:
        a, b = _f32(lo, 16), _f32(hi, 16)
        _check(lib().snk_mlp_set_range(self._h, _fptr(a), _fptr(b), float(margin)))

    def forward(self, x_ptr: int, n: int, y_ptr: int, bf16: bool = False, stream: int = 0) -> None:
        _check(lib().snk_mlp_forward(self._h, ctypes.c_void_p(x_ptr), int(n), ctypes.c_void_p(y_ptr), int(bf16),
                                     ctypes.c_void_p(stream) if stream else None))

    def loss_grad(self, x_ptr: int, t_ptr: int, n: int, g_ptr: int, under: float = 10.0, stream: int = 0) -> None:
        _check(lib().snk_mlp_loss_grad(self._h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(t_ptr), int(n),
                                       float(under), ctypes.c_void_p(g_ptr),
                                       ctypes.c_void_p(stream) if stream else None))

    def loss_grad_noalloc(self, x_ptr: int, t_ptr: int, n: int, g_ptr: int, under: float = 10.0,
                          stream: int = 0) -> None:
        """loss_grad without any device allocation (at most 65536 samples per call)."""
        _check(lib().snk_mlp_loss_grad_noalloc(self._h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(t_ptr), int(n),
                                               float(under), ctypes.c_void_p(g_ptr),
                                               ctypes.c_void_p(stream) if stream else None))

    def backward(self, x_ptr: int, dy_ptr: int, n: int, g_ptr: int, stream: int = 0) -> None:
        _check(lib().snk_mlp_backward(self._h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(dy_ptr), int(n),
                                      ctypes.c_void_p(g_ptr), ctypes.c_void_p(stream) if stream else None))

    def adam_step(self, g_ptr: int, lr: float, t: int, stream: int = 0) -> None:
        _check(lib().snk_mlp_adam_step(self._h, ctypes.c_void_p(g_ptr), float(lr), int(t),
                                       ctypes.c_void_p(stream) if stream else None))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().snk_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_mfma_bf16(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A @ B through one bf16 matrix-core op: 16x16 @ 16x16, or 16x32 @ 32x16."""
    A = np.ascontiguousarray(A, np.float32)
    B = np.ascontiguousarray(B, np.float32)
    k32 = A.shape == (16, 32)
    if not ((A.shape == (16, 16) and B.shape == (16, 16)) or (k32 and B.shape == (32, 16))):
        raise ValueError("shapes must be 16x16 @ 16x16 or 16x32 @ 32x16")
    D = np.zeros((16, 16), np.float32)
    _check(lib().snk_debug_mfma_bf16(A.ctypes.data, B.ctypes.data, D.ctypes.data, int(k32)))
    return D


SCREENER_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "screener_weights.npz")


def load_screener(path: Optional[str] = None, device: int = 0) -> Mlp:
    """The trained block screener (parameters, feature normalisation, training range and
    margin as written by train_screener) on `device`."""
    d = np.load(path or SCREENER_WEIGHTS, allow_pickle=False)
    m = Mlp(device)
    m.set_params(d["params"])
    m.set_normalisation(d["mean"], d["std"])
    m.set_range(d["lo"], d["hi"], float(d["margin"]))
    m.info = str(d["info"]) if "info" in d else ""
    return m
