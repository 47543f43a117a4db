"""The C-ABI library loads, exports every entry point declared in include/*.h, and rejects
invalid arguments on the host before touching a device (no compute calls without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2303_14280_amd import snk, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = "".join(open(os.path.join(ROOT, "include", h)).read() for h in sorted(os.listdir(os.path.join(ROOT, "include")))
                  if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n.startswith("sn")))


def test_library_exports_every_declared_symbol():
    L = snk.lib()
    names = declared_functions()
    assert "sn_k_build" in names and "snk_ctx_create" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_version_and_status_strings():
    L = snk.lib()
    assert L.snk_version() == 1
    assert L.snk_status_string(0) == b"ok"
    assert L.snk_status_string(1) == b"invalid argument"
    assert L.snk_status_string(99) == b"unknown status"


def tiny():
    return synth.make_custom([1, 1], [[0, 0, 0], [0, 0, 1.4]], [[(0, [1.2, 0.3], [0.5, 0.5]), (1, [0.8], [1.0])],
                                                              [(0, [1.0], [1.0])]], grid=(10, 26), n_occ=1)


def _expect(status, fn):
    with pytest.raises(snk.SnkError) as ei:
        fn()
    assert ei.value.status == status, str(ei.value)


@pytest.mark.parametrize("field,value", [("shell_l", 3), ("shell_nprim", 0), ("shell_nprim", 9),
                                         ("exps", -1.0), ("exps", np.nan), ("coefs", np.inf)])
def test_invalid_basis_rejected(field, value):
    s = tiny()
    arr = getattr(s, field).copy()
    arr[0] = value
    bad = synth.System(**{**s.__dict__, field: arr})
    n = snk.nbf_of(bad)
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(bad, P=np.zeros((n, n))))


def test_invalid_grid_rejected():
    s = tiny()
    w = s.grid_w.copy()
    w[3] = -1.0
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(s.with_grid(s.grid_xyz, w, s.grid_atom)))
    xyz = s.grid_xyz.copy()
    xyz[2, 1] = np.nan
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(s.with_grid(xyz, s.grid_w, s.grid_atom)))


def test_invalid_options_rejected():
    s = tiny()
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(s, batch_points=300))
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(s, precision=7))
    _expect(snk.SNK_E_ARG, lambda: snk.sn_k_build(s, eps_basis=-1.0))


def test_shape_checked_in_binding():
    s = tiny()
    with pytest.raises(ValueError):
        snk.sn_k_build(s, P=np.zeros((2, 2)))


def test_null_pointers_rejected():
    L = snk.lib()
    h = ctypes.c_void_p()
    assert L.snk_ctx_create(None, None, None, None, ctypes.byref(h)) == snk.SNK_E_ARG
    assert L.snk_ctx_build(None, None, None, None) == snk.SNK_E_ARG
    assert L.snk_boys_device(None, 10, 2, None, None) == snk.SNK_E_ARG
    assert L.snk_boys_device(None, 10, 7, None, None) == snk.SNK_E_ARG
    assert L.snk_vxc_build(None, None, snk.SNK_XC_LDA, None, None, None) == snk.SNK_E_ARG
    assert L.snk_ctx_build_kxc(None, None, None, snk.SNK_XC_LDA, None, None, None, None) == snk.SNK_E_ARG


def test_dfj_validation_on_host():
    """snk_dfj_create rejects invalid orbital or auxiliary shells before touching a device."""
    import types
    s = tiny()
    aux = types.SimpleNamespace(shell_center=np.zeros((1, 3)), shell_l=np.zeros(1, np.int32),
                                shell_nprim=np.array([2], np.int32), shell_prim_off=np.zeros(1, np.int32),
                                exps=np.array([1.0, 0.5]), coefs=np.array([1.0, 1.0]))
    _expect(snk.SNK_E_ARG, lambda: snk.DfJ(s, aux))
    aux.shell_nprim[0] = 1
    aux.exps[0] = -1.0
    _expect(snk.SNK_E_ARG, lambda: snk.DfJ(s, aux))
    L = snk.lib()
    assert L.snk_dfj_naux(None) == 0
