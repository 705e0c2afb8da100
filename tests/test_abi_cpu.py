"""C-ABI checks that need no GPU: the library loads, exports every symbol the header declares,
and rejects invalid sizes and arguments before touching the device."""
import ctypes
import os
import re

import pytest

import paper_2009_06657_amd as lr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "lrdm.h")).read()
    return sorted(set(re.findall(r"\b(lrdm_[A-Za-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lr.load_library()
    syms = header_symbols()
    assert len(syms) >= 19
    for s in syms:
        assert hasattr(lib, s), s
    assert set(lr.lrdm.SYMBOLS) == set(syms)
    assert b"gfx950" in lib.lrdm_version()


def test_workspace_sizes():
    s, w = lr.workspace_size(20, 64, lr.C64, 2)
    assert s == 2 ** 20 * 64 * 8
    assert w > 0
    s, _ = lr.workspace_size(6, 13, lr.C128, 4)
    assert s == 64 * 16 * 16                     # r_pad = 16, complex128
    s, _ = lr.workspace_size(8, 8, lr.C64, 4, lr.FLAG_PLAIN)
    assert s == 256 * 32 * 8                     # plain form: ld = m_pad * r_pad


@pytest.mark.parametrize("args,status", [
    ((0, 8, 0, 2, 0), 1), ((31, 8, 0, 2, 0), 1), ((10, 0, 0, 2, 0), 1), ((10, 65, 0, 2, 0), 1),
    ((10, 8, 0, 0, 0), 1), ((10, 8, 0, 5, 0), 1), ((10, 8, 7, 2, 0), 1),
    ((10, 64, 0, 4, 0), 6),      # m * r_pad = 256 > 128
    ((10, 64, 1, 2, 0), 6),      # complex128 limited to r_pad <= 32
])
def test_workspace_size_rejects(args, status):
    lib = lr.load_library()
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    st = lib.lrdm_workspace_size(*args, ctypes.byref(s), ctypes.byref(w))
    assert st == status
    assert lib.lrdm_last_error(None)


def test_init_validates_before_device_work():
    lib = lr.load_library()
    h = ctypes.c_void_p()
    # null buffers
    assert lib.lrdm_init(ctypes.byref(h), 8, 8, 0, 2, 0, None, 0, None, 0, None) == 1
    # buffers too small (fake, never dereferenced: the size check comes first)
    assert lib.lrdm_init(ctypes.byref(h), 8, 8, 0, 2, 0, 256, 16, 512, 16, None) == 2
    # null handle everywhere
    assert lib.lrdm_compress(None, 1, 0.0, 0, 1, None) == 1
    assert lib.lrdm_apply_gate(None, 1, None, None) == 1
    assert lib.lrdm_destroy(None) == 1
    assert b"null" in lib.lrdm_last_error(None)


def test_python_binding_fails_loudly_without_library(tmp_path):
    import importlib

    mod = importlib.import_module("paper_2009_06657_amd.lrdm")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(RuntimeError):
            mod.load_library(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved
