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
    return sorted(set(re.findall(r"\b(lrdm_[A-Za-z_0-9]+)\s*\(", text)))


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


# ------------------------------------------------------------------- program-level calls
def _flat(ops, n=4):
    from workloads import circuits as C

    return lr.lrdm.FlatProgram(C.Program(n, ops, 4, "c64", 4))


def _validate(fp, n=4):
    lib = lr.load_library()
    return lib.lrdm_program_validate(fp.ref, n, None, 0)


def test_program_validation_accepts_a_workload():
    from workloads import circuits as C

    for prog in (C.cfg1_program(layers=2), C.cfg4_program(C.cfg4_angles(n=5, layers=2), n=5),
                 C.cfg2_program(n=6, iterations=1)):
        fp = lr.lrdm.FlatProgram(prog)
        assert _validate(fp, prog.n) == 0, lr.load_library().lrdm_last_error(None)
    fp = lr.lrdm.FlatProgram(C.cfg4_program(C.cfg4_angles(n=5, layers=2), n=5))
    assert fp.n_params == 2 * 5 * 2 and fp.n_layers == 2


def test_program_validation_rejects():
    import numpy as np

    from workloads import circuits as C

    lib = lr.load_library()
    bad = {
        "qubit out of range": [C.Gate((4,), C.H)],
        "repeated": [C.Gate((1, 1), C.CZ, True)],
        "not unitary": [C.Gate((0,), np.array([[1, 1], [0, 1]]))],
        "followed by a compression": [C.Kraus(0, C.depolarizing(0.1))],
        "not complete": [C.Kraus(0, np.stack([C.I2, C.X])), C.Compress(4)],
        "unit modulus": [C.DiagWeight(np.full(5, 2.0))],
    }
    for why, ops in bad.items():
        assert _validate(_flat(ops)) == 1, why
        assert lib.lrdm_last_error(None).decode().startswith("op "), why
    # rotation axis out of range and a parameter index beyond n_params
    fp = _flat([C.Gate((0,), C.rx(0.3), False, "rx", (0, "X"))])
    fp.ops[0].axis = 4
    assert _validate(fp) == 1
    fp.ops[0].axis = 1
    theta = (ctypes.c_double * 1)(0.3)
    fp.ops[0].param = 3
    assert lib.lrdm_program_validate(fp.ref, 4, theta, 1) == 1
    # coefficients beyond the array
    fp = _flat([C.Gate((0,), C.H)])
    fp.ops[0].off = 4
    assert _validate(fp) == 1
    # null program, n out of range, null handles for the program calls
    assert lib.lrdm_program_validate(None, 4, None, 0) == 1
    assert lib.lrdm_program_validate(_flat([C.Gate((0,), C.H)]).ref, 0, None, 0) == 1
    fp = _flat([C.Gate((0,), C.H)])
    assert lib.lrdm_run(None, fp.ref, None, 0, None, 0, None) == 1
    kb, mb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lrdm_energy_grad_bytes(None, fp.ref, ctypes.byref(kb), ctypes.byref(mb)) == 1
    need = ctypes.c_size_t()
    assert lib.lrdm_batch_run(None, None, None, None, None, 0, ctypes.byref(need), None, None) == 1
    assert lib.lrdm_layout(None, None, None, None, None) == 1
