"""Python binding of liblrdm (argument marshalling only).

Every step of the low-rank evolution runs in the HIP library; this module converts NumPy
matrices to the FP64 interleaved layout of include/lrdm.h, allocates the caller-owned device
buffers with torch, and passes pointers and the current HIP stream through ctypes.  It raises
if the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrdm.so")

C64, C128 = 0, 1
FLAG_PLAIN = 0x1
FLAG_OVERLAP = 0x2
STATUS = {0: "LRDM_OK", 1: "LRDM_E_ARG", 2: "LRDM_E_NOMEM", 3: "LRDM_E_HIP", 4: "LRDM_E_EIG",
          5: "LRDM_E_STATE", 6: "LRDM_E_UNSUPPORTED"}
SYMBOLS = ["lrdm_workspace_size", "lrdm_init", "lrdm_reset", "lrdm_destroy", "lrdm_apply_gate",
           "lrdm_apply_diagonal_weight", "lrdm_apply_kraus", "lrdm_compress", "lrdm_probabilities",
           "lrdm_expect_pauli", "lrdm_expect_z", "lrdm_sample", "lrdm_get_L", "lrdm_set_L",
           "lrdm_synchronize", "lrdm_timing_begin", "lrdm_timing_end", "lrdm_last_error",
           "lrdm_version", "lrdm_record_bytes", "lrdm_compress_record", "lrdm_checkpoint",
           "lrdm_restore", "lrdm_apply_pauli_sum", "lrdm_pauli_overlap", "lrdm_compress_adjoint",
           "lrdm_fdm_state_bytes", "lrdm_fdm_init", "lrdm_fdm_reset", "lrdm_fdm_destroy",
           "lrdm_fdm_apply_gate", "lrdm_fdm_apply_kraus", "lrdm_fdm_apply_diagonal_weight", "lrdm_fdm_probabilities",
           "lrdm_fdm_synchronize", "lrdm_fdm_last_error", "lrdm_batch_create", "lrdm_batch_begin",
           "lrdm_batch_end", "lrdm_batch_instantiate", "lrdm_batch_launch", "lrdm_batch_info",
           "lrdm_batch_times", "lrdm_batch_destroy", "lrdm_layout", "lrdm_run", "lrdm_energy_grad_bytes",
           "lrdm_energy_grad", "lrdm_batch_run", "lrdm_program_validate", "lrdm_expect_z_noalloc",
           "lrdm_set_tuning", "lrdm_get_tuning",
           "lrdm_apply_kraus2", "lrdm_set_sparse", "lrdm_to_full", "lrdm_run_switching"]

OP_GATE, OP_ROTATION, OP_WEIGHT, OP_KRAUS, OP_COMPRESS, OP_LAYER, OP_KRAUS2 = range(7)
_AXIS = {"X": 1, "Y": 2, "Z": 3}


class LrdmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CompressInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int), ("n_eig", ctypes.c_int), ("discarded", ctypes.c_double),
                ("discarded_total", ctypes.c_double), ("trace_before", ctypes.c_double),
                ("boundary_gap", ctypes.c_double), ("lambda_max", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tuning(ctypes.Structure):
    """lrdm_tuning of include/lrdm.h (0 = default)."""
    _fields_ = [("gram_blocks", ctypes.c_int), ("gram4_blocks", ctypes.c_int), ("gate_local_max", ctypes.c_int),
                ("aux_cus", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class COp(ctypes.Structure):
    """lrdm_op of include/lrdm.h."""
    _fields_ = [("kind", ctypes.c_int), ("k", ctypes.c_int), ("q0", ctypes.c_int), ("q1", ctypes.c_int),
                ("axis", ctypes.c_int), ("param", ctypes.c_int), ("r", ctypes.c_int), ("tie", ctypes.c_int),
                ("renorm", ctypes.c_int), ("eps", ctypes.c_double), ("off", ctypes.c_int64)]


class CProgram(ctypes.Structure):
    """lrdm_program of include/lrdm.h."""
    _fields_ = [("n_ops", ctypes.c_int), ("ops", ctypes.POINTER(COp)), ("coef", ctypes.POINTER(ctypes.c_double)),
                ("n_coef", ctypes.c_int64)]


class FlatProgram:
    """A workloads.circuits.Program as the flat operation array of the C ABI (lrdm_program).
    Parametrised gates (param = (index, axis)) become rotations whose matrix is the gate's own
    (no params array is passed), so the C side applies exactly the Python program's matrices and
    knows each rotation's generator for the gradient."""

    def __init__(self, program):
        from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

        ops, coef = [], []

        def put(a):
            off = len(coef)
            coef.extend(_cplx(a).ravel().tolist())
            return off

        self.n_params = 0
        for op in program.ops:
            o = COp()
            if isinstance(op, Gate):
                if getattr(op, "param", None) is not None:
                    o.kind, o.k, o.q0 = OP_ROTATION, 1, int(op.qubits[0])
                    o.param, o.axis = int(op.param[0]), _AXIS[op.param[1]]
                    self.n_params = max(self.n_params, o.param + 1)
                else:
                    o.kind, o.k = OP_GATE, len(op.qubits)
                    o.q0 = int(op.qubits[0])
                    o.q1 = int(op.qubits[1]) if len(op.qubits) > 1 else -1
                o.off = put(op.u)
            elif isinstance(op, DiagWeight):
                o.kind, o.off = OP_WEIGHT, put(op.phase)
            elif isinstance(op, Kraus):
                ks = np.asarray(op.ops, dtype=np.complex128)
                o.kind, o.k, o.q0, o.off = OP_KRAUS, ks.shape[0], int(op.qubit), put(ks)
                if op.qubit2 >= 0:
                    o.kind, o.q1 = OP_KRAUS2, int(op.qubit2)
            elif isinstance(op, Compress):
                o.kind, o.r, o.eps, o.tie, o.renorm = OP_COMPRESS, int(op.r), float(op.eps), int(op.tie), int(op.renorm)
            elif isinstance(op, LayerEnd):
                o.kind = OP_LAYER
            else:
                raise TypeError(f"unknown op {op!r}")
            ops.append(o)
        self.ops = (COp * max(len(ops), 1))(*ops)
        self.coef = np.ascontiguousarray(coef, dtype=np.float64) if coef else np.zeros(1)
        self.c = CProgram(len(ops), self.ops, _dptr(self.coef), len(coef))
        self.n_layers = sum(o.kind == OP_LAYER for o in ops) + (1 if ops and ops[-1].kind != OP_LAYER else 0)

    @property
    def ref(self):
        return ctypes.byref(self.c)


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblrdm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2009_06657_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded (loaded before
    # torch, it would start a second runtime in the process, which finds no device for the
    # handle's own streams)
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    P, I, D, U, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lrdm_workspace_size": [I, I, I, I, U, ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
        "lrdm_init": [ctypes.POINTER(P), I, I, I, I, U, P, SZ, P, SZ, P],
        "lrdm_reset": [P],
        "lrdm_destroy": [P],
        "lrdm_apply_gate": [P, I, ctypes.POINTER(I), dp],
        "lrdm_apply_diagonal_weight": [P, dp],
        "lrdm_apply_kraus": [P, I, I, dp],
        "lrdm_compress": [P, I, D, I, I, ctypes.POINTER(CompressInfo)],
        "lrdm_probabilities": [P, P],
        "lrdm_expect_pauli": [P, I, P, P, P, I, dp],
        "lrdm_expect_z": [P, dp, dp, dp],
        "lrdm_sample": [P, I, dp, ctypes.POINTER(ctypes.c_uint64)],
        "lrdm_get_L": [P, P, I, ctypes.POINTER(I)],
        "lrdm_set_L": [P, P, I, I],
        "lrdm_synchronize": [P],
        "lrdm_timing_begin": [P, I],
        "lrdm_timing_end": [P, ctypes.POINTER(I), dp, dp],
        "lrdm_set_tuning": [P, P],
        "lrdm_get_tuning": [P, P],
        "lrdm_record_bytes": [P, ctypes.POINTER(SZ)],
        "lrdm_compress_record": [P, I, D, I, I, P, ctypes.POINTER(CompressInfo)],
        "lrdm_checkpoint": [P, P, ctypes.POINTER(I)],
        "lrdm_restore": [P, P, I],
        "lrdm_apply_pauli_sum": [P, P, I, P, P, P],
        "lrdm_pauli_overlap": [P, P, I, P, P, dp],
        "lrdm_compress_adjoint": [P, P, P, I, I, dp],
        "lrdm_fdm_state_bytes": [I, ctypes.POINTER(SZ)],
        "lrdm_fdm_init": [ctypes.POINTER(P), I, P, SZ, P],
        "lrdm_fdm_reset": [P],
        "lrdm_fdm_destroy": [P],
        "lrdm_fdm_apply_gate": [P, I, ctypes.POINTER(I), dp],
        "lrdm_fdm_apply_kraus": [P, I, I, dp],
        "lrdm_fdm_apply_diagonal_weight": [P, dp],
        "lrdm_fdm_probabilities": [P, P],
        "lrdm_fdm_synchronize": [P],
        "lrdm_batch_create": [ctypes.POINTER(P), I, ctypes.POINTER(P), P],
        "lrdm_batch_begin": [P],
        "lrdm_batch_end": [P, ctypes.POINTER(SZ)],
        "lrdm_batch_instantiate": [P, P, SZ],
        "lrdm_batch_launch": [P],
        "lrdm_batch_info": [P, ctypes.POINTER(I), ctypes.POINTER(I)],
        "lrdm_batch_times": [P, dp, dp],
        "lrdm_batch_destroy": [P],
        "lrdm_layout": [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(SZ)],
        "lrdm_run": [P, ctypes.POINTER(CProgram), dp, I, P, SZ, ctypes.POINTER(I)],
        "lrdm_energy_grad_bytes": [P, ctypes.POINTER(CProgram), ctypes.POINTER(SZ), ctypes.POINTER(SZ)],
        "lrdm_energy_grad": [P, P, ctypes.POINTER(CProgram), dp, I, I, P, P, P, dp, dp, P, SZ, ctypes.POINTER(I)],
        "lrdm_batch_run": [P, ctypes.POINTER(ctypes.POINTER(CProgram)), P, P, P, SZ, ctypes.POINTER(SZ), dp, dp],
        "lrdm_program_validate": [ctypes.POINTER(CProgram), I, dp, I],
        "lrdm_expect_z_noalloc": [P, I, I, I, I, P, dp, dp, dp],
        "lrdm_apply_kraus2": [P, I, I, I, dp],
        "lrdm_set_sparse": [P, I, P, dp],
        "lrdm_to_full": [P, P],
        "lrdm_run_switching": [P, P, ctypes.POINTER(CProgram), dp, I, ctypes.POINTER(I)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lrdm_last_error.argtypes = [P]
    lib.lrdm_last_error.restype = ctypes.c_char_p
    lib.lrdm_fdm_last_error.argtypes = [P]
    lib.lrdm_fdm_last_error.restype = ctypes.c_char_p
    lib.lrdm_version.argtypes = []
    lib.lrdm_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(st: int, handle=None):
    if st != 0:
        lib = load_library()
        msg = lib.lrdm_last_error(handle).decode()
        raise LrdmError(st, msg)


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def expect_z_noalloc(L_dev_ptr: int, n: int, ld: int, ncols: int, dtype: int = C64, stream=None):
    """lrdm_expect_z_noalloc on a device factor (pointer, state layout): (z, zz, trace)."""
    lib = load_library()
    z, zz, tr = np.zeros(n), np.zeros(max(n - 1, 1)), np.zeros(1)
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else None
    _check(lib.lrdm_expect_z_noalloc(ctypes.c_void_p(L_dev_ptr), n, ld, ncols, dtype, s, _dptr(z), _dptr(zz), _dptr(tr)))
    return z, zz[: n - 1], float(tr[0])


def workspace_size(n: int, r_max: int, dtype: int = C64, m_max: int = 4, flags: int = 0):
    lib = load_library()
    s, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.lrdm_workspace_size(n, r_max, dtype, m_max, flags, ctypes.byref(s), ctypes.byref(w)))
    return s.value, w.value


class LowRankDM:
    """A handle over caller-owned device memory; method names follow the C ABI."""

    def __init__(self, n: int, r_max: int, dtype: int = C64, m_max: int = 4, flags: int = 0,
                 device: str = "cuda:0", stream=None, tuning=None):
        """tuning: None (the library's launch shapes), "table" (the autotuner's entry for this
        shape, if any: paper_2009_06657_amd/tuning_table.json) or a dict of lrdm_tuning fields."""
        import torch

        self.lib = load_library()
        self.n, self.r_max, self.dtype, self.m_max, self.flags = n, r_max, dtype, m_max, flags
        sb, wb = workspace_size(n, r_max, dtype, m_max, flags)
        self.device = torch.device(device)
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = ctypes.c_void_p()
        _check(self.lib.lrdm_init(ctypes.byref(self.h), n, r_max, dtype, m_max, flags,
                                  self.state.data_ptr(), sb, self.work.data_ptr(), wb,
                                  ctypes.c_void_p(self.stream.cuda_stream)))
        ld, r_pad = ctypes.c_int(), ctypes.c_int()
        _check(self.lib.lrdm_layout(self.h, None, ctypes.byref(ld), ctypes.byref(r_pad), None), self.h)
        self.r_pad = r_pad.value
        self.ld = ld.value
        self.tuning = None
        if tuning == "table":
            from . import autotune

            self.tuning = autotune.apply(self)
        elif tuning:
            self.set_tuning(**tuning)
            self.tuning = dict(tuning)

    # -------------------------------------------------------------- lifetime
    def close(self):
        if self.h:
            self.lib.lrdm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        _check(self.lib.lrdm_reset(self.h), self.h)

    def synchronize(self):
        _check(self.lib.lrdm_synchronize(self.h), self.h)

    # -------------------------------------------------------------- evolution
    def apply_gate(self, qubits: Sequence[int], u):
        q = (ctypes.c_int * len(qubits))(*[int(x) for x in qubits])
        m = _cplx(u)
        _check(self.lib.lrdm_apply_gate(self.h, len(qubits), q, _dptr(m)), self.h)

    def apply_diagonal_weight(self, phase):
        m = _cplx(phase)
        _check(self.lib.lrdm_apply_diagonal_weight(self.h, _dptr(m)), self.h)

    def apply_kraus(self, qubit: int, ops, qubit2: int = -1):
        """A one-qubit channel, or with qubit2 >= 0 a two-qubit channel (4 x 4 operators, local
        index b(qubit) + 2 b(qubit2); plain form)."""
        ops = np.asarray(ops, dtype=np.complex128)
        m = _cplx(ops)
        if qubit2 >= 0:
            _check(self.lib.lrdm_apply_kraus2(self.h, int(qubit), int(qubit2), ops.shape[0], _dptr(m)), self.h)
        else:
            _check(self.lib.lrdm_apply_kraus(self.h, int(qubit), ops.shape[0], _dptr(m)), self.h)

    def set_sparse(self, idx, amp):
        """L = sum_i amp[i] |idx[i]> (a sparse superposition initial state)."""
        ix = np.ascontiguousarray(idx, dtype=np.uint64)
        a = _cplx(np.asarray(amp, dtype=np.complex128))
        _check(self.lib.lrdm_set_sparse(self.h, ix.shape[0], ix.ctypes.data, _dptr(a)), self.h)

    def to_full(self, fdm: "FullRankDM"):
        """fdm's rho <- L L^H."""
        _check(self.lib.lrdm_to_full(self.h, fdm.h), self.h)

    def run_switching(self, program, fdm: "Optional[FullRankDM]") -> int:
        """lrdm_run_switching: the program with the switch to full density matrix evolution once
        the intermediate rank reaches 2^n; returns the index of the switching channel or -1."""
        fp = program if isinstance(program, FlatProgram) else FlatProgram(program)
        at = ctypes.c_int(-2)
        _check(self.lib.lrdm_run_switching(self.h, fdm.h if fdm is not None else None, fp.ref, None, 0,
                                           ctypes.byref(at)), self.h)
        return at.value

    def compress(self, r: int, eps: float = 0.0, tie: int = 0, renorm: int = 1,
                 info: bool = False) -> Optional[dict]:
        ci = CompressInfo()
        _check(self.lib.lrdm_compress(self.h, int(r), float(eps), int(tie), int(renorm),
                                      ctypes.byref(ci) if info else None), self.h)
        return ci.as_dict() if info else None

    def run(self, program, ckpt=None) -> Optional[list]:
        """lrdm_run: the whole program (a workloads.circuits.Program or a FlatProgram) from the
        current state; with ckpt (a device tensor of layers x state bytes rounded up to 256) the
        state at the start of every layer is kept there and the column bounds are returned."""
        fp = program if isinstance(program, FlatProgram) else FlatProgram(program)
        ranks = (ctypes.c_int * max(fp.n_layers, 1))()
        _check(self.lib.lrdm_run(self.h, fp.ref, None, 0,
                                 ctypes.c_void_p(ckpt.data_ptr()) if ckpt is not None else None,
                                 ckpt.numel() * ckpt.element_size() if ckpt is not None else 0,
                                 ranks if ckpt is not None else None), self.h)
        return list(ranks)[: fp.n_layers] if ckpt is not None else None

    # -------------------------------------------------------------- outputs
    def probabilities(self, out=None):
        import torch

        if out is None:
            out = torch.empty(2 ** self.n, dtype=torch.float64, device=self.device)
        _check(self.lib.lrdm_probabilities(self.h, ctypes.c_void_p(out.data_ptr())), self.h)
        return out

    def expect_z(self):
        z = np.zeros(self.n)
        zz = np.zeros(max(self.n - 1, 1))
        tr = np.zeros(1)
        _check(self.lib.lrdm_expect_z(self.h, _dptr(z), _dptr(zz), _dptr(tr)), self.h)
        return z, zz[: self.n - 1], float(tr[0])

    def expect_pauli(self, xmask, zmask, coeff=None, summed: bool = False):
        xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        nt = xm.shape[0]
        out = np.zeros(1 if summed else nt)
        cf = np.ascontiguousarray(coeff, dtype=np.float64) if coeff is not None else None
        _check(self.lib.lrdm_expect_pauli(self.h, nt, xm.ctypes.data, zm.ctypes.data,
                                          cf.ctypes.data if cf is not None else None,
                                          1 if summed else 0, _dptr(out)), self.h)
        return float(out[0]) if summed else out

    def sample(self, uniforms) -> np.ndarray:
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        out = np.zeros(u.shape[0], dtype=np.uint64)
        _check(self.lib.lrdm_sample(self.h, u.shape[0], _dptr(u),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))), self.h)
        return out

    def get_L(self) -> np.ndarray:
        """The factor as a (2^n, ld) complex128 array (converted from the bulk precision)."""
        dt = np.complex64 if self.dtype == C64 else np.complex128
        buf = np.zeros((2 ** self.n, self.ld), dtype=dt)
        rk = ctypes.c_int()
        _check(self.lib.lrdm_get_L(self.h, buf.ctypes.data, 1, ctypes.byref(rk)), self.h)
        return buf.astype(np.complex128)

    def set_L(self, L: np.ndarray):
        dt = np.complex64 if self.dtype == C64 else np.complex128
        a = np.ascontiguousarray(np.asarray(L), dtype=dt)
        _check(self.lib.lrdm_set_L(self.h, a.ctypes.data, 1, a.shape[1]), self.h)

    # -------------------------------------------------------------- reverse sweep
    def record_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(self.lib.lrdm_record_bytes(self.h, ctypes.byref(b)), self.h)
        return b.value

    def compress_record(self, r: int, rec, eps: float = 0.0, tie: int = 0, renorm: int = 1):
        """lrdm_compress that also fills `rec` (a device tensor of record_bytes() bytes)."""
        _check(self.lib.lrdm_compress_record(self.h, int(r), float(eps), int(tie), int(renorm),
                                             ctypes.c_void_p(rec.data_ptr()), None), self.h)

    def checkpoint(self, dst) -> int:
        """Copy the state buffer into `dst` (a device tensor of state.numel() bytes); returns the
        column bound to pass back to restore()."""
        rk = ctypes.c_int()
        _check(self.lib.lrdm_checkpoint(self.h, ctypes.c_void_p(dst.data_ptr()), ctypes.byref(rk)), self.h)
        return rk.value

    def restore(self, src, rank: int):
        _check(self.lib.lrdm_restore(self.h, ctypes.c_void_p(src.data_ptr()), int(rank)), self.h)

    def apply_pauli_sum_from(self, src: "LowRankDM", xmask, zmask, coeff):
        """This handle's factor <- H src's factor, H = sum_t coeff[t] P_t."""
        xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        cf = np.ascontiguousarray(coeff, dtype=np.float64)
        _check(self.lib.lrdm_apply_pauli_sum(self.h, src.h, xm.shape[0], xm.ctypes.data, zm.ctypes.data,
                                             cf.ctypes.data), self.h)

    def pauli_overlap(self, ket: "LowRankDM", xmask, zmask) -> np.ndarray:
        """Tr(self^H P_t ket) for every term, complex."""
        xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        out = np.zeros(2 * xm.shape[0])
        _check(self.lib.lrdm_pauli_overlap(self.h, ket.h, xm.shape[0], xm.ctypes.data, zm.ctypes.data,
                                           _dptr(out)), ket.h)
        return out[0::2] + 1j * out[1::2]

    def compress_adjoint(self, x_ckpt, rec, qubit: int, ops):
        """Reverse of one channel + compression on this (adjoint) handle."""
        ops = np.asarray(ops, dtype=np.complex128)
        m = _cplx(ops)
        _check(self.lib.lrdm_compress_adjoint(self.h, ctypes.c_void_p(x_ckpt.data_ptr()),
                                              ctypes.c_void_p(rec.data_ptr()), int(qubit), ops.shape[0],
                                              _dptr(m)), self.h)

    # -------------------------------------------------------------- timing
    def timing_begin(self, kernel_class: int):
        _check(self.lib.lrdm_timing_begin(self.h, int(kernel_class)), self.h)

    def set_tuning(self, **kw):
        """lrdm_set_tuning: fields of lrdm_tuning by name (unnamed fields keep 0 = default)."""
        t = Tuning(**{k: int(v) for k, v in kw.items()})
        _check(self.lib.lrdm_set_tuning(self.h, ctypes.byref(t)), self.h)

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(self.lib.lrdm_get_tuning(self.h, ctypes.byref(t)), self.h)
        return t.as_dict()

    def timing_end(self):
        n = ctypes.c_int()
        mean, tot = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.lrdm_timing_end(self.h, ctypes.byref(n), ctypes.byref(mean), ctypes.byref(tot)),
               self.h)
        return n.value, mean.value, tot.value


class FullRankDM:
    """The full-rank density-matrix comparator (complex64 rho of 8 * 4^n bytes on the device)."""

    def __init__(self, n: int, device: str = "cuda:0", stream=None):
        import torch

        self.lib = load_library()
        self.n = n
        b = ctypes.c_size_t()
        _check(self.lib.lrdm_fdm_state_bytes(n, ctypes.byref(b)))
        self.device = torch.device(device)
        self.state = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = ctypes.c_void_p()
        _check(self.lib.lrdm_fdm_init(ctypes.byref(self.h), n, self.state.data_ptr(), b.value,
                                      ctypes.c_void_p(self.stream.cuda_stream)))

    def _chk(self, st):
        if st != 0:
            raise LrdmError(st, self.lib.lrdm_fdm_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.lib.lrdm_fdm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self):
        self._chk(self.lib.lrdm_fdm_reset(self.h))

    def apply_gate(self, qubits: Sequence[int], u):
        q = (ctypes.c_int * len(qubits))(*[int(x) for x in qubits])
        m = _cplx(u)
        self._chk(self.lib.lrdm_fdm_apply_gate(self.h, len(qubits), q, _dptr(m)))

    def apply_kraus(self, qubit: int, ops):
        ops = np.asarray(ops, dtype=np.complex128)
        m = _cplx(ops)
        self._chk(self.lib.lrdm_fdm_apply_kraus(self.h, int(qubit), ops.shape[0], _dptr(m)))

    def apply_diagonal_weight(self, phase):
        m = _cplx(phase)
        self._chk(self.lib.lrdm_fdm_apply_diagonal_weight(self.h, _dptr(m)))

    def probabilities(self, out=None):
        import torch

        if out is None:
            out = torch.empty(2 ** self.n, dtype=torch.float64, device=self.device)
        self._chk(self.lib.lrdm_fdm_probabilities(self.h, ctypes.c_void_p(out.data_ptr())))
        return out

    def synchronize(self):
        self._chk(self.lib.lrdm_fdm_synchronize(self.h))

    def rho(self) -> np.ndarray:
        """rho as a (2^n, 2^n) complex128 array (test helper; copies 8 * 4^n bytes)."""
        self.synchronize()
        a = self.state.view(dtype=__import__("torch").complex64).cpu().numpy()
        return a.reshape(2 ** self.n, 2 ** self.n).astype(np.complex128)


class Batch:
    """Many complex64 handles recorded once and replayed as one captured hipGraph (lockstep
    batched launches; see lrdm_batch_* in include/lrdm.h).

        b = Batch(handles)
        with b.recording():
            for dm, prog in zip(handles, programs):
                dm.reset(); run_program(dm, prog)
        b.launch(); done_ms, total_ms = b.times()
    """

    def __init__(self, handles: Sequence[LowRankDM], stream=None):
        import torch

        self.lib = load_library()
        self.handles = list(handles)
        dev = self.handles[0].device
        self.device = dev
        self.stream = stream   # None: the library captures and replays on a stream of its own
        arr = (ctypes.c_void_p * len(self.handles))(*[h.h.value for h in self.handles])
        self.b = ctypes.c_void_p()
        _check(self.lib.lrdm_batch_create(ctypes.byref(self.b), len(self.handles), arr,
                                          ctypes.c_void_p(stream.cuda_stream) if stream is not None else None))
        self.plan = None

    def begin(self):
        _check(self.lib.lrdm_batch_begin(self.b))

    def end(self):
        import torch

        nbytes = ctypes.c_size_t()
        _check(self.lib.lrdm_batch_end(self.b, ctypes.byref(nbytes)))
        self.plan = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        _check(self.lib.lrdm_batch_instantiate(self.b, ctypes.c_void_p(self.plan.data_ptr()), nbytes.value))

    def recording(self):
        import contextlib

        @contextlib.contextmanager
        def ctx():
            self.begin()
            try:
                yield self
            finally:
                self.end()
        return ctx()

    def run(self, programs):
        """lrdm_batch_run: reset every handle, record its program (one per handle, in order),
        capture the graph and replay it once; returns (done_ms, total_ms)."""
        import torch

        flats = [p if isinstance(p, FlatProgram) else FlatProgram(p) for p in programs]
        arr = (ctypes.POINTER(CProgram) * len(flats))(*[ctypes.pointer(f.c) for f in flats])
        need = ctypes.c_size_t()
        done = np.zeros(len(self.handles))
        tot = np.zeros(1)
        plan = self.plan
        st = self.lib.lrdm_batch_run(self.b, arr, None, None,
                                     ctypes.c_void_p(plan.data_ptr()) if plan is not None else None,
                                     plan.numel() if plan is not None else 0, ctypes.byref(need), _dptr(done), _dptr(tot))
        if st == 2:   # LRDM_E_NOMEM: the plan buffer is missing or too small
            self.plan = torch.empty(need.value, dtype=torch.uint8, device=self.device)
            st = self.lib.lrdm_batch_run(self.b, arr, None, None, ctypes.c_void_p(self.plan.data_ptr()),
                                         need.value, ctypes.byref(need), _dptr(done), _dptr(tot))
        _check(st)
        return done, float(tot[0])

    def launch(self):
        _check(self.lib.lrdm_batch_launch(self.b))

    def info(self):
        s, l = ctypes.c_int(), ctypes.c_int()
        _check(self.lib.lrdm_batch_info(self.b, ctypes.byref(s), ctypes.byref(l)))
        return s.value, l.value

    def times(self):
        done = np.zeros(len(self.handles))
        tot = np.zeros(1)
        _check(self.lib.lrdm_batch_times(self.b, _dptr(done), _dptr(tot)))
        return done, float(tot[0])

    def close(self):
        if self.b:
            self.lib.lrdm_batch_destroy(self.b)
            self.b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_program_fdm(fdm: FullRankDM, program):
    """Gates, Hamming-weight phases and channels of a Program on the full-rank comparator
    (compressions do not apply there)."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    for op in program.ops:
        if isinstance(op, Gate):
            fdm.apply_gate(op.qubits, op.u)
        elif isinstance(op, Kraus):
            fdm.apply_kraus(op.qubit, op.ops)
        elif isinstance(op, DiagWeight):
            fdm.apply_diagonal_weight(op.phase)
        elif isinstance(op, (Compress, LayerEnd)):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")


def run_program(dm: LowRankDM, program, on_layer=None):
    """Issue every op of a workloads.circuits.Program through the C ABI, in order."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    if getattr(program, "init", None) is not None:
        dm.set_sparse(*program.init)
    for op in program.ops:
        if isinstance(op, Gate):
            dm.apply_gate(op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            dm.apply_diagonal_weight(op.phase)
        elif isinstance(op, Kraus):
            dm.apply_kraus(op.qubit, op.ops, op.qubit2)
        elif isinstance(op, Compress):
            dm.compress(op.r, op.eps, op.tie, op.renorm)
        elif isinstance(op, LayerEnd):
            if on_layer is not None:
                on_layer(op.index)
        else:
            raise TypeError(f"unknown op {op!r}")
