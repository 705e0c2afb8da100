"""Exact full-rank density-matrix evolution (FDM) and the noiseless statevector (test
infrastructure only).

FDM follows Eq. "full rank evolution" (Sec. II.A): rho <- sum_a E_a rho E_a^H for a channel and
rho <- U rho U^H for a gate.  The statevector run drops the channels; it gives rho_noiseless in
the distortion measure of Sec. III.
"""
from __future__ import annotations

import numpy as np

from .linalg import apply_gate, popcount


def _sandwich(rho: np.ndarray, n: int, qubits, U: np.ndarray) -> np.ndarray:
    """U rho U^H for a k-qubit U embedded on `qubits`."""
    a = apply_gate(rho, n, qubits, U)                 # U rho
    b = apply_gate(a.conj().T, n, qubits, U)          # U (U rho)^H = U rho^H U^H
    return b.conj().T                                 # (U rho^H U^H)^H = U rho U^H


def _initial(program) -> np.ndarray:
    """|0...0>, or the program's sparse superposition sum_i a_i |x_i>."""
    psi = np.zeros(2 ** program.n, dtype=np.complex128)
    if program.init is None:
        psi[0] = 1.0
    else:
        idx, amp = program.init
        psi[np.asarray(idx, dtype=np.int64)] = np.asarray(amp, dtype=np.complex128)
    return psi


def fdm_gate(rho, n, qubits, U):
    return _sandwich(rho, n, qubits, U)


def fdm_channel(rho, n, qubit, ops, qubit2: int = -1):
    qs = (qubit,) if qubit2 < 0 else (qubit, qubit2)
    return sum(_sandwich(rho, n, qs, E) for E in ops)


def fdm_diag_weight(rho, n, phase):
    w = popcount(np.arange(2 ** n, dtype=np.uint64))
    d = np.asarray(phase, dtype=np.complex128)[w]
    return d[:, None] * rho * d.conj()[None, :]


def run_fdm(program) -> np.ndarray:
    """Exact evolution of the full 2^n x 2^n density matrix; compressions are skipped."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    n = program.n
    psi0 = _initial(program)
    rho = np.outer(psi0, psi0.conj())
    for op in program.ops:
        if isinstance(op, Gate):
            rho = fdm_gate(rho, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            rho = fdm_diag_weight(rho, n, op.phase)
        elif isinstance(op, Kraus):
            rho = fdm_channel(rho, n, op.qubit, op.ops, op.qubit2)
        elif isinstance(op, (Compress, LayerEnd)):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")
    return rho


def run_sv(program) -> np.ndarray:
    """Noiseless statevector of the same circuit (channels and compressions skipped)."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    n = program.n
    psi = _initial(program)[:, None]
    w = popcount(np.arange(2 ** n, dtype=np.uint64))
    for op in program.ops:
        if isinstance(op, Gate):
            psi = apply_gate(psi, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            psi = psi * np.asarray(op.phase)[w][:, None]
        elif isinstance(op, (Kraus, Compress, LayerEnd)):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")
    return psi[:, 0]
