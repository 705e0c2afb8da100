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


def fdm_gate(rho, n, qubits, U):
    return _sandwich(rho, n, qubits, U)


def fdm_channel(rho, n, qubit, ops):
    return sum(_sandwich(rho, n, (qubit,), E) for E in ops)


def fdm_diag_weight(rho, n, phase):
    w = popcount(np.arange(2 ** n, dtype=np.uint64))
    d = np.asarray(phase, dtype=np.complex128)[w]
    return d[:, None] * rho * d.conj()[None, :]


def run_fdm(program) -> np.ndarray:
    """Exact evolution of the full 2^n x 2^n density matrix; compressions are skipped."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    n = program.n
    rho = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
    rho[0, 0] = 1.0
    for op in program.ops:
        if isinstance(op, Gate):
            rho = fdm_gate(rho, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            rho = fdm_diag_weight(rho, n, op.phase)
        elif isinstance(op, Kraus):
            rho = fdm_channel(rho, n, op.qubit, op.ops)
        elif isinstance(op, (Compress, LayerEnd)):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")
    return rho


def run_sv(program) -> np.ndarray:
    """Noiseless statevector of the same circuit (channels and compressions skipped)."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    n = program.n
    psi = np.zeros((2 ** n, 1), dtype=np.complex128)
    psi[0, 0] = 1.0
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
