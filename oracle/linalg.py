"""Column-wise gate application for the oracle (test infrastructure only).

Each column of L is a statevector of n qubits; a gate G acts on every column, L <- G L
(Eq. "low rank evolution G", Sec. II.A).  Qubit q is bit q of the basis index x.
"""
import numpy as np


def popcount(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    c = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        c += (x & np.uint64(1)).astype(np.int64)
        x = x >> np.uint64(1)
    return c


def apply_gate(L: np.ndarray, n: int, qubits, U: np.ndarray) -> np.ndarray:
    """Return G L where G is the k-qubit matrix U acting on `qubits` (local index
    i = sum_j b(qubits[j]) 2^j) and identity elsewhere; L has shape (2^n, V)."""
    qubits = tuple(int(q) for q in qubits)
    k = len(qubits)
    V = L.shape[1]
    t = L.reshape((2,) * n + (V,))
    # In a C-order reshape the axis of qubit q is n-1-q.  U reshaped to 2k binary axes has its
    # most significant local bit (qubits[k-1]) first, for both the output and the input half.
    in_axes = [n - 1 - qubits[j] for j in reversed(range(k))]
    Ut = np.asarray(U, dtype=np.complex128).reshape((2,) * (2 * k))
    res = np.tensordot(Ut, t, axes=(list(range(k, 2 * k)), in_axes))
    res = np.moveaxis(res, list(range(k)), in_axes)
    return np.ascontiguousarray(res).reshape(2 ** n, V)
