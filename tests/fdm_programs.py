"""Seeded mixed programs for the full-rank comparator tests: random 1- and 2-qubit unitaries,
CNOT, diagonal CZ and RZ gates, and single-qubit channels in random order."""
import numpy as np

from workloads import circuits as C


def rand_unitary(rng, k):
    a = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def mixed_program(n, seed, count=60):
    rng = np.random.default_rng(seed)
    chans = [C.depolarizing(0.05), C.amplitude_damping(0.2), C.phase_flip(0.1), C.bit_flip(0.07)]
    ops = []
    for _ in range(count):
        kind = int(rng.integers(0, 6))
        if n == 1:
            kind = (0, 4, 5)[kind % 3]
            q0, q1 = 0, 0
        else:
            q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
        if kind == 0:
            ops.append(C.Gate((q0,), rand_unitary(rng, 1)))
        elif kind == 1:
            ops.append(C.Gate((q0, q1), C.CNOT))
        elif kind == 2:
            ops.append(C.Gate((q0, q1), C.CZ, diagonal=True))
        elif kind == 3:
            ops.append(C.Gate((q0, q1), rand_unitary(rng, 2)))
        elif kind == 4:
            ops.append(C.Gate((q0,), C.rz(rng.uniform(-3, 3)), diagonal=True))
        else:
            ops.append(C.Kraus(q0, chans[int(rng.integers(0, 4))]))
    return C.Program(n, ops, 2 ** n, "c64", 4, "mixed", 1)
