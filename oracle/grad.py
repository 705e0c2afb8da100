"""Energy gradients of a noisy parametrised circuit under LRET (FP64; test infrastructure only).

The paper defines the forward map only (Sec. II, Algorithm 1).  The quantity differentiated
here is the energy E(theta) = sum_k c_k Tr(L^H P_k L) of the final factor (the observable
formula of Sec. II.D), where theta are the angles of rotation gates R_P(theta) = exp(-i theta P/2)
and every compression is the eigenvalue truncation of Sec. II.B with a fixed kept rank k.

Two independent routes are given:

  * energy_grad_fd      -- central finite differences of the forward oracle (h = 1e-4);
  * energy_grad_adjoint -- reverse mode, one backward sweep, FP64.

Reverse-mode rules (loss l real, adjoint Lbar defined by dl = 2 Re Tr(Lbar^H dL)):

  * energy seed:  Lbar = H L.
  * gate L_a = U L_b:  Lbar_b = U^H Lbar_a, and for U = exp(-i theta P/2) on one qubit
    dl/dtheta = Im Tr(Lbar_a^H P L_a).
  * Kraus concatenation L' = [E_1 L | ... | E_m L]:  Lbar = sum_a E_a^H Lbar'_a.
  * truncation L_n = c L' V_K (Theorem 1 gives the truncated state c^2 L' P_K L'^H, with P_K the
    projector on the kept eigenvectors of G = L'^H L' and c = (sum_K lambda)^(-1/2) when
    renormalising, else 1).  With Z = V_D^H (c L'^H Lbar_n), Zhat_ji = Z_ji / (lambda_i -
    lambda_j) for kept i and discarded j, Ghat = V_K Zhat^H V_D^H and s = Re Tr(Lbar_n^H L_n):
        Lbar' = c Lbar_n V_K^H + L' (Ghat + Ghat^H) - s c^2 L' P_K
    (the last term only when renormalising).  It follows from the first-order change of the
    spectral projector, dP_K = sum_{i in K, j in D} (v_j v_j^H dG v_i v_i^H + h.c.) /
    (lambda_i - lambda_j), and of c^2 = 1 / Tr(P_K G); rotations inside the kept set drop out
    because the loss depends on L_n only through L_n L_n^H.  Pairs with lambda_i = lambda_j
    (possible only when both belong to the null space of L', where Z_ji = 0) contribute nothing.

Pins: tests/test_oracle_grad.py checks the adjoint against central differences, against the
exact parameter-shift rule when nothing is truncated, and the truncation rule against central
differences of a single compression.
"""
from __future__ import annotations

import numpy as np

from .linalg import apply_gate, popcount
from .lret import compress, init_state, kraus_expand, select_rank

PAULI = {
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def apply_pauli_sum(L: np.ndarray, n: int, xmasks, zmasks, coeffs) -> np.ndarray:
    """H L for H = sum_k c_k P_k, P_k = i^{|x_k & z_k|} X^{x_k} Z^{z_k} (qubit q = bit q)."""
    idx = np.arange(2 ** n, dtype=np.uint64)
    out = np.zeros_like(L)
    for xm, zm, c in zip(xmasks, zmasks, coeffs):
        xm, zm = int(xm), int(zm)
        ny = bin(xm & zm).count("1")
        sign = 1.0 - 2.0 * (popcount(idx & np.uint64(zm)) & 1)
        # (P L)[x ^ xm] = i^ny (-1)^{|x & zm|} L[x]
        PL = np.empty_like(L)
        PL[(idx ^ np.uint64(xm)).astype(np.int64)] = ((1j) ** ny) * sign[:, None] * L
        out += float(c) * PL
    return out


def energy(program, xmasks, zmasks, coeffs) -> float:
    """E = sum_k c_k Tr(L^H P_k L) of the final factor of the LRET run of `program`."""
    from .lret import run_lret

    L = run_lret(program)
    return float(np.real(np.vdot(L, apply_pauli_sum(L, program.n, xmasks, zmasks, coeffs))))


def energy_grad_fd(make_program, theta: np.ndarray, xmasks, zmasks, coeffs, h: float = 1e-4,
                   indices=None) -> np.ndarray:
    """Central differences [E(theta + h e_i) - E(theta - h e_i)] / (2 h) of the forward oracle;
    make_program(theta) builds the circuit for a flat or shaped angle array."""
    th = np.array(theta, dtype=np.float64)
    flat = th.reshape(-1)
    idx = range(flat.size) if indices is None else indices
    g = np.zeros(flat.size)
    for i in idx:
        p = flat.copy(); p[i] += h
        m = flat.copy(); m[i] -= h
        g[i] = (energy(make_program(p.reshape(th.shape)), xmasks, zmasks, coeffs)
                - energy(make_program(m.reshape(th.shape)), xmasks, zmasks, coeffs)) / (2 * h)
    return g


def compress_adjoint(A: np.ndarray, Lbar_n: np.ndarray, r: int, eps: float = 0.0, tie: int = 0,
                     renorm: int = 1) -> np.ndarray:
    """Adjoint of L_n = c A V_K with respect to A (= L', the concatenated factor)."""
    G = A.conj().T @ A
    G = 0.5 * (G + G.conj().T)
    lam, V = np.linalg.eigh(G)
    lam, V = lam[::-1], V[:, ::-1]
    trace = float(np.real(np.trace(G)))
    k = select_rank(lam, trace, r, eps, tie)
    kept = float(np.sum(np.maximum(lam[:k], 0.0)))
    c = 1.0 / np.sqrt(kept) if renorm else 1.0
    VK, VD = V[:, :k], V[:, k:]
    L_n = c * (A @ VK)
    Abar = c * (Lbar_n[:, :k] @ VK.conj().T)
    if VD.shape[1] > 0:
        Z = VD.conj().T @ (c * (A.conj().T @ Lbar_n[:, :k]))      # |D| x |K|
        den = lam[None, :k] - lam[k:, None]                          # lambda_i - lambda_j
        tiny = 1e-13 * max(trace, 1e-300)
        Zh = np.where(np.abs(den) > tiny, Z / np.where(np.abs(den) > tiny, den, 1.0), 0.0)
        Gh = VK @ Zh.conj().T @ VD.conj().T
        Abar = Abar + A @ (Gh + Gh.conj().T)
    if renorm:
        s = float(np.real(np.vdot(Lbar_n[:, :k], L_n)))
        Abar = Abar - s * c * c * (A @ (VK @ VK.conj().T))
    return Abar


def energy_grad_adjoint(program, n_params: int, xmasks, zmasks, coeffs):
    """(E, dE/dtheta) by one reverse sweep over the recorded forward run of `program`.

    Gate ops carry `param = (index, axis)` for R_axis(theta[index]); other gates are constant."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    from .lret import apply_diag_weight

    n = program.n
    L = init_state(n)
    tape = []      # (op, state before op)
    for op in program.ops:
        if isinstance(op, Gate):
            tape.append((op, L))
            L = apply_gate(L, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            tape.append((op, L))
            L = apply_diag_weight(L, n, op.phase)
        elif isinstance(op, Kraus):
            tape.append((op, L))
            L = kraus_expand(L, n, op.qubit, op.ops)
        elif isinstance(op, Compress):
            tape.append((op, L))
            L, _ = compress(L, op.r, op.eps, op.tie, op.renorm)
        elif isinstance(op, LayerEnd):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")
    HL = apply_pauli_sum(L, n, xmasks, zmasks, coeffs)
    E = float(np.real(np.vdot(L, HL)))
    Lbar = HL
    grad = np.zeros(n_params)
    L_after = L
    for op, L_before in reversed(tape):
        if isinstance(op, Gate):
            if op.param is not None:
                idx, axis = op.param
                PL = apply_gate(L_after, n, op.qubits, PAULI[axis])
                grad[idx] += float(np.imag(np.vdot(Lbar, PL)))
            Lbar = apply_gate(Lbar, n, op.qubits, np.asarray(op.u).conj().T)
        elif isinstance(op, DiagWeight):
            Lbar = apply_diag_weight(Lbar, n, np.conj(op.phase))
        elif isinstance(op, Kraus):
            c = L_before.shape[1]
            Lbar = sum(apply_gate(Lbar[:, a * c:(a + 1) * c], n, (op.qubit,), np.asarray(E).conj().T)
                       for a, E in enumerate(op.ops))
        elif isinstance(op, Compress):
            Lbar = compress_adjoint(L_before, Lbar, op.r, op.eps, op.tie, op.renorm)
        L_after = L_before
    return E, grad


def parameter_shift(make_program, theta: np.ndarray, xmasks, zmasks, coeffs, indices) -> np.ndarray:
    """[E(theta + pi/2 e_i) - E(theta - pi/2 e_i)] / 2: exact for R_P(theta) when the map from
    the gate's output state to E is linear in rho, i.e. when no compression truncates."""
    th = np.array(theta, dtype=np.float64)
    flat = th.reshape(-1)
    g = np.zeros(flat.size)
    for i in indices:
        p = flat.copy(); p[i] += np.pi / 2
        m = flat.copy(); m[i] -= np.pi / 2
        g[i] = 0.5 * (energy(make_program(p.reshape(th.shape)), xmasks, zmasks, coeffs)
                      - energy(make_program(m.reshape(th.shape)), xmasks, zmasks, coeffs))
    return g
