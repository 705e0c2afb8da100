"""Low Rank simulation with Eigenvalue Truncation (LRET), FP64 oracle (test infrastructure only).

Follows the paper step by step:
  * state rho = L L^H with L in C^{2^N x V}                 (Eq. "low rank decomposition", Sec. II.A)
  * gate: L <- G L                                          (Eq. "low rank evolution G")
  * Kraus channel: L <- [sqrt(p_1) K_1 L, ..., sqrt(p_A) K_A L]   (Eq. "low rank evolution K")
  * truncation after each channel group (one- or two-qubit)   (Sec. II.C; Algorithm 1)
  * a switch to full density matrix evolution once the intermediate rank reaches 2^N
                                                              (Sec. II.C, last paragraph)
  * truncation through the small matrix L^H L instead of rho   (Sec. II.B, Theorem 1 of App. B)

Readings where the paper is silent (each also listed in the design notes):
  * Compressed factor.  Theorem 1 gives the eigenvectors of rho' = L'L'^H as u_i = L' v_i /
    sqrt(lambda_i), so the truncated state sum_{i<=k} lambda_i u_i u_i^H equals
    (L' V_k)(L' V_k)^H: the new factor is L' V_k (times the renormalisation scale c).
  * Rank rule.  k = min(r, N, k_eps).  k_eps is the smallest k whose kept mass
    K_k = sum_{i<=k} max(lambda_i, 0) reaches (1 - eps) Tr G: the eigenvalues are taken in
    descending order until their sum reaches the target (Sec. II.B), measured against the trace
    rather than against 1; eps = 0 disables the threshold (fixed-rank mode).
  * Ties.  tie=1 ("cluster") lowers k while lambda_k - lambda_{k+1} <= TAU_CLUSTER * Tr G, so
    that the kept set is gap-separated and the truncated state is unique; beyond the Gram order
    N the spectrum of rho' continues with zeros (lambda_{N+1} = 0), so the rule does not depend
    on how many zero columns the factor carries; tie=0 keeps the eigensolver's order.
  * Renormalisation.  renorm=1 scales the kept part to unit trace, c = K_k^{-1/2}; renorm=0 is
    the paper-literal truncation (c = 1).
  * Discarded mass delta = Tr G - K_k.
"""
from __future__ import annotations

import numpy as np

from .linalg import apply_gate, popcount

TAU_CLUSTER = 1e-6


def init_state(n: int) -> np.ndarray:
    """L^(0) = [1, 0, ..., 0]^T: the |0...0> fiducial state (Algorithm 1)."""
    L = np.zeros((2 ** n, 1), dtype=np.complex128)
    L[0, 0] = 1.0
    return L


def apply_diag_weight(L: np.ndarray, n: int, phase: np.ndarray) -> np.ndarray:
    """L[x, :] *= phase[popcount(x)] -- a diagonal gate that depends on the Hamming weight."""
    w = popcount(np.arange(2 ** n, dtype=np.uint64))
    return L * np.asarray(phase, dtype=np.complex128)[w][:, None]


def init_sparse(n: int, idx, amp) -> np.ndarray:
    """A sparse linear combination of basis states, sum_i a_i |x_i>, as a one-column factor (the
    other initial states Algorithm 1 admits, Sec. II.D)."""
    L = np.zeros((2 ** n, 1), dtype=np.complex128)
    L[np.asarray(idx, dtype=np.int64), 0] = np.asarray(amp, dtype=np.complex128)
    return L


def kraus_expand(L: np.ndarray, n: int, qubit: int, ops: np.ndarray, qubit2: int = -1) -> np.ndarray:
    """L' = [E_1 L | E_2 L | ... | E_A L] with E_a = sqrt(p_a) K_a acting on `qubit` (or on the
    pair (qubit, qubit2) for a two-qubit channel, Sec. II.C) (Eq. "low rank evolution K"); the
    column count grows A-fold, block-major by a."""
    qs = (qubit,) if qubit2 < 0 else (qubit, qubit2)
    return np.concatenate([apply_gate(L, n, qs, E) for E in ops], axis=1)


def intermediate_rank(n: int, A: int, V: int, M: int) -> float:
    """V_I with V_I^3 = N (A V)^3 / M (Eq. "intermediate rank", Sec. II.C): A Kraus matrices per
    group of M qubits acting on a factor of V columns."""
    return (n / M) ** (1.0 / 3.0) * A * V


def select_rank(lam_desc: np.ndarray, trace: float, r: int, eps: float, tie: int,
                tau: float = TAU_CLUSTER) -> int:
    """Number of kept eigenvalues k from descending eigenvalues (rank rule, Sec. II.B)."""
    N = lam_desc.shape[0]
    k = min(r, N)
    lp = np.maximum(lam_desc, 0.0)
    if eps > 0.0:
        kept = np.cumsum(lp)
        target = (1.0 - eps) * trace
        hit = np.nonzero(kept >= target)[0]
        k_eps = int(hit[0]) + 1 if hit.size else N
        k = min(k, k_eps)
    if tie == 1:
        # beyond the Gram order the spectrum of rho' continues with zeros (rank <= N)
        while k > 1 and (lam_desc[k - 1] - (lam_desc[k] if k < N else 0.0)) <= tau * trace:
            k -= 1
    return max(k, 1)


def compress(L: np.ndarray, r: int, eps: float = 0.0, tie: int = 0, renorm: int = 1):
    """Eigenvalue truncation of rho' = L'L'^H through G = L'^H L' (Theorem 1).

    Returns (L_new, info) with L_new = c L' V_k and info = {k, discarded, trace, gap, lam_k
    (the smallest kept eigenvalue), lam, scale}."""
    G = L.conj().T @ L                       # Gram matrix, V x V (Theorem 1: shares rho's spectrum)
    G = 0.5 * (G + G.conj().T)
    lam, V = np.linalg.eigh(G)               # ascending
    lam = lam[::-1]
    V = np.ascontiguousarray(V[:, ::-1])     # descending; contiguous so the product goes to BLAS
    trace = float(np.real(np.trace(G)))
    k = select_rank(lam, trace, r, eps, tie)
    kept = float(np.sum(np.maximum(lam[:k], 0.0)))
    c = 1.0 / np.sqrt(kept) if renorm else 1.0
    L_new = c * (L @ V[:, :k])
    gap = float(lam[k - 1] - lam[k]) if k < lam.shape[0] else float("inf")
    info = dict(k=k, discarded=max(trace - kept, 0.0), trace=trace, gap=gap, lam_k=float(lam[k - 1]),
                lam=lam.copy(), scale=c)
    return L_new, info


def run_lret(program, L0: np.ndarray | None = None, log: list | None = None) -> np.ndarray:
    """Algorithm 1: gates, then for every channel group concatenate and truncate.  Ops are
    executed in program order; returns the final factor L^(D)."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    n = program.n
    if L0 is not None:
        L = np.array(L0, dtype=np.complex128)
    elif program.init is not None:
        L = init_sparse(n, *program.init)
    else:
        L = init_state(n)
    for op in program.ops:
        if isinstance(op, Gate):
            L = apply_gate(L, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            L = apply_diag_weight(L, n, op.phase)
        elif isinstance(op, Kraus):
            L = kraus_expand(L, n, op.qubit, op.ops, op.qubit2)
        elif isinstance(op, Compress):
            L, info = compress(L, op.r, op.eps, op.tie, op.renorm)
            if log is not None:
                info.pop("lam")
                log.append(info)
        elif isinstance(op, LayerEnd):
            pass
        else:
            raise TypeError(f"unknown op {op!r}")
    return L


def run_lret_switching(program):
    """Algorithm 1 with the switch of Sec. II.C: before each channel group, if its intermediate
    rank V_I (A Kraus matrices on M qubits, V the current column count) reaches 2^N, the low-rank
    evolution stops, rho = L L^H is formed and the remaining operations run as full density
    matrix evolution (compressions no longer apply).  Returns (rho, index of the operation at
    which the switch happened, or -1) with rho = L L^H when no switch happened."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    from .fdm import fdm_channel, fdm_diag_weight, fdm_gate

    n = program.n
    L = init_sparse(n, *program.init) if program.init is not None else init_state(n)
    rho = None
    switched = -1
    for i, op in enumerate(program.ops):
        if rho is None and isinstance(op, Kraus):
            if intermediate_rank(n, op.ops.shape[0], L.shape[1], len(op.qubits)) >= 2 ** n:
                rho = L @ L.conj().T
                switched = i
        if rho is not None:
            if isinstance(op, Gate):
                rho = fdm_gate(rho, n, op.qubits, op.u)
            elif isinstance(op, DiagWeight):
                rho = fdm_diag_weight(rho, n, op.phase)
            elif isinstance(op, Kraus):
                rho = fdm_channel(rho, n, op.qubit, op.ops, op.qubit2)
            elif not isinstance(op, (Compress, LayerEnd)):
                raise TypeError(f"unknown op {op!r}")
            continue
        if isinstance(op, Gate):
            L = apply_gate(L, n, op.qubits, op.u)
        elif isinstance(op, DiagWeight):
            L = apply_diag_weight(L, n, op.phase)
        elif isinstance(op, Kraus):
            L = kraus_expand(L, n, op.qubit, op.ops, op.qubit2)
        elif isinstance(op, Compress):
            L, _ = compress(L, op.r, op.eps, op.tie, op.renorm)
        elif not isinstance(op, LayerEnd):
            raise TypeError(f"unknown op {op!r}")
    return (L @ L.conj().T if rho is None else rho), switched
