"""Distortion of the low-rank path against the exact noisy state, layer by layer.

The error measure of Sec. III (Eq. "distortion") compares computational-basis diagonals:
distortion = T(rho_LRET, rho_exact) / T(rho_exact, rho_noiseless) with
T(A, B) = sum_i |A_ii - B_ii| (as written, without the 1/2 of total variation).

All three states are evolved on the GPU by this library: the low-rank factor with its
eigenvalue truncations (LowRankDM), the exact noisy state as a full-rank density matrix
(FullRankDM, no truncation), and the noiseless state as a rank-one factor that sees the same
gates and no channels.  Only the three 2^n diagonals come back to the host after each layer,
where the two sums are taken in FP64.  The exact state needs 8 * 4^n bytes of device memory
(2.1 GB at n = 14, 34 GB at n = 16).
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

from .lrdm import C64, FullRankDM, LowRankDM


def _host(t) -> np.ndarray:
    return t.cpu().numpy().astype(np.float64)


def distortion(p_lret: np.ndarray, p_exact: np.ndarray, p_noiseless: np.ndarray) -> float:
    """T(rho_LRET, rho_exact) / T(rho_exact, rho_noiseless) on diagonals (Sec. III)."""
    den = float(np.sum(np.abs(p_exact - p_noiseless)))
    return float(np.sum(np.abs(p_lret - p_exact))) / den if den > 0.0 else float("nan")


def exact_diagonals(program) -> List[np.ndarray]:
    """Diagonal of the exact noisy state after every layer: the program's gates, phases and
    channels on the full-rank density matrix (its compressions do not apply there)."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    f = FullRankDM(program.n)
    out = []
    try:
        for op in program.ops:
            if isinstance(op, Gate):
                f.apply_gate(op.qubits, op.u)
            elif isinstance(op, Kraus):
                f.apply_kraus(op.qubit, op.ops)
            elif isinstance(op, DiagWeight):
                f.apply_diagonal_weight(op.phase)
            elif isinstance(op, LayerEnd):
                out.append(_host(f.probabilities()))
            elif not isinstance(op, Compress):
                raise TypeError(f"the full-rank comparator cannot apply {op!r}")
    finally:
        f.close()
    return out


def lowrank_diagonals(program, r_max: int = 0, dtype: int = C64) -> Dict[str, object]:
    """Diagonal of the low-rank state after every layer, with the rank each compression kept.

    Returns {"P": [per-layer diagonal], "ranks": [per-layer rank after its last compression],
    "max_rank", "compressions", "cap_hits", "discarded_total"}.  A cap hit is a compression
    whose threshold rank lay above the column bound r (k = r while more than eps Tr G was
    discarded): there the truncation is set by r, not by eps."""
    from workloads.circuits import Compress, DiagWeight, Gate, Kraus, LayerEnd

    r_max = r_max or program.r
    dm = LowRankDM(program.n, r_max, dtype, max(program.m_max, 2))
    P, ranks, rank, n_c, caps, disc = [], [], 1, 0, 0, 0.0
    try:
        for op in program.ops:
            if isinstance(op, Gate):
                dm.apply_gate(op.qubits, op.u)
            elif isinstance(op, DiagWeight):
                dm.apply_diagonal_weight(op.phase)
            elif isinstance(op, Kraus):
                dm.apply_kraus(op.qubit, op.ops)
            elif isinstance(op, Compress):
                info = dm.compress(op.r, op.eps, op.tie, op.renorm, info=True)
                rank, n_c = info["rank"], n_c + 1
                if rank >= op.r and info["discarded"] > op.eps * info["trace_before"]:
                    caps += 1
                disc = info["discarded_total"]
            elif isinstance(op, LayerEnd):
                P.append(_host(dm.probabilities()))
                ranks.append(rank)
            else:
                raise TypeError(f"unknown op {op!r}")
    finally:
        dm.close()
    return {"P": P, "ranks": ranks, "max_rank": max(ranks) if ranks else 1, "compressions": n_c,
            "cap_hits": caps, "discarded_total": disc}


def noiseless_program(program):
    """The same program with its channels and compressions removed (same gates, same layers)."""
    from workloads.circuits import Compress, Kraus, Program

    ops = [op for op in program.ops if not isinstance(op, (Kraus, Compress))]
    return Program(program.n, ops, 8, "c64", 2, program.name + "-noiseless", program.layers, {})


def program_distortion(program, dtype: int = C64) -> Dict[str, object]:
    """Per-layer distortion of any program made of gates, channels and compressions, with the
    rank kept after each layer (lowrank_diagonals' fields besides "P")."""
    exact = exact_diagonals(program)
    ideal = lowrank_diagonals(noiseless_program(program))["P"]
    lo = lowrank_diagonals(program, dtype=dtype)
    out = {k: v for k, v in lo.items() if k != "P"}
    out["distortion"] = [distortion(a, e, i) for a, e, i in zip(lo["P"], exact, ideal)]
    out["exact_minus_noiseless"] = [float(np.sum(np.abs(e - i))) for e, i in zip(exact, ideal)]
    return out


def distortion_study(n: int, depth: int, kind: str, channel: str, p: float, eps_list: Sequence[float],
                     seed: int, r: int, tie: int = 0, dtype: int = C64) -> Dict[str, object]:
    """Per-layer distortion of one random circuit (workloads.circuits.random_circuit) for every
    threshold in eps_list.  The exact and noiseless diagonals are computed once and shared.

    Returns {"exact_minus_noiseless": [T per layer], "eps": {eps: {"distortion": [per layer],
    "ranks", "max_rank", "compressions", "cap_hits"}}}."""
    from workloads import circuits as C

    noisy = C.random_circuit(n, depth, kind, channel, p=p, r=r, eps=0.0, seed=seed)
    exact = exact_diagonals(noisy)
    ideal = lowrank_diagonals(noiseless_program(noisy))["P"]
    res: Dict[str, object] = {"exact_minus_noiseless": [float(np.sum(np.abs(e - i))) for e, i in zip(exact, ideal)],
                              "eps": {}}
    for eps in eps_list:
        prog = C.random_circuit(n, depth, kind, channel, p=p, r=r, eps=eps, seed=seed, tie=tie)
        lo = lowrank_diagonals(prog, dtype=dtype)
        res["eps"][eps] = {"distortion": [distortion(a, e, i) for a, e, i in zip(lo["P"], exact, ideal)],
                           "ranks": lo["ranks"], "max_rank": lo["max_rank"],
                           "compressions": lo["compressions"], "cap_hits": lo["cap_hits"]}
    return res
