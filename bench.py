"""Benchmark: noisy-circuit layers/s of the low-rank density-matrix path on one MI355X.

Workload (one step): the random brickwork circuit with n = 20 qubits, rank r = 64, 40 layers
of Haar SU(2) on every qubit plus CZ on alternating pairs, and per qubit per layer amplitude
damping (gamma = 0.002) -> compress -> dephasing (p = 0.001) -> compress (1600 compressions);
then <Z_i Z_{i+1}> for all neighbours and 10^4 samples.  Complex FP32 bulk (FP32 MFMA Gram and
projection), FP64 eigensolve.  Inputs are seeded and synthetic.

Prints one JSON line (rank 0).  --gpus > 1 is not supported: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "noisy-circuit layers/s at n=20 r=64 vs full-rank DM, same GPU; %HBM peak; grads/s"
FP32_MFMA_PEAK = 157.3e12
FP64_PEAK = 78.6e12      # vector (and MFMA): 256 CUs x 2.4 GHz x 128 flop per CU and clock
HBM_PEAK = 8.0e12
CLASS_NAMES = {0: "gate_pass", 1: "gram", 2: "gram_reduce", 3: "eigensolve", 4: "projection", 5: "small_fp64",
               6: "gram_pair"}


# Blocks of the projection matrix W (2 x 2 blocks of r x r, input value -> output value of the
# channel's qubit) that are not identically zero for amplitude damping followed by dephasing:
# no Kraus operator of either channel maps |0> to |1> (amplitude damping only lowers, dephasing
# is diagonal), so the composed W has a zero block from input half 0 to output half 1, and 3 of
# the 4 blocks carry work.
PROJ_NONZERO_BLOCKS = 3


def algorithmic_flops(n: int, r_pad: int, cls: int, m: int = 2, k: int = 64, blocks: int = PROJ_NONZERO_BLOCKS) -> float:
    """Real flops one launch must do (complex MAC = 8 flops).  Gram and projection work on the
    split view X = [L_0 | L_1] (2^(n-1) x 2r): the Gram matrix is Hermitian (half of X^H X),
    the projection is X W with W of size 2r x 2r, of which `blocks` of the four r x r blocks are
    not identically zero.  The eigensolve of the order-N Gram matrix (N = m r_pad) counts the
    Householder reduction to tridiagonal form, (16/3) N^3, and the back-transform of the k kept
    eigenvectors, 8 N^2 k (the O(N^2) tridiagonal part is left out)."""
    rows, w = 2 ** (n - 1), 2 * r_pad
    if cls == 1:
        return 8.0 * rows * w * w / 2
    if cls == 6:   # 4-way Gram of a bit pair, the Hermitian Y^H Y with Y = [X_0 | X_1] over 2^(n-2)
        # rows: the two halves (split Grams over half the rows each) and the full cross block
        return 2 * 8.0 * (rows / 2) * w * w / 2 + 8.0 * (rows / 2) * w * w
    if cls == 4:
        return 8.0 * rows * w * w * blocks / 4
    if cls == 3:
        N = m * r_pad
        return 16.0 / 3.0 * N ** 3 + 8.0 * N * N * k
    raise ValueError(cls)


COUNTERS_FILE = os.path.join(ROOT, "profiles", "all_kernels_brickwork_n20_r64_hbm_counters.md")
CLASS_SOURCE = {0: "k_gate.hip", 1: "k_gram.hip", 3: "k_eig.hip", 4: "k_proj.hip", 6: "k_gram.hip"}


def measured_traffic(cls: int):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter read for a 1 GiB copy), or None
    when there is no summary or the kernel source has changed since the counters were taken."""
    import hashlib
    import re

    key = CLASS_NAMES[cls]
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    m = re.search(rf"^traffic_bytes_per_launch {key}: (\d+)$", text, re.M)
    src = CLASS_SOURCE.get(cls)
    h = re.search(rf"^kernel_source_sha256 {re.escape(src)}: ([0-9a-f]+)$", text, re.M) if src else None
    if not m or not h:
        return None
    path = os.path.join(ROOT, "paper_2009_06657_amd", "csrc", src)
    if hashlib.sha256(open(path, "rb").read()).hexdigest() != h.group(1):
        return None
    return int(m.group(1))


MFMA_FILE = os.path.join(ROOT, "profiles", "gemm_kernels_brickwork_n20_r64_mfma_counters.md")


def measured_mfma(cls: int):
    """MFMA counters of a GEMM kernel class from the committed rocprofv3 summary: busy fraction of
    the matrix cores over the kernel (SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x SIMDs)) and the
    FP32 MFMA operations it issued per launch (SQ_INSTS_VALU_MFMA_MOPS_F32 x 512), or None when
    there is no summary or the kernel source has changed since it was taken."""
    import hashlib
    import re

    key = CLASS_NAMES[cls]
    try:
        text = open(MFMA_FILE).read()
    except OSError:
        return None
    busy = re.search(rf"^mfma_busy_frac {key}: ([0-9.eE+-]+)$", text, re.M)
    flops = re.search(rf"^mfma_flops_per_launch {key}: ([0-9.eE+-]+)$", text, re.M)
    src = CLASS_SOURCE.get(cls)
    h = re.search(rf"^kernel_source_sha256 {re.escape(src)}: ([0-9a-f]+)$", text, re.M) if src else None
    if not busy or not flops or not h:
        return None
    path = os.path.join(ROOT, "paper_2009_06657_amd", "csrc", src)
    if hashlib.sha256(open(path, "rb").read()).hexdigest() != h.group(1):
        return None
    return {"busy_frac": float(busy.group(1)), "mfma_flops_per_launch": float(flops.group(1))}


def _against_golden(g, path, dm, zz, samples) -> dict:
    z, _, _ = dm.expect_z()
    P = dm.probabilities().cpu().numpy()
    idx = np.concatenate([np.array(g["prob_largest_idx"]), np.array(g["prob_random_idx"])])
    ref = np.concatenate([np.array(g["prob_largest"]), np.array(g["prob_random"])])
    dP = np.abs(P[idx] - ref)
    diff = np.nonzero(np.asarray(samples, dtype=np.uint64) != np.array(g["samples"], dtype=np.uint64))[0]
    margin = np.array(g["sample_margin"])
    return {"available": True, "golden": os.path.relpath(path, ROOT), "layers_compared": g.get("layers"),
            "zz": float(np.max(np.abs(np.asarray(zz) - np.array(g["zz"])))),
            "z": float(np.max(np.abs(z - np.array(g["z"])))),
            "prob_8192_fixed_idx": float(dP.max()),
            "prob_8192_fixed_idx_rel": float(np.max(dP / np.maximum(ref, 1e-300))),
            "trace": abs(float(np.sum(P)) - g["trace"]),
            "samples_differing": int(diff.size), "samples": int(len(samples)),
            "samples_differing_max_margin": float(margin[diff].max()) if diff.size else 0.0}


def error_vs_oracle(dm, prog, zz, samples, flags, uniforms) -> dict:
    """The step's outputs against the FP64 oracle's for the same circuit (tests/golden, written by
    tests/golden/make_cfg3_golden.py from the oracle alone): <Z_i Z_{i+1}> and <Z_i>, Prob(x) at
    8192 fixed indices (absolute and relative to the oracle's value), and the samples (those that
    differ, and the largest distance of their uniform to a CDF step of the oracle's distribution).
    Where no oracle run of the whole circuit is stored, the first four layers are run again with
    the same flags and compared with the stored oracle run of those layers."""
    import paper_2009_06657_amd as lr
    from workloads import circuits as C

    path = os.path.join(ROOT, "tests", "golden", f"cfg3_n20_r64_l{prog.layers}.json")
    if prog.n != 20 or prog.r != 64:
        return {"available": False, "reason": f"no oracle run stored for n={prog.n} r={prog.r}"}
    if os.path.exists(path):
        with open(path) as f:
            g = json.load(f)
        g.setdefault("layers", prog.layers)
        return _against_golden(g, path, dm, zz, samples)
    path4 = os.path.join(ROOT, "tests", "golden", "cfg3_n20_r64_l4.json")
    if not os.path.exists(path4):
        return {"available": False, "reason": f"no oracle run stored for n=20 r=64 layers={prog.layers} or 4"}
    with open(path4) as f:
        g = json.load(f)
    g.setdefault("layers", 4)
    prog4 = C.cfg3_program(layers=4)
    dm4 = lr.LowRankDM(prog4.n, prog4.r, lr.C64, prog4.m_max, flags)
    zz4, samples4, _ = run_step(dm4, prog4, uniforms)
    out = _against_golden(g, path4, dm4, zz4, samples4)
    out["note"] = f"no oracle run of all {prog.layers} layers stored: the first 4 layers, same flags"
    dm4.close()
    return out


def unflagged_comparator(prog, uniforms, ms_overlap: float, steps: int = 2) -> dict:
    """The same workload on one stream (no LRDM_FLAG_OVERLAP): every eigensolve waits for the
    Gram pass before it and the projection waits for it."""
    import torch

    import paper_2009_06657_amd as lr

    dm = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max)
    run_step(dm, prog, uniforms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        zz, _, _ = run_step(dm, prog, uniforms)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    dm.close()
    return {"layers_per_s": prog.layers * 1e3 / ms, "ms_per_step": ms, "overlap_speedup": ms / ms_overlap}


def plain_comparator(prog, uniforms, ms_fused: float, steps: int = 2) -> dict:
    """The plain low-rank form on the same workload and GPU: the Kraus concatenation
    [E_1 L | E_2 L] materialised in HBM (Eq. "low rank evolution K" taken literally, 2^20 x 128
    complex64), its full (m r) x (m r) Gram matrix, and the projection L' V_k, one compression at
    a time (no chaining of the two channels on a qubit)."""
    import torch

    import paper_2009_06657_amd as lr

    dm = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max, lr.FLAG_PLAIN)
    run_step(dm, prog, uniforms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        zz, _, tr = run_step(dm, prog, uniforms)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    br = {}
    for cls in (1, 3, 4):
        dm.timing_begin(cls)
        run_step(dm, prog, uniforms)
        br[cls] = dm.timing_end()
    rows, ld = 2 ** prog.n, dm.ld
    k = prog.r
    gram_flops = 8.0 * rows * ld * ld / 2            # Hermitian half of the (m r)^2 complex Gram
    proj_flops = 8.0 * rows * ld * k                 # L' (2^n x m r) times V_k (m r x k)
    dm.close()
    del dm
    torch.cuda.empty_cache()
    return {"workload": "same circuit, plain form (LRDM_FLAG_PLAIN): materialised Kraus concatenation, "
                        f"Gram of order {ld}, projection L' V_k, every compression separately",
            "layers_per_s": prog.layers * 1e3 / ms, "ms_per_step": ms, "fused_over_plain": ms / ms_fused,
            "trace_after": tr,
            "gram": {"launches": br[1][0], "mean_ms": br[1][1], "tflops": gram_flops / (br[1][1] * 1e-3) / 1e12,
                     "frac_fp32_mfma": gram_flops / (br[1][1] * 1e-3) / FP32_MFMA_PEAK},
            "projection": {"launches": br[4][0], "mean_ms": br[4][1],
                           "tflops": proj_flops / (br[4][1] * 1e-3) / 1e12,
                           "frac_fp32_mfma": proj_flops / (br[4][1] * 1e-3) / FP32_MFMA_PEAK},
            "eigensolve_mean_ms": br[3][1]}


def run_step(dm, prog, uniforms):
    from paper_2009_06657_amd import run_program

    dm.reset()
    run_program(dm, prog)
    z, zz, tr = dm.expect_z()
    s = dm.sample(uniforms)
    return zz, s, tr


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_layer_sample(n: int, r: int, budget_s: float, max_gates: int = 1 << 30, max_comp: int = 1 << 30):
    """From a steady-state rank-r factor: the gates and channel+compress steps of one brickwork
    layer that fit the budget; returns (per-gate s, gates done, per-compress s, compresses done,
    gates per layer, compresses per layer)."""
    import oracle
    from oracle.lret import compress, kraus_expand
    from workloads import circuits as C

    prog = C.cfg3_program(n=n, r=r, layers=1)
    L = C.random_orthogonal_factor(n, r, seed=4242)
    gates = [op for op in prog.ops if isinstance(op, C.Gate)]
    chans = [op for op in prog.ops if isinstance(op, C.Kraus)]
    t0 = time.perf_counter()
    g_done = 0
    for op in gates[:max_gates]:
        L = oracle.apply_gate(L, n, op.qubits, op.u)
        g_done += 1
        if time.perf_counter() - t0 > 0.25 * budget_s:
            break
    per_gate = (time.perf_counter() - t0) / g_done
    done, t_comp = 0, 0.0
    for ch in chans[:max_comp]:
        t1 = time.perf_counter()
        L, _ = compress(kraus_expand(L, n, ch.qubit, ch.ops), r)
        t_comp += time.perf_counter() - t1
        done += 1
        if t_comp > 0.75 * budget_s:
            break
    return per_gate, g_done, t_comp / done, done, len(gates), len(chans)


def cpu_baseline(n: int, r: int, budget_s: float = 20.0) -> dict:
    """The CPU oracle on the host cores.  The headline value: a bounded sample of the benchmark
    layer (from a steady-state rank-r factor, the layer's gates and as many channel+compress steps
    as fit the budget, extrapolated to the 30 gates and 40 compressions of a layer) with every BLAS
    thread; the same sample with one thread (one gate, one compression); and whole-run oracle
    times of the three smaller workloads."""
    import oracle
    from oracle import grad as OG
    from workloads import circuits as C

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max((p.get("num_threads", 1) for p in threadpool_info()), default=os.cpu_count())
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    per_gate, g_done, per_comp, done, ng, nc = _oracle_layer_sample(n, r, budget_s)
    t_layer = per_gate * ng + per_comp * nc
    out = {"value": 1.0 / t_layer, "unit": "layers/s", "cores": int(cores), "kind": "oracle",
           "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count(),
           "sample": (f"n={n} r={r}, from a steady-state rank-{r} factor: {g_done} of {ng} "
                      f"gates and {done} of {nc} channel+compress steps of one brickwork "
                      f"layer, extrapolated to the whole layer ({per_gate:.2f} s per gate, "
                      f"{per_comp:.2f} s per compress)")}
    if threadpool_limits is not None:
        with threadpool_limits(1):
            g1, _, c1, _, _, _ = _oracle_layer_sample(n, r, 1e9, max_gates=1, max_comp=1)
        out["one_thread"] = {"value": 1.0 / (g1 * ng + c1 * nc), "unit": "layers/s",
                             "sample": f"one gate ({g1:.2f} s) and one channel+compress step ({c1:.2f} s), "
                                       "extrapolated to the layer"}
    whole = {}
    t0 = time.perf_counter()
    prog = C.cfg1_program()
    oracle.run_lret(prog)
    whole["depolarizing_n6_r13_c128"] = {"s": time.perf_counter() - t0, "layers": prog.layers,
                                         "layers_per_s": prog.layers / (time.perf_counter() - t0)}
    t0 = time.perf_counter()
    prog = C.cfg2_program()
    oracle.run_lret(prog)
    whole["grover_n14_r32"] = {"s": time.perf_counter() - t0, "layers": prog.layers,
                               "layers_per_s": prog.layers / (time.perf_counter() - t0)}
    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    t0 = time.perf_counter()
    OG.energy_grad_adjoint(C.cfg4_program(theta), theta.size, xm, zm, co)
    dt = time.perf_counter() - t0
    whole["ansatz_n12_r16_energy_and_gradient"] = {"s": dt, "grads_per_s": 1.0 / dt,
                                                    "method": "the oracle's FP64 reverse sweep"}
    out["whole_runs"] = whole
    return out


def gradient_throughput(reps: int = 3) -> dict:
    """Energy + full gradient of the differentiable noisy ansatz (n=12, r=16, 8 layers of RY/RZ
    + CZ ladder, depolarizing 0.002 after every gate layer with a compression after each channel,
    200 Pauli terms, 192 angles) through the reverse sweep, complex64 bulk / FP64 eigensolve."""
    import torch

    import paper_2009_06657_amd as lr
    from paper_2009_06657_amd.adjoint import EnergyGradient
    from workloads import circuits as C

    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    eng = EnergyGradient(12, 16, 4, xm, zm, co, dtype=lr.C64)
    prog = C.cfg4_program(theta)
    eng.forward(prog)
    eng.backward(theta.size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        E = eng.forward(prog)
        g = eng.backward(theta.size)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = {"value": 1.0 / dt, "unit": "grads/s", "ms_per_grad": 1e3 * dt, "n_params": int(theta.size),
           "workload": "noisy RY/RZ ansatz n=12 r=16, 8 layers, depolarizing 0.002, 200 Pauli terms",
           "energy": E}
    gold = os.path.join(ROOT, "tests", "golden", "cfg4_grad.json")
    if os.path.exists(gold):
        with open(gold) as f:
            ref = json.load(f)
        out["max_abs_err_vs_fd"] = float(np.max(np.abs(g - np.array(ref["grad_fd"]))))
        out["abs_err_energy"] = abs(E - ref["energy"])
    eng.close()
    return out


def fdm_comparator(sizes=(10, 12, 14, 16), lret_n: int = 0) -> dict:
    """Same-GPU comparison with the full-rank density matrix: the brickwork layer (SU(2) on every
    qubit, CZ, amplitude damping + dephasing per qubit) on the full-rank kernel at n <= 16
    (rho of 8 * 4^n bytes; n = 20 would need 8.8 TB), the low-rank path at n = 16, r = 64 for a
    measured same-n ratio, and T_full(16) * 4^(20 - 16) as the extrapolated n = 20 layer time.
    The timed full-rank layers are queued together and run at one synchronization, so the
    host's operator fusion joins each layer's channels with the next layer's gates."""
    import torch

    import paper_2009_06657_amd as lr
    from workloads import circuits as C

    lret_n = lret_n or max(sizes)
    per_layer = {}
    for n in sizes:
        reps = 4
        prog = C.cfg3_program(n=n, r=64, layers=1 + reps)
        layers = [[]]
        for op in prog.ops:
            if isinstance(op, C.LayerEnd):
                layers.append([])
            else:
                layers[-1].append(op)
        f = lr.FullRankDM(n)

        def run_layers(ls):
            for seg in ls:
                lr.run_program_fdm(f, C.Program(n, seg, prog.r, prog.dtype, prog.m_max, "seg", 1))
            f.synchronize()

        run_layers(layers[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run_layers(layers[1:1 + reps])
        torch.cuda.synchronize()
        per_layer[n] = (time.perf_counter() - t0) / reps
        f.close()
        del f
        torch.cuda.empty_cache()
    # low-rank path at the largest full-rank size
    prog = C.cfg3_program(n=lret_n, r=64, layers=4)
    dm = lr.LowRankDM(lret_n, 64, lr.C64, prog.m_max)
    lr.run_program(dm, prog)
    dm.synchronize()
    dm.reset()
    t0 = time.perf_counter()
    lr.run_program(dm, prog)
    dm.synchronize()
    t_lret = (time.perf_counter() - t0) / 4
    dm.close()
    nmax = max(sizes)
    extrap = per_layer[nmax] * 4.0 ** (20 - nmax)
    return {"workload": "brickwork layer: SU(2) on every qubit + CZ, amplitude damping 0.002 and "
                        "dephasing 0.001 per qubit (full rank: exact channels; low rank: compress to r=64 after each)",
            "full_rank_ms_per_layer": {str(n): 1e3 * t for n, t in per_layer.items()},
            f"low_rank_ms_per_layer_n{lret_n}_r64": 1e3 * t_lret,
            f"speedup_same_n{nmax}": per_layer[nmax] / t_lret,
            "full_rank_ms_per_layer_n20_extrapolated": 1e3 * extrap,
            "extrapolation": f"T_full({nmax}) * 4^(20 - {nmax})"}


def fixed_rank_distortion() -> dict:
    """Distortion (Sec. III, Eq. "distortion") of the fixed-rank workloads against the full-rank
    density matrix on the same GPU: n = 6 depolarizing (r = 13, complex128), noisy Grover at
    n = 14 (r = 32) and the RY/RZ/CZ ansatz at n = 12 (r = 16), per layer and at the end."""
    import paper_2009_06657_amd as lr
    from paper_2009_06657_amd import accuracy as A
    from workloads import circuits as C

    t0 = time.perf_counter()
    per_workload = {}
    for name, prog, dt in (("n6_r13_depolarizing_c128", C.cfg1_program(), lr.C128),
                           ("grover_n14_r32", C.cfg2_program(), lr.C64),
                           ("ry_rz_cz_n12_r16", C.cfg4_program(C.cfg4_angles()), lr.C64)):
        res = A.program_distortion(prog, dtype=dt)
        # layers whose exact diagonal is within 1e-3 of the noiseless one (e.g. a uniform
        # superposition, which depolarizing noise leaves uniform) give no meaningful ratio
        by_layer = [d if den >= 1e-3 else None for d, den in zip(res["distortion"], res["exact_minus_noiseless"])]
        per_workload[name] = {"distortion_final": res["distortion"][-1], "distortion_by_layer": by_layer,
                         "layers": len(res["distortion"]), "max_rank": res["max_rank"], "r": prog.r,
                         "compressions": res["compressions"]}
        print(f"accuracy: {name} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    return per_workload


def accuracy_sweep(seeds=(1, 2, 3), depth: int = 12) -> dict:
    """Synthetic re-runs of the paper's accuracy studies (Sec. III.A): distortion of the low-rank
    path against the full-rank density matrix, both on this GPU, on seeded random circuits from
    the paper's gate set, averaged over seeds, at depths 4, 8 and 12 (one run per circuit gives
    every depth).  Studies: depolarizing p = 0.1 % over n and eps (Fig. 4); p = 0.3 % and 1 %
    with eps/p in {1, 0.3, 0.1, 0.03, 0.01} (Fig. 5); bit flip and amplitude damping p = 0.1 %
    (Fig. 7); the three circuit types under bit flip at n = 13, eps = 1e-4 (Fig. 8); and Fig. 5's
    strengths with depolarizing written as X, Y and Z flips (a compression after each, r = 64).
    First, the
    distortion of the fixed-rank workloads: n = 6 depolarizing (r = 13, complex128), noisy Grover
    at n = 14 (r = 32) and the RY/RZ/CZ ansatz at n = 12 (r = 16).  Rank caps:
    r = 32 for depolarizing (four Kraus operators, Gram order 4r <= 128), 64 otherwise; the
    compressions whose threshold rank lay above the cap are counted."""
    import paper_2009_06657_amd as lr
    from paper_2009_06657_amd import accuracy as A

    lr.load_library()
    t0 = time.perf_counter()
    fixed = fixed_rank_distortion()
    depths = [d for d in (4, 8, 12) if d <= depth]
    studies = []
    eps_grid = (1e-2, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5)
    for n in (4, 6, 8, 10, 12):
        studies.append(("fig4-depolarizing", n, "dense-local", "dep", 1e-3, eps_grid))
    for p in (3e-3, 1e-2):
        for n in (6, 8, 10, 12):
            studies.append(("fig5-noise-strength", n, "dense-local", "dep", p, tuple(p * f for f in (1, .3, .1, .03, .01))))
    for p in (3e-3, 1e-2):   # the same, depolarizing written as three flips: rank cap 64
        for n in (6, 8, 10, 12):
            studies.append(("fig5-noise-strength-flips", n, "dense-local", "dep3", p, tuple(p * f for f in (1, .3, .1, .03, .01))))
    for ch in ("bitflip", "ad"):
        for n in (4, 6, 8, 10, 12):
            studies.append(("fig7-channels", n, "dense-local", ch, 1e-3, eps_grid))
    for kind in ("dense-global", "dense-local", "sparse-local"):
        studies.append(("fig8-circuit-types", 13, kind, "bitflip", 1e-3, (1e-4,)))
    rows = []
    for name, n, kind, ch, p, eps_list in studies:
        r = 32 if ch == "dep" else 64
        runs = [A.distortion_study(n, depth, kind, ch, p, eps_list, seed, r) for seed in seeds]
        for eps in eps_list:
            per = [run["eps"][eps] for run in runs]
            rows.append({"study": name, "n": n, "kind": kind, "channel": ch, "p": p, "eps": eps,
                         "distortion": {str(d): float(np.mean([q["distortion"][d - 1] for q in per])) for d in depths},
                         "distortion_max_over_seeds": {str(d): float(np.max([q["distortion"][d - 1] for q in per]))
                                                       for d in depths},
                         "rank_by_layer": [float(np.mean([q["ranks"][t] for q in per])) for t in range(depth)],
                         "max_rank": int(max(q["max_rank"] for q in per)),
                         "cap_hits": int(sum(q["cap_hits"] for q in per)),
                         "compressions": int(sum(q["compressions"] for q in per))})
        print(f"accuracy: {name} n={n} {kind} {ch} p={p:g} done ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    return {"workload": f"random circuits (dense/sparse x local/global, paper gate set), depth {depth}, "
                        f"seeds {list(seeds)}; low rank (complex FP32, FP64 eigensolve, plain threshold "
                        "rule) vs full-rank density matrix (complex FP32), both on the GPU",
            "seconds": time.perf_counter() - t0, "fixed_rank": fixed, "rows": rows}


def batched_serving(count: int = 256, loop_budget_s: float = 30.0) -> dict:
    """The serving mix: `count` independent brickwork instances (n ~ U{8..16}, r ~ U{8,16,32},
    10..30 layers, depolarizing p ~ U(1e-4, 5e-3), compress after every channel, <Z> per
    instance) recorded once and replayed as one captured graph of lockstep batched launches,
    against looping the unbatched path over the same instances (timed until `loop_budget_s`, the
    rest extrapolated by layer count)."""
    import torch

    import paper_2009_06657_amd as lr
    from workloads import circuits as C

    progs = C.cfg5_instances(count)
    layers = np.array([p.layers for p in progs], dtype=np.float64)
    hs = [lr.LowRankDM(p.n, p.r, lr.C64, p.m_max) for p in progs]
    b = lr.Batch(hs)
    with b.recording():
        for dm, p in zip(hs, progs):
            dm.reset()
            lr.run_program(dm, p)
    steps, launches = b.info()
    b.launch()
    b.times()
    t0 = time.perf_counter()
    b.launch()
    done_ms, total_ms = b.times()
    zs = [dm.expect_z()[0] for dm in hs]
    wall = time.perf_counter() - t0
    b.close()
    for dm in hs:
        dm.close()
    del hs
    torch.cuda.empty_cache()
    # unbatched loop over the same instances (one handle reused per shape)
    per_inst = np.full(count, np.nan)
    t_start = time.perf_counter()
    cache = {}
    for i, p in enumerate(progs):
        key = (p.n, p.r, p.m_max)
        if key not in cache:
            cache[key] = lr.LowRankDM(p.n, p.r, lr.C64, p.m_max)
        dm = cache[key]
        t1 = time.perf_counter()
        dm.reset()
        lr.run_program(dm, p)
        dm.expect_z()
        per_inst[i] = time.perf_counter() - t1
        if time.perf_counter() - t_start > loop_budget_s:
            break
    ran = ~np.isnan(per_inst)
    loop_time = float(np.nansum(per_inst)) * (layers.sum() / layers[ran].sum())
    for dm in cache.values():
        dm.close()
    return {"workload": f"{count} brickwork instances, n U{{8..16}}, r U{{8,16,32}}, 10-30 layers, "
                        "depolarizing U(1e-4, 5e-3), compress after every channel, <Z> per instance",
            "instances": count, "total_layers": int(layers.sum()),
            "lockstep_steps": steps, "graph_launches": launches,
            "batched_layers_per_s": float(layers.sum() / (total_ms * 1e-3)),
            "batched_ms": total_ms, "batched_wall_ms_with_outputs": 1e3 * wall,
            "latency_ms_p50": float(np.percentile(done_ms, 50)), "latency_ms_p99": float(np.percentile(done_ms, 99)),
            "looped_layers_per_s": float(layers.sum() / loop_time), "looped_ms": 1e3 * loop_time,
            "looped_instances_timed": int(ran.sum()),
            "looped_latency_ms_p50": float(np.nanpercentile(per_inst, 50) * 1e3),
            "looped_latency_ms_p99": float(np.nanpercentile(per_inst, 99) * 1e3),
            "speedup": loop_time / (total_ms * 1e-3)}


def copy_calibration(torch, nbytes: int = 1 << 30, reps: int = 3) -> None:
    """A plain device-to-device copy of a known size: the HBM counters read for it (bytes
    fetched, bytes written per dispatch) give the scale factor applied to the same counters
    read for the path's kernels."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-breakdown", action="store_true",
                    help="profiler runs: skip the per-class kernel timing (one extra step per class) and every "
                         "other leg, print only the timed steps")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain low-rank form comparator")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient-throughput leg")
    ap.add_argument("--no-fdm", action="store_true", help="skip the full-rank comparator leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-serving leg")
    ap.add_argument("--fdm-only", action="store_true",
                    help="only run the full-rank comparator leg and print its result")
    ap.add_argument("--fdm-sizes", type=str, default="10,12,14,16",
                    help="qubit counts of the full-rank comparator leg (comma-separated, <= 16)")
    ap.add_argument("--no-distortion", action="store_true",
                    help="skip the distortion of the fixed-rank workloads against the full-rank DM")
    ap.add_argument("--accuracy-only", action="store_true",
                    help="only run the distortion sweeps (random circuits, low rank vs full rank) and print them")
    ap.add_argument("--no-tuning", action="store_true",
                    help="the library's default launch shapes instead of the autotuner's table")
    ap.add_argument("--no-overlap", action="store_true",
                    help="time the single-stream path (no LRDM_FLAG_OVERLAP) as the headline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(sharding is described in the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calib:
        copy_calibration(torch)
        return
    fdm_sizes = tuple(int(x) for x in args.fdm_sizes.split(","))
    if not fdm_sizes or min(fdm_sizes) < 1 or max(fdm_sizes) > 16:
        print("--fdm-sizes: qubit counts must lie in [1, 16]", file=sys.stderr)
        sys.exit(2)
    if args.fdm_only:
        print(json.dumps({"vs_full_rank_dm": fdm_comparator(fdm_sizes)}), flush=True)
        return
    if args.accuracy_only:
        print(json.dumps({"accuracy": accuracy_sweep()}), flush=True)
        return

    import paper_2009_06657_amd as lr
    from workloads import circuits as C

    prog = C.cfg3_program(layers=args.layers)
    uniforms = C.sample_uniforms(prog.meta["samples"], prog.meta["sample_seed"])
    # overlapped compressions: eigensolves on one XCD beside the passes over L on the others
    flags = 0 if args.no_overlap else lr.FLAG_OVERLAP
    dm = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max, flags, device="cuda:0",
                      tuning=None if args.no_tuning else "table")

    for _ in range(args.warmup):
        run_step(dm, prog, uniforms)
    torch.cuda.synchronize()

    # the timed steps carry no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        zz, samples, tr = run_step(dm, prog, uniforms)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per-class kernel times: one further step per class, every launch of that class bracketed
    # by HIP events on the stream it runs on (a flush's back-to-back gate passes by one pair)
    br = {}
    for cls in (() if args.no_breakdown else (0, 1, 2, 3, 4, 5, 6)):
        dm.timing_begin(cls)
        run_step(dm, prog, uniforms)
        n_, m_, t_ = dm.timing_end()
        br[cls] = (n_, m_, t_)
    if args.no_breakdown:   # profiler runs: the kernel times come from the trace instead
        print(json.dumps({"metric": METRIC, "value": args.layers * args.steps / elapsed, "unit": "layers/s",
                          "ms_per_step": 1e3 * elapsed / args.steps, "profiling_run": True}), flush=True)
        return
    # the dominant kernel class: the most time per step
    dominant = max((0, 1, 3, 4, 6), key=lambda c: br[c][2])

    layers = args.layers * args.steps
    ms_per_step = 1e3 * elapsed / args.steps
    ms_per_layer = ms_per_step / args.layers

    def roof(cls, bound, peak):
        nl, mean_ms, _ = br[cls]
        if bound == "hbm":   # a gate pass reads and writes the factor once
            work, unit, scale = 2.0 * 2 ** prog.n * dm.r_pad * 8, "GB/s", 1e9
        else:
            work, unit, scale = algorithmic_flops(prog.n, dm.r_pad, cls), "TFLOP/s", 1e12
        achieved = work / (mean_ms * 1e-3)
        out = {"bound": bound, "kernel": CLASS_NAMES[cls], "achieved": achieved / scale, "peak": peak / scale,
               "unit": unit, "frac": achieved / peak, "traffic": measured_traffic(cls), "launches": nl,
               "mean_ms": mean_ms, "work_per_launch": work}
        mf = measured_mfma(cls)
        if mf is not None:
            out["mfma_counters"] = mf
        return out

    def roof_of(cls):
        if cls == 0:
            return roof(0, "hbm", HBM_PEAK)
        if cls == 3:
            r_ = roof(3, "alu", FP64_PEAK)
            # the eigensolve runs on the serial path, its reduction and eigenvector kernels on one
            # work-group (the multisection uses one per wave, the back-transform 16): its fraction
            # of a single CU's FP64 peak (256 CUs) is the meaningful utilisation figure
            r_["peak_one_cu"] = FP64_PEAK / 256 / 1e12
            r_["frac_one_cu"] = r_["frac"] * 256
            return r_
        return roof(cls, "mfma", FP32_MFMA_PEAK)

    out = {
        "metric": METRIC, "value": layers / elapsed, "unit": "layers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "random brickwork, amplitude damping + dephasing per qubit per layer, "
                               "compress after every channel, <ZZ> + 1e4 samples",
                   "n": prog.n, "r": prog.r, "layers": args.layers, "compressions_per_step": prog.n_compress(),
                   "eigensolve": "f64", "trace_after": tr,
                   "overlap": "eigensolves on one XCD's CUs beside the Gram and projection passes on the other "
                              "seven; split Gram of the next qubit from the 4-way Gram of the bit pair"
                              if flags else "off",
                   "tuning": {"applied": dm.tuning, "in_use": dm.get_tuning(),
                              "source": "paper_2009_06657_amd/tuning_table.json (autotune.py)" if dm.tuning
                              else "library defaults"}},
        "roofline": roof_of(dominant),
        "roofline_projection": roof_of(4),
        "roofline_gram": roof_of(1),
        "roofline_gram_pair": roof_of(6) if br.get(6, (0,))[0] else None,
        "roofline_gate_pass": roof_of(0),
        "roofline_eigensolve": roof_of(3),
        "breakdown_one_step": {CLASS_NAMES[c]: {"launches": br[c][0], "mean_ms": br[c][1], "total_ms": br[c][2]}
                               for c in br},
    }
    out["max_abs_err_vs_oracle"] = error_vs_oracle(dm, prog, zz, samples, flags, uniforms)
    if flags:
        out["without_overlap"] = unflagged_comparator(prog, uniforms, ms_per_step)
    if not args.no_plain:
        out["vs_plain_low_rank"] = plain_comparator(prog, uniforms, ms_per_step)
    if not args.no_grad:
        out["grads_per_s"] = gradient_throughput()
    if not args.no_batch:
        out["batched_serving"] = batched_serving()
    if not args.no_fdm:
        fd = fdm_comparator(fdm_sizes)
        fd["speedup_n20_vs_extrapolated_full_rank"] = fd["full_rank_ms_per_layer_n20_extrapolated"] / ms_per_layer
        out["vs_full_rank_dm"] = fd
    if not args.no_distortion:
        out["distortion"] = fixed_rank_distortion()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prog.n, prog.r)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
