"""Writes cfg5_instances.json: <Z_i>, the trace and the per-compression kept ranks of eight
instances of the serving mix (256 brickwork instances, n ~ U{8..16}, r ~ U{8,16,32}, depth
~ U{10..30}, depolarizing p ~ U(1e-4, 5e-3), a compression after every channel, seeds 5000 + i),
from the FP64 oracle only, both with the eigensolver-order cut of the mix (tie = 0) and with the
gap-separated cut (tie = 1).  The chosen instances cover the largest shapes of the mix (n = 16 at
r = 8, 16 and 32) and a few smaller ones.

Conditioning: each run is repeated twice with a seeded relative perturbation of 1e-7 (the
rounding of a complex64 factor) added to every entry of the factor before each compression; the
largest change of <Z_i> over the two is stored as z_spread.  A cut between nearly equal
eigenvalues turns the kept subspace by about perturbation / gap, so a large spread marks an
instance whose complex64 result is not determined to the 1e-5 bar by its input.

    python tests/golden/make_cfg5_golden.py
"""
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.lret import compress, init_state, kraus_expand  # noqa: E402
from workloads import circuits as C  # noqa: E402

INSTANCES = (32, 63, 15, 96, 52, 102, 41, 0)
ETA = 1e-7


def run(prog, perturb=0.0, pseed=0):
    """The oracle's steps (Algorithm 1); with perturb > 0, a seeded relative perturbation of that
    size on every entry of the factor before each compression.  Returns (Prob, log)."""
    rng = np.random.default_rng(pseed)
    n = prog.n
    L = init_state(n)
    log = []
    for op in prog.ops:
        if isinstance(op, C.Gate):
            L = oracle.apply_gate(L, n, op.qubits, op.u)
        elif isinstance(op, C.Kraus):
            L = kraus_expand(L, n, op.qubit, op.ops)
            if perturb > 0:
                g = rng.standard_normal(L.shape) + 1j * rng.standard_normal(L.shape)
                L = L + perturb * np.abs(L) * g / np.sqrt(2.0)
        elif isinstance(op, C.Compress):
            L, info = compress(L, op.r, op.eps, op.tie, op.renorm)
            info.pop("lam")
            log.append(info)
    return oracle.probabilities(L), log


def results(prog):
    P, log = run(prog)
    z = oracle.expect_z(P, prog.n)
    spread = 0.0
    for ps in (1, 2):
        Pp, _ = run(prog, ETA, ps)
        spread = max(spread, float(np.max(np.abs(oracle.expect_z(Pp, prog.n) - z))))
    return {"z": z.tolist(), "trace": float(P.sum()), "z_spread": spread,
            "ranks": [int(e["k"]) for e in log],
            "discarded_total": float(sum(e["discarded"] for e in log)),
            "min_gap": float(min((e["gap"] / e["trace"] for e in log
                                  if np.isfinite(e["gap"]) and e["lam_k"] > 1e-12 * e["trace"]), default=1.0))}


def main():
    progs = C.cfg5_instances(256)
    out = {"workload": "serving mix: 256 brickwork instances (seeds 5000 + i), depolarizing, compress after "
                       "every channel; oracle <Z_i> of the listed instances", "eta": ETA, "instances": []}
    for i in INSTANCES:
        p = progs[i]
        t0 = time.perf_counter()
        p1 = copy.deepcopy(p)
        for op in p1.ops:
            if isinstance(op, C.Compress):
                op.tie = 1
        out["instances"].append({"index": i, "n": p.n, "r": p.r, "layers": p.layers,
                                 "tie0": results(p), "tie1": results(p1)})
        e = out["instances"][-1]
        print(f"instance {i}: n={p.n} r={p.r} layers={p.layers} spread {e['tie0']['z_spread']:.1e} / "
              f"{e['tie1']['z_spread']:.1e} ({time.perf_counter() - t0:.1f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg5_instances.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
