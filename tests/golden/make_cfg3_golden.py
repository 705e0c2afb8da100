"""Writes the oracle's outputs for the random brickwork benchmark circuit (n = 20, r = 64,
Haar SU(2) on every qubit + alternating CZ pairs, amplitude damping 0.002 -> compress ->
dephasing 0.001 -> compress per qubit per layer, seed 1003), from the FP64 oracle only.

For every layer: <Z_i>, <Z_i Z_{i+1}>, the trace and the running discarded mass.  For every
compression: the kept rank, the discarded mass, Tr G, the boundary gap and the smallest kept
eigenvalue.  At each snapshot
layer (default 4 and 40) one JSON file cfg3_n20_r64_l<L>.json with all of the above up to that
layer plus
  * Prob(x) at 8192 fixed indices: the 4096 largest and 4096 others drawn uniformly (seed 3103);
  * the inverse-CDF samples for the 10^4 uniforms of seed 3003 and, for each, the distance of
    u * CDF(last) to the nearer end of its CDF step, relative to CDF(last) (a sample may only
    differ where that margin is within the rounding of the running sums).

    python tests/golden/make_cfg3_golden.py [--layers 40] [--snapshots 4,40] [--state-dir DIR]

The 4-layer file takes about 20 minutes on 8 cores, the 40-layer one a few hours; --state-dir
keeps the factor after every layer so that an interrupted run resumes there.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.lret import apply_diag_weight, compress, init_state, kraus_expand  # noqa: E402
from workloads import circuits as C  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_LARGEST = 4096
N_RANDOM = 4096
INDEX_SEED = 3103


def fixed_indices(P):
    order = np.argsort(-P, kind="stable")
    top = np.sort(order[:N_LARGEST])
    rest = np.setdiff1d(np.arange(P.shape[0]), top)
    rnd = np.random.Generator(np.random.PCG64(INDEX_SEED)).choice(rest, size=N_RANDOM, replace=False)
    return np.sort(top), np.sort(rnd)


def sample_margins(P, u, x):
    cdf = np.cumsum(P)
    tot = cdf[-1]
    t = u * tot
    lo = np.where(x > 0, cdf[np.maximum(x.astype(np.int64) - 1, 0)], 0.0)
    hi = cdf[x.astype(np.int64)]
    return np.minimum(t - lo, hi - t) / tot


def snapshot(path, prog, L, per_layer, per_comp, layers_done, seconds):
    n = prog.n
    P = oracle.probabilities(L)
    top, rnd = fixed_indices(P)
    u = C.sample_uniforms(prog.meta["samples"], prog.meta["sample_seed"])
    x = oracle.sample_inverse_cdf(P, u)
    out = {"workload": "random brickwork n=20 r=64, amplitude damping 0.002 -> compress -> dephasing 0.001 "
                       "-> compress per qubit per layer, seed 1003 (oracle, complex128)",
           "n": n, "r": prog.r, "layers": layers_done, "seed": 1003, "sample_seed": prog.meta["sample_seed"],
           "oracle_seconds": seconds,
           "per_layer": per_layer, "per_compression": per_comp,
           "z": oracle.expect_z(P, n).tolist(), "zz": oracle.expect_zz(P, n).tolist(),
           "trace": float(P.sum()),
           "prob_largest_idx": top.tolist(), "prob_largest": P[top].tolist(),
           "prob_random_idx": rnd.tolist(), "prob_random": P[rnd].tolist(), "index_seed": INDEX_SEED,
           "samples": [int(v) for v in x], "sample_margin": sample_margins(P, u, x).tolist()}
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--snapshots", type=str, default="4,40")
    ap.add_argument("--state-dir", type=str, default="")
    a = ap.parse_args()
    snaps = {int(s) for s in a.snapshots.split(",") if s}
    prog = C.cfg3_program(layers=a.layers)
    n = prog.n
    layers = [[]]
    for op in prog.ops:
        if isinstance(op, C.LayerEnd):
            layers.append([])
        else:
            layers[-1].append(op)
    layers = [seg for seg in layers if seg]
    L = init_state(n)
    per_layer, per_comp = [], []
    start = 0
    acc = 0.0
    t_prev = 0.0
    sfile = os.path.join(a.state_dir, "cfg3_state.npz") if a.state_dir else ""
    if sfile and os.path.exists(sfile):
        d = np.load(sfile, allow_pickle=False)
        L = d["L"]
        meta = json.loads(str(d["meta"]))
        start, per_layer, per_comp, acc, t_prev = meta["layers"], meta["per_layer"], meta["per_comp"], meta["acc"], meta["seconds"]
        print(f"resumed after layer {start}", flush=True)
    t0 = time.perf_counter() - t_prev
    for l in range(start, a.layers):
        for op in layers[l]:
            if isinstance(op, C.Gate):
                L = oracle.apply_gate(L, n, op.qubits, op.u)
            elif isinstance(op, C.DiagWeight):
                L = apply_diag_weight(L, n, op.phase)
            elif isinstance(op, C.Kraus):
                L = kraus_expand(L, n, op.qubit, op.ops)
            elif isinstance(op, C.Compress):
                L, info = compress(L, op.r, op.eps, op.tie, op.renorm)
                acc += info["discarded"]
                per_comp.append({"k": int(info["k"]), "discarded": info["discarded"], "trace": info["trace"],
                                 "gap": info["gap"] if np.isfinite(info["gap"]) else None,
                                 "lam_k": info["lam_k"]})
        P = oracle.probabilities(L)
        per_layer.append({"z": oracle.expect_z(P, n).tolist(), "zz": oracle.expect_zz(P, n).tolist(),
                          "trace": float(P.sum()), "discarded_total": acc})
        el = time.perf_counter() - t0
        print(f"layer {l + 1}/{a.layers} done ({el:.0f} s, rank {L.shape[1]})", flush=True)
        if l + 1 in snaps:
            snapshot(os.path.join(HERE, f"cfg3_n20_r64_l{l + 1}.json"), prog, L, per_layer, per_comp, l + 1, el)
        if sfile:
            meta = {"layers": l + 1, "per_layer": per_layer, "per_comp": per_comp, "acc": acc, "seconds": el}
            tmp = sfile + ".tmp.npz"
            np.savez(tmp, L=L, meta=np.array(json.dumps(meta)))
            os.replace(tmp, sfile)


if __name__ == "__main__":
    main()
