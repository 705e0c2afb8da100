"""Autotuner of liblrdm's launch shapes (lrdm_tuning, include/lrdm.h) per workload.

A coordinate search: for one field at a time, every candidate value is timed on whole layers of
the workload on the GPU (the minimum over a few repetitions of reset -> layers -> synchronise),
and the fastest value is kept when it beats the current choice by more than the timing noise.
The winners go to a JSON table keyed by the workload's shape (n, r, precision, stream mode), which
`load`/`apply` read back, so a handle of that shape starts with the tuned launch shapes
(LowRankDM(..., tuning="table")).

    python -m paper_2009_06657_amd.autotune --n 20 --r 64 --layers 2 --overlap --write

The fields change only how work-groups split the rows (split-K Gram blocks, 4-way Gram blocks,
local qubits of a gate pass, CUs of the eigensolver stream), never the operations, so results
differ from the defaults only by rounding order.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "tuning_table.json")

# candidate values per field (0 = the library's default); aux_cus in whole XCDs
CANDIDATES = {
    "gram_blocks": [0, 128, 160, 192, 224, 256],
    "gram4_blocks": [0, 96, 128, 160, 192, 224, 256],
    "gate_local_max": [0, 5, 6, 7],
    "aux_cus": [0, 64],
}
OVERLAP_ONLY = ("gram4_blocks", "aux_cus")
NOISE = 0.01   # a candidate must beat the current choice by more than this fraction


def key(n: int, r: int, dtype: str, overlap: bool) -> str:
    return f"n{n}_r{r}_{dtype}_{'overlap' if overlap else 'single'}"


def search(time_with, fields=None, overlap=True, noise=NOISE, log=None):
    """Coordinate search.  time_with(tuning: dict) -> seconds (raises ValueError for a value the
    library rejects).  Returns (best tuning, best time, default time, every measurement)."""
    fields = fields or CANDIDATES
    best: dict = {}
    t_default = time_with({})
    t_best = t_default
    seen = {json.dumps({}, sort_keys=True): t_default}
    for field, cands in fields.items():
        if field in OVERLAP_ONLY and not overlap:
            continue
        for v in cands:
            trial = dict(best)
            if v:
                trial[field] = v
            else:
                trial.pop(field, None)
            tag = json.dumps(trial, sort_keys=True)
            if tag in seen:
                continue
            try:
                t = time_with(trial)
            except ValueError:
                continue
            seen[tag] = t
            if log:
                log(f"  {field}={v}: {t * 1e3:.2f} ms")
            if t < t_best * (1.0 - noise):
                best, t_best = trial, t
    return best, t_best, t_default, seen


def _time_layers(dm, prog, reps: int) -> float:
    import paper_2009_06657_amd as lr

    best = float("inf")
    for _ in range(reps):
        dm.reset()
        dm.synchronize()
        t0 = time.perf_counter()
        lr.run_program(dm, prog)
        dm.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune_workload(prog, overlap: bool, reps: int = 3, log=print) -> dict:
    """Tune the launch shapes for one workload (a workloads.circuits.Program); returns the table
    entry."""
    import paper_2009_06657_amd as lr

    dt = lr.C64 if prog.dtype == "c64" else lr.C128
    dm = lr.LowRankDM(prog.n, prog.r, dt, prog.m_max, lr.FLAG_OVERLAP if overlap else 0)
    lr.run_program(dm, prog)   # warm-up (first launches, device code loads)
    dm.synchronize()

    def time_with(tuning: dict) -> float:
        try:
            dm.set_tuning(**tuning)
        except lr.LrdmError as e:
            if e.status == 1:   # LRDM_E_ARG: a value outside what this device or mode takes
                raise ValueError(str(e))
            raise
        return _time_layers(dm, prog, reps)

    best, t_best, t_def, seen = search(time_with, overlap=overlap, log=log)
    dm.set_tuning(**best)
    resolved = dm.get_tuning()
    dm.close()
    return {"tuning": best, "resolved": resolved, "layers": prog.layers,
            "ms_per_layer": 1e3 * t_best / prog.layers, "default_ms_per_layer": 1e3 * t_def / prog.layers,
            "measured": {k: 1e3 * v / prog.layers for k, v in seen.items()}}


def load(n: int, r: int, dtype: str, overlap: bool, path: str = TABLE):
    """The tuned lrdm_tuning fields for this shape, or None."""
    try:
        with open(path) as f:
            table = json.load(f)
    except OSError:
        return None
    e = table.get("entries", {}).get(key(n, r, dtype, overlap))
    return dict(e["tuning"]) if e else None


def apply(dm, path: str = TABLE) -> dict | None:
    """Set the table's tuning on a LowRankDM of a tuned shape; returns what was applied."""
    import paper_2009_06657_amd as lr

    t = load(dm.n, dm.r_max, "c64" if dm.dtype == lr.C64 else "c128", bool(dm.flags & lr.FLAG_OVERLAP), path)
    if t:
        dm.set_tuning(**t)
    return t


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=20)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--layers", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--overlap", action="store_true")
    ap.add_argument("--write", action="store_true", help="merge the result into the table")
    ap.add_argument("--table", default=TABLE, help="the table to merge into (default: the package's)")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(PKG))
    import torch  # noqa: F401  (the HIP runtime the library binds to)
    from workloads import circuits as C

    prog = C.cfg3_program(n=args.n, r=args.r, layers=args.layers)
    k = key(args.n, args.r, prog.dtype, args.overlap)
    print(f"tuning {k} on {args.layers} brickwork layers", flush=True)
    entry = tune_workload(prog, args.overlap, args.reps, log=lambda s: print(s, flush=True))
    entry["workload"] = f"random brickwork, amplitude damping + dephasing, {args.layers} layers"
    print(json.dumps({k: entry}), flush=True)
    if args.write:
        try:
            with open(args.table) as f:
                table = json.load(f)
        except OSError:
            table = {"about": "lrdm_tuning per workload shape, written by paper_2009_06657_amd/autotune.py",
                     "entries": {}}
        table["entries"][k] = entry
        with open(args.table, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
