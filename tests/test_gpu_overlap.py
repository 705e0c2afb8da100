"""Overlapped compressions (LRDM_FLAG_OVERLAP) against the FP64 oracle.

With the flag, a channel on qubit q that follows a compression on qubit p != q takes its split
Gram matrix from the 4-way Gram of the bit pair (p, q), formed before the projection on p and
transformed by that projection's W in FP64, and the eigensolves run on a second stream beside
the projections and Gram passes (Sec. II.B: the Gram matrix of the projected factor).  Same
method, different rounding order: probabilities within 1e-5 (complex64) and 1e-10 (complex128)
of the oracle, ranks equal to the unflagged run, over brickwork programs with the channels in
ascending, descending and shuffled qubit order (p < q and p > q), single channels per qubit,
random circuits (channels on the touched qubits only), the smallest sizes (n = 2, r_pad = 8)
and a reset in the middle of a pending compression."""
import sys

import numpy as np
import pytest

import oracle
from workloads import circuits as C

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lr():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2009_06657_amd as lr

    lr.load_library()
    return lr


def _reorder(prog, seed):
    """The same program with each layer's per-qubit channel blocks in a seeded order (seed < 0:
    descending qubit order).  A block is a qubit's channels with their compressions."""
    rng = np.random.default_rng(seed if seed >= 0 else 0)
    out, gates, blocks, cur = [], [], [], None
    for op in prog.ops:
        if isinstance(op, C.Kraus):
            if cur is None or cur[0] != op.qubit:
                cur = (op.qubit, [])
                blocks.append(cur)
            cur[1].append(op)
        elif isinstance(op, C.Compress):
            cur[1].append(op)
        elif isinstance(op, C.LayerEnd):
            order = list(range(len(blocks)))
            if seed < 0:
                order = order[::-1]
            else:
                rng.shuffle(order)
            out += gates
            for i in order:
                out += blocks[i][1]
            out.append(op)
            gates, blocks, cur = [], [], None
        else:
            if blocks:   # gates after channels within a layer: keep the order
                for b in blocks:
                    out += b[1]
                blocks, cur = [], None
            gates.append(op)
    out += gates
    for b in blocks:
        out += b[1]
    return C.Program(prog.n, out, prog.r, prog.dtype, prog.m_max, prog.name, prog.layers, dict(prog.meta))


def _run(lr, prog, flags):
    """Probabilities and ranks; with the flag the program also runs without per-compression
    reports (nothing waits between the streams), which must give the same bits."""
    dm = lr.LowRankDM(prog.n, prog.r, lr.C64 if prog.dtype == "c64" else lr.C128, prog.m_max, flags)
    ranks = []
    for op in prog.ops:
        if isinstance(op, C.Gate):
            dm.apply_gate(op.qubits, op.u)
        elif isinstance(op, C.DiagWeight):
            dm.apply_diagonal_weight(op.phase)
        elif isinstance(op, C.Kraus):
            dm.apply_kraus(op.qubit, op.ops)
        elif isinstance(op, C.Compress):
            ranks.append(dm.compress(op.r, op.eps, op.tie, op.renorm, info=True)["rank"])
    P = dm.probabilities().cpu().numpy()
    if flags:
        dm.reset()
        lr.run_program(dm, prog)
        assert np.array_equal(dm.probabilities().cpu().numpy(), P)
    dm.close()
    return P, ranks


CASES = [("c64", 9, 16, 3, 0), ("c64", 10, 64, 2, 1), ("c64", 8, 32, 3, -1), ("c128", 8, 32, 3, 2),
         ("c128", 7, 8, 3, -1), ("c64", 2, 8, 4, 3), ("c128", 3, 16, 3, 0)]


@pytest.mark.parametrize("dtype,n,r,layers,order", CASES)
def test_overlap_brickwork_against_oracle(lr, dtype, n, r, layers, order):
    prog = C.cfg3_program(n=n, r=r, layers=layers, dtype=dtype)
    if order != 0:
        prog = _reorder(prog, order)
    _say(f"[overlap] {dtype} n={n} r={r} layers={layers} channel order {order}")
    P, k = _run(lr, prog, lr.FLAG_OVERLAP)
    P0, k0 = _run(lr, prog, 0)
    log = []
    Pref = oracle.probabilities(oracle.run_lret(prog, log=log))
    err, err0 = float(np.max(np.abs(P - Pref))), float(np.max(np.abs(P0 - Pref)))
    _say(f"  max|dP| overlap {err:.2e}, unflagged {err0:.2e}, between {np.max(np.abs(P - P0)):.2e}")
    assert k == k0
    assert err <= (1e-5 if dtype == "c64" else 1e-10)


@pytest.mark.parametrize("kind,channel,seed", [("dense-global", "ad", 3), ("sparse-local", "dep", 4),
                                               ("dense-local", "deph", 5)])
def test_overlap_random_circuits(lr, kind, channel, seed):
    """Channels only on the qubits a gate touched (sparse) or on every qubit, one channel per
    qubit and step: every pair (p, q) of consecutive channels appears, and gates interrupt."""
    prog = C.random_circuit(7, 5, kind, channel, p=0.02, r=8, eps=0.0, seed=seed, dtype="c128", tie=1)
    P, k = _run(lr, prog, lr.FLAG_OVERLAP)
    P0, k0 = _run(lr, prog, 0)
    Pref = oracle.probabilities(oracle.run_lret(prog))
    err = float(np.max(np.abs(P - Pref)))
    _say(f"[overlap random] {kind} {channel}: max|dP| {err:.2e} (unflagged {np.max(np.abs(P0 - Pref)):.2e})")
    assert k == k0
    assert err <= 1e-10


def _with_outputs(h, prog):
    """The program with <Z> read after every 17th operation (each read settles the pending
    projection, so the next compression forms its Gram matrix directly)."""
    zs = []
    for i, op in enumerate(prog.ops):
        if isinstance(op, C.Gate):
            h.apply_gate(op.qubits, op.u)
        elif isinstance(op, C.Kraus):
            h.apply_kraus(op.qubit, op.ops)
        elif isinstance(op, C.Compress):
            h.compress(op.r, op.eps, op.tie, op.renorm)
        if i % 17 == 0 and not isinstance(op, C.Kraus):
            zs.append(h.expect_z())
    return zs, h.probabilities().cpu().numpy()


def test_overlap_reset_and_outputs_mid_program(lr):
    """A reset while a compression is pending, then outputs between channels: the unflagged
    results within 1e-5, and the same call sequence again on the reset handle gives the same
    bits."""
    prog = C.cfg3_program(n=8, r=16, layers=2)
    dm = lr.LowRankDM(8, 16, lr.C64, 2, lr.FLAG_OVERLAP)
    ref = lr.LowRankDM(8, 16, lr.C64, 2)
    kr = [op for op in prog.ops if isinstance(op, C.Kraus)]
    for h in (dm, ref):
        h.apply_kraus(kr[0].qubit, kr[0].ops)
        h.compress(16)
        h.apply_kraus(kr[2].qubit, kr[2].ops)   # another qubit: the pair path, left pending
        h.compress(16)
        h.reset()
    zs1, P1 = _with_outputs(dm, prog)
    zs2, P2 = _with_outputs(ref, prog)
    for (z1, _, t1), (z2, _, t2) in zip(zs1, zs2):
        assert np.max(np.abs(z1 - z2)) < 1e-5 and abs(t1 - t2) < 1e-5
    assert np.max(np.abs(P1 - P2)) < 1e-5
    dm.reset()
    zs3, P3 = _with_outputs(dm, prog)
    assert np.array_equal(P3, P1)
    assert all(np.array_equal(a[1], b[1]) for a, b in zip(zs1, zs3))
    dm.close(); ref.close()


@pytest.mark.parametrize("n,blocks", [(6, 0), (7, 0), (8, 3), (9, 5)])
def test_streamed_pair_gram_edges_against_oracle(lr, n, blocks):
    """The streamed 4-way Gram (complex64, r_pad = 64) at its smallest sizes: 16 rows of Y in one
    work-group (n = 6), and work-group counts that leave the last work-group without rows
    (n = 8 with 3 work-groups, n = 9 with 5), against the oracle."""
    prog = C.cfg3_program(n=n, r=64, layers=2)
    dm = lr.LowRankDM(n, 64, lr.C64, prog.m_max, lr.FLAG_OVERLAP)
    if blocks:
        dm.set_tuning(gram4_blocks=blocks)
    _say(f"[stream gram] n={n} r=64 gram4_blocks={blocks or 'default'}")
    lr.run_program(dm, prog)
    P = dm.probabilities().cpu().numpy()
    Pref = oracle.probabilities(oracle.run_lret(prog))
    err = float(np.max(np.abs(P - Pref)))
    _say(f"  max|dP| {err:.2e}")
    assert err <= 1e-5
    dm.close()


@pytest.mark.parametrize("flags", [0, 2])
def test_tuned_launch_shapes_against_oracle(lr, flags):
    """Launch shapes away from the defaults (fewer split-K Gram blocks, a smaller gate tile, fewer
    4-way Gram blocks and a second XCD for the eigensolves): the same oracle parity, and the
    library refuses shapes outside lrdm_tuning's ranges."""
    prog = C.cfg3_program(n=10, r=64, layers=2)
    dm = lr.LowRankDM(10, 64, lr.C64, prog.m_max, flags)
    tun = {"gram_blocks": 5, "gate_local_max": 4}
    if flags:
        tun.update(gram4_blocks=3, aux_cus=64)
    dm.set_tuning(**tun)
    got = dm.get_tuning()
    _say(f"[tuning] flags={flags} in use {got}")
    assert got["gate_local_max"] == 4 and got["gram_blocks"] == 5
    if flags:
        assert got["gram4_blocks"] == 3 and got["aux_cus"] in (0, 64)   # 0: the runtime refused CU masks
    lr.run_program(dm, prog)
    P = dm.probabilities().cpu().numpy()
    Pref = oracle.probabilities(oracle.run_lret(prog))
    err = float(np.max(np.abs(P - Pref)))
    _say(f"  max|dP| {err:.2e}")
    assert err <= 1e-5
    for bad in ({"gram_blocks": 300}, {"gate_local_max": 9}, {"gram4_blocks": 1}, {"aux_cus": 48}):
        with pytest.raises(lr.LrdmError) as e:
            dm.set_tuning(**bad)
        assert e.value.status == 1
    if not flags:
        with pytest.raises(lr.LrdmError):
            dm.set_tuning(aux_cus=64)
    dm.close()
