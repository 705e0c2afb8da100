"""The program-level entry points (include/lrdm.h): lrdm_run (Algorithm 1 over a flat operation
array, with per-layer checkpoints), lrdm_energy_grad (forward pass and reverse sweep in one
call) and lrdm_batch_run (record, capture and replay a whole batch in one call), called through
ctypes and compared with the operation-level path and the oracle."""
import ctypes
import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import grad as OG
from workloads import circuits as C

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg4_grad.json")


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


def test_run_equals_operation_calls_and_checkpoints_resume(lr):
    import torch

    prog = C.cfg3_program(n=11, r=32, layers=3)
    _say("[lrdm_run] brickwork n=11 r=32 3 layers")
    a = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max)
    lr.run_program(a, prog)
    La = a.get_L()
    b = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max)
    fp = lr.lrdm.FlatProgram(prog)
    S = (b.state.numel() + 255) // 256 * 256
    ckpt = torch.empty(fp.n_layers * S, dtype=torch.uint8, device=b.device)
    ranks = b.run(fp, ckpt)
    assert np.array_equal(b.get_L(), La)
    assert ranks[0] == 1 and len(ranks) == 3
    # resume from the checkpoint of layer 1: run layers 1 and 2 again
    c = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max)
    c.restore(ckpt[S: S + b.state.numel()], ranks[1])
    layer_ops = []
    cur = []
    for op in prog.ops:
        cur.append(op)
        if isinstance(op, C.LayerEnd):
            layer_ops.append(cur)
            cur = []
    rest = C.Program(prog.n, layer_ops[1] + layer_ops[2], prog.r, prog.dtype, prog.m_max)
    c.run(rest)
    assert np.array_equal(c.get_L(), La)
    # an invalid program enqueues nothing: the state is unchanged
    bad = C.Program(prog.n, [C.Gate((0,), C.H), C.Gate((1,), np.array([[1, 1], [0, 1]]))], prog.r)
    with pytest.raises(lr.LrdmError) as e:
        c.run(bad)
    assert e.value.status == 1
    assert np.array_equal(c.get_L(), La)
    for h in (a, b, c):
        h.close()


def test_run_with_overlap_equals_operation_calls(lr):
    """lrdm_run on an LRDM_FLAG_OVERLAP handle issues the same launches as the operation calls on
    one (the same bits), with per-layer checkpoints taken between the streams' work."""
    import torch

    prog = C.cfg3_program(n=10, r=32, layers=3)
    a = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max, lr.FLAG_OVERLAP)
    lr.run_program(a, prog)
    La = a.get_L()
    b = lr.LowRankDM(prog.n, prog.r, lr.C64, prog.m_max, lr.FLAG_OVERLAP)
    fp = lr.lrdm.FlatProgram(prog)
    S = (b.state.numel() + 255) // 256 * 256
    ckpt = torch.empty(fp.n_layers * S, dtype=torch.uint8, device=b.device)
    b.run(fp, ckpt)
    assert np.array_equal(b.get_L(), La)
    Pref = oracle.probabilities(oracle.run_lret(prog))
    assert float(np.max(np.abs(b.probabilities().cpu().numpy() - Pref))) <= 1e-5
    a.close(); b.close()


def test_energy_grad_direct_call_matches_finite_differences(lr):
    """n = 12, r = 16 noisy ansatz (192 angles, 200 Pauli terms), complex64: lrdm_energy_grad
    called through ctypes, energy and gradient against the oracle's central differences."""
    import torch

    with open(GOLDEN) as f:
        gold = json.load(f)
    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    prog = C.cfg4_program(theta)
    _say("[lrdm_energy_grad] n=12 r=16, 8 layers, direct call")
    lib = lr.load_library()
    h = lr.LowRankDM(12, 16, lr.C64, 4)
    bar = lr.LowRankDM(12, 16, lr.C64, 4)
    fp = lr.lrdm.FlatProgram(prog)
    keep_b, min_b = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lrdm_energy_grad_bytes(h.h, fp.ref, ctypes.byref(keep_b), ctypes.byref(min_b)) == 0
    assert min_b.value < keep_b.value
    for nbytes in (keep_b.value, min_b.value):
        store = torch.empty(nbytes, dtype=torch.uint8, device=h.device)
        E = np.zeros(1)
        g = np.zeros(theta.size)
        kept = ctypes.c_int()
        xa, za, ca = (np.ascontiguousarray(a) for a in (xm, zm, co))
        st = lib.lrdm_energy_grad(h.h, bar.h, fp.ref, None, theta.size, len(xm), xa.ctypes.data, za.ctypes.data,
                                  ca.ctypes.data, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(store.data_ptr()),
                                  nbytes, ctypes.byref(kept))
        assert st == 0, lib.lrdm_last_error(None)
        assert kept.value == (1 if nbytes == keep_b.value else 0)
        err_e = abs(E[0] - gold["energy"])
        err_g = float(np.max(np.abs(g - np.array(gold["grad_fd"]))))
        _say(f"  store {nbytes >> 20} MiB (keep all: {kept.value}): |dE| {err_e:.2e}  max|dg| vs FD {err_g:.2e}")
        assert err_e <= 1e-5 and err_g <= 1e-4
        if nbytes == keep_b.value:
            g_keep, E_keep = g.copy(), E[0]
        else:
            assert E[0] == E_keep and np.array_equal(g, g_keep)
    # too small a store is refused before anything runs
    st = lib.lrdm_energy_grad(h.h, bar.h, fp.ref, None, theta.size, len(xm), xa.ctypes.data, za.ctypes.data,
                              ca.ctypes.data, E.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(store.data_ptr()),
                              min_b.value - 256, None)
    assert st == 2
    h.close(); bar.close()


def test_autograd_two_forwards_before_backward(lr):
    """Each autograd node differentiates its own forward: E(theta_1) + 3 E(theta_2) on one engine."""
    import torch

    from paper_2009_06657_amd.adjoint import EnergyGradient, make_noisy_energy

    n, r, layers = 5, 4, 2
    rng = np.random.default_rng(31)
    t1 = rng.uniform(-np.pi, np.pi, size=(layers, n, 2))
    t2 = rng.uniform(-np.pi, np.pi, size=(layers, n, 2))
    xm, zm, co, _ = C.random_pauli_sum(n, terms=20, max_weight=3, seed=31)
    make = lambda t: C.cfg4_program(t, n=n, r=r, p=0.02, dtype="c128")  # noqa: E731
    eng = EnergyGradient(n, r, 4, xm, zm, co, dtype=lr.C128)
    NoisyEnergy = make_noisy_energy()
    a = torch.tensor(t1, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(t2, dtype=torch.float64, requires_grad=True)
    loss = NoisyEnergy.apply(a, eng, make) + 3.0 * NoisyEnergy.apply(b, eng, make)
    loss.backward()
    _, g1 = OG.energy_grad_adjoint(make(t1), t1.size, xm, zm, co)
    _, g2 = OG.energy_grad_adjoint(make(t2), t2.size, xm, zm, co)
    np.testing.assert_allclose(a.grad.numpy().reshape(-1), g1, atol=1e-9)
    np.testing.assert_allclose(b.grad.numpy().reshape(-1), 3.0 * g2, atol=3e-9)
    eng.close()


def test_batch_run_equals_recorded_batch(lr):
    progs = [C.brickwork_program(n, 3, r, [("dep", 0.003)], seed=70 + i)
             for i, (n, r) in enumerate([(6, 8), (8, 16), (7, 32), (9, 8)])]
    _say("[lrdm_batch_run] 4 instances")
    ha = [lr.LowRankDM(p.n, p.r, lr.C64, p.m_max) for p in progs]
    ba = lr.Batch(ha)
    with ba.recording():
        for dm, p in zip(ha, progs):
            dm.reset()
            lr.run_program(dm, p)
    ba.launch()
    ba.times()
    hb = [lr.LowRankDM(p.n, p.r, lr.C64, p.m_max) for p in progs]
    bb = lr.Batch(hb)
    done, total = bb.run(progs)
    assert total > 0 and np.all(done > 0)
    for x, y in zip(ha, hb):
        x.synchronize(); y.synchronize()
        assert np.array_equal(x.get_L(), y.get_L())
    bb.launch()            # a second replay of the graph lrdm_batch_run captured
    done2, _ = bb.times()
    for x, y in zip(ha, hb):
        y.synchronize()
        assert np.array_equal(x.get_L(), y.get_L())
    ba.close(); bb.close()
    for h in ha + hb:
        h.close()
