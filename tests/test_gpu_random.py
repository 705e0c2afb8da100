"""GPU parity on the randomized-benchmarking circuits (Sec. III.A) with the paper's adaptive
truncation threshold (eps = 1e-4, Sec. II.B): probabilities against the oracle's LRET run
(complex64 <= 1e-5, complex128 <= 1e-10) and the kept rank of every compression.  The rank is an
integer that both sides decide in FP64 from their own eigenvalues; it is compared wherever the
oracle's kept mass is not within 1e-12 Tr G of the threshold (there either answer is valid).
These Clifford-rich circuits have exactly degenerate eigenvalues at the cut, so they run with the
cluster policy (tie = 1): the kept set is gap-separated and the truncated state unique."""
import sys

import numpy as np
import pytest

from oracle import lret as OL
from oracle.observables import probabilities
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


def _oracle(prog):
    """The oracle's steps, keeping each compression's rank and whether it sits on the threshold."""
    L = OL.init_state(prog.n)
    ranks, borderline = [], []
    for op in prog.ops:
        if isinstance(op, C.Gate):
            L = OL.apply_gate(L, prog.n, op.qubits, op.u)
        elif isinstance(op, C.Kraus):
            L = OL.kraus_expand(L, prog.n, op.qubit, op.ops)
        elif isinstance(op, C.Compress):
            L, info = OL.compress(L, op.r, op.eps, op.tie, op.renorm)
            lam, tr = info["lam"], info["trace"]
            cum = np.cumsum(np.maximum(lam, 0.0)) - (1.0 - op.eps) * tr
            k = info["k"]
            hit = np.nonzero(cum >= 0)[0]
            k_eps = min(int(hit[0]) + 1 if hit.size else lam.shape[0], op.r)
            near = any(abs(cum[j]) <= 1e-12 * tr for j in range(max(k_eps - 2, 0), min(k_eps + 1, lam.shape[0])))
            if op.tie == 1:   # the cluster rule's own cut: gap against TAU_CLUSTER Tr G
                near = near or any(abs((lam[j - 1] - lam[j]) - OL.TAU_CLUSTER * tr) <= 1e-12 * tr
                                   for j in range(max(k, 1), min(k_eps + 1, lam.shape[0])))
            ranks.append(k)
            borderline.append(bool(near))
    return probabilities(L), ranks, borderline


def _gpu(lr, prog, dt):
    dm = lr.LowRankDM(prog.n, prog.r, dt, prog.m_max)
    ranks = []
    for op in prog.ops:
        if isinstance(op, C.Gate):
            dm.apply_gate(op.qubits, op.u)
        elif isinstance(op, C.Kraus):
            dm.apply_kraus(op.qubit, op.ops)
        elif isinstance(op, C.Compress):
            ranks.append(dm.compress(op.r, op.eps, op.tie, op.renorm, info=True)["rank"])
    P = dm.probabilities().double().cpu().numpy()
    dm.close()
    return P, ranks


@pytest.mark.parametrize("kind", C.CIRCUIT_KINDS)
@pytest.mark.parametrize("channel", ["dep", "bitflip", "ad"])
def test_random_circuit_adaptive_threshold(lr, kind, channel):
    _say(f"random {kind} {channel} eps=1e-4")
    prog = C.random_circuit(7, 6, kind, channel, p=0.002, r=32, eps=1e-4, seed=21, tie=1)
    P_ref, k_ref, near = _oracle(prog)
    P, k = _gpu(lr, prog, lr.C64)
    err = float(np.max(np.abs(P - P_ref)))
    same = [a == b for a, b, x in zip(k, k_ref, near) if not x]
    _say(f"  max|dP| {err:.2e}  ranks {min(k)}..{max(k)}, {len(same)} compared, {sum(near)} on the threshold")
    assert len(k) == len(k_ref)
    assert all(same)
    assert max(k_ref) < 32          # the threshold, not the rank cap, decided every rank
    assert err <= 1e-5


@pytest.mark.parametrize("kind", ["dense-global", "sparse-local"])
def test_random_circuit_adaptive_threshold_complex128(lr, kind):
    _say(f"random {kind} c128 eps=1e-4")
    prog = C.random_circuit(6, 5, kind, "dep", p=0.005, r=32, eps=1e-4, seed=33, dtype="c128", tie=1)
    P_ref, k_ref, near = _oracle(prog)
    P, k = _gpu(lr, prog, lr.C128)
    assert all(a == b for a, b, x in zip(k, k_ref, near) if not x)
    assert float(np.max(np.abs(P - P_ref))) <= 1e-10
