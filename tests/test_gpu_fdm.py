"""GPU parity of the full-rank density-matrix comparator against the FP64 oracle (complex64:
<= 1e-5 absolute on every entry of rho and on Prob)."""
import sys

import numpy as np
import pytest

from oracle import fdm as ofdm
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


def _rand_unitary(rng, k):
    a = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _mixed_program(n, seed, count=60):
    rng = np.random.default_rng(seed)
    chans = [C.depolarizing(0.05), C.amplitude_damping(0.2), C.phase_flip(0.1), C.bit_flip(0.07)]
    ops = []
    for _ in range(count):
        kind = int(rng.integers(0, 6))
        if n == 1:
            kind = (0, 4, 5)[kind % 3]
            q0, q1 = 0, 0
        else:
            q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
        if kind == 0:
            ops.append(C.Gate((q0,), _rand_unitary(rng, 1)))
        elif kind == 1:
            ops.append(C.Gate((q0, q1), C.CNOT))
        elif kind == 2:
            ops.append(C.Gate((q0, q1), C.CZ, diagonal=True))
        elif kind == 3:
            ops.append(C.Gate((q0, q1), _rand_unitary(rng, 2)))
        elif kind == 4:
            ops.append(C.Gate((q0,), C.rz(rng.uniform(-3, 3)), diagonal=True))
        else:
            ops.append(C.Kraus(q0, chans[int(rng.integers(0, 4))]))
    return C.Program(n, ops, 2 ** n, "c64", 4, "mixed", 1)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8])
def test_fdm_mixed_program(lr, n):
    _say(f"fdm mixed n={n}")
    prog = _mixed_program(n, 10 + n)
    ref = ofdm.run_fdm(prog)
    f = lr.FullRankDM(n)
    lr.run_program_fdm(f, prog)
    rho = f.rho()
    err = np.max(np.abs(rho - ref))
    _say(f"  max |d rho| {err:.2e}")
    assert err <= 1e-5
    p = f.probabilities().cpu().numpy()
    assert np.max(np.abs(p - np.real(np.diag(ref)))) <= 1e-5


def test_fdm_brickwork_layers_and_invariants(lr):
    """The brickwork layer structure (SU(2) + CZ, amplitude damping + dephasing per qubit) at
    n = 9: rho matches the oracle, is Hermitian with unit trace."""
    _say("fdm brickwork n=9")
    prog = C.cfg3_program(n=9, r=512, layers=3)
    ref = ofdm.run_fdm(prog)
    f = lr.FullRankDM(9)
    lr.run_program_fdm(f, prog)
    rho = f.rho()
    assert np.max(np.abs(rho - ref)) <= 1e-5
    assert abs(np.trace(rho).real - 1) <= 1e-5
    assert np.max(np.abs(rho - rho.conj().T)) <= 1e-6


def test_fdm_equals_full_rank_lret(lr):
    """r >= 2^n: the low-rank path keeps everything and both GPU paths agree."""
    _say("fdm vs lret n=5")
    prog = C.cfg1_program(n=5, r=32, layers=3, dtype="c64")
    f = lr.FullRankDM(5)
    lr.run_program_fdm(f, prog)
    dm = lr.LowRankDM(5, 32, lr.C64, 4)
    lr.run_program(dm, prog)
    p_f = f.probabilities().cpu().numpy()
    p_l = dm.probabilities().cpu().numpy()
    assert np.max(np.abs(p_f - p_l)) <= 2e-5


def test_fdm_errors(lr):
    f = lr.FullRankDM(3)
    with pytest.raises(lr.LrdmError):
        f.apply_gate((0,), np.array([[1, 1], [0, 1]]))
    with pytest.raises(lr.LrdmError):
        f.apply_kraus(0, np.array([[[1, 0], [0, 0.5]]]))
    with pytest.raises(lr.LrdmError):
        f.apply_gate((3,), C.H)
