"""GPU parity of the full-rank density-matrix comparator against the FP64 oracle (complex64:
<= 1e-5 absolute on every entry of rho and on Prob)."""
import sys

import numpy as np
import pytest

from fdm_programs import mixed_program as _mixed_program
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


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8, 10])
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


@pytest.mark.parametrize("n", [1, 4, 7])
def test_fdm_hamming_weight_phase(lr, n):
    """Hamming-weight phases on both sides of rho: noisy Grover (real phases, Sec. III.C) and
    random complex unit-modulus phases between queued gates and channels."""
    _say(f"fdm hamming-weight phase n={n}")
    rng = np.random.default_rng(70 + n)
    ops = []
    for t in range(3):
        ops += [C.Gate((q,), C.haar_su2(rng)) for q in range(n)]
        ops.append(C.DiagWeight(np.exp(1j * rng.uniform(0, 2 * np.pi, n + 1))))
        ops += [C.Kraus(q, C.depolarizing(0.01)) for q in range(n)]
        if n > 1:
            ops.append(C.Gate((0, n - 1), C.CNOT))
    progs = [C.Program(n, ops, 8)]
    if n >= 4:
        progs.append(C.cfg2_program(n=n, r=16, iterations=2, p=0.003))
    for prog in progs:
        ref = ofdm.run_fdm(prog)
        f = lr.FullRankDM(n)
        lr.run_program_fdm(f, prog)
        rho = f.rho()
        err = np.max(np.abs(rho - ref))
        _say(f"  {prog.name or 'random phases'}: max |d rho| {err:.2e}")
        assert err <= 1e-5
        f.close()


def test_fdm_errors(lr):
    f = lr.FullRankDM(3)
    with pytest.raises(lr.LrdmError):
        f.apply_diagonal_weight(np.array([1, 1, 1, 1.5]))
    with pytest.raises(lr.LrdmError):
        f.apply_gate((0,), np.array([[1, 1], [0, 1]]))
    with pytest.raises(lr.LrdmError):
        f.apply_kraus(0, np.array([[[1, 0], [0, 0.5]]]))
    with pytest.raises(lr.LrdmError):
        f.apply_gate((3,), C.H)
