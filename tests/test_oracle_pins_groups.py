"""Pins of the oracle's two-qubit channels and channel groups (Sec. II.C: noise as one- and
two-qubit Kraus operators, a Kraus layer split into groups of M qubits with one truncation per
group), its sparse initial states (Sec. II.D) and its switch to full density matrix evolution
(Sec. II.C, last paragraph), each against something other than the oracle's own formula:
Kronecker brute force, closed forms, exact identities of channel composition, the statevector
and the full-rank evolution."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import fdm as ofdm
from oracle.lret import compress, init_sparse, intermediate_rank, kraus_expand, run_lret_switching
from workloads import circuits as C


def full_matrix(n, qubits, U):
    """Brute-force 2^n x 2^n matrix of a k-qubit U on `qubits` (local index sum_j b(q_j) 2^j)."""
    d = 2 ** n
    k = len(qubits)
    M = np.zeros((d, d), dtype=np.complex128)
    for x in range(d):
        li = sum(((x >> q) & 1) << j for j, q in enumerate(qubits))
        for lo in range(2 ** k):
            y = x
            for j, q in enumerate(qubits):
                y = (y & ~(1 << q)) | (((lo >> j) & 1) << q)
            M[y, x] += U[lo, li]
    return M


def rand_L(rng, n, V):
    L = rng.standard_normal((2 ** n, V)) + 1j * rng.standard_normal((2 ** n, V))
    return L / np.linalg.norm(L)


TWO = {"dep2": C.depolarizing2(0.03), "zz": C.correlated_dephasing(0.05),
       "ad x deph": C.grouped_channel(C.amplitude_damping(0.04), C.phase_flip(0.02)),
       "dep x dep": C.grouped_channel(C.depolarizing(0.02), C.depolarizing(0.01))}


@pytest.mark.parametrize("name", list(TWO))
def test_two_qubit_channel_completeness_and_superoperator(name):
    ops = TWO[name]
    np.testing.assert_allclose(sum(E.conj().T @ E for E in ops), np.eye(4), atol=1e-15)
    rng = np.random.default_rng(11)
    n, q0, q1 = 4, 3, 1
    L = rand_L(rng, n, 3)
    rho = L @ L.conj().T
    ref = sum(full_matrix(n, (q0, q1), E) @ rho @ full_matrix(n, (q0, q1), E).conj().T for E in ops)
    Lp = kraus_expand(L, n, q0, ops, q1)
    assert Lp.shape == (2 ** n, 3 * len(ops))
    np.testing.assert_allclose(Lp @ Lp.conj().T, ref, atol=1e-14)
    np.testing.assert_allclose(ofdm.fdm_channel(rho, n, q0, ops, q1), ref, atol=1e-14)


def test_grouped_channel_equals_the_two_channels_in_turn():
    """A product channel on (q0, q1) is the two one-qubit channels applied one after the other
    (exactly, without truncation in between)."""
    rng = np.random.default_rng(12)
    n = 5
    rho = rand_L(rng, n, 4)
    rho = rho @ rho.conj().T
    A, B = C.amplitude_damping(0.07), C.depolarizing(0.05)
    seq = ofdm.fdm_channel(ofdm.fdm_channel(rho, n, 2, A), n, 4, B)
    grp = ofdm.fdm_channel(rho, n, 2, C.grouped_channel(A, B), 4)
    np.testing.assert_allclose(grp, seq, atol=1e-15)


def test_two_qubit_depolarizing_closed_form():
    """(1-p) rho + p/15 sum_{P != II} P rho P scales every non-identity two-qubit Pauli
    expectation by 1 - 16 p / 15 and keeps the trace."""
    rng = np.random.default_rng(13)
    n, p = 2, 0.09
    L = rand_L(rng, n, 2)
    rho = L @ L.conj().T
    Lp = kraus_expand(L, n, 0, C.depolarizing2(p), 1)
    out = Lp @ Lp.conj().T
    for a, b in itertools.product(range(4), repeat=2):
        P = np.kron(C.PAULI_LIST[b], C.PAULI_LIST[a])
        before, after = np.trace(P @ rho).real, np.trace(P @ out).real
        scale = 1.0 if (a, b) == (0, 0) else 1 - 16 * p / 15
        assert abs(after - scale * before) < 1e-14


def test_grouped_program_equals_fdm_when_rank_suffices():
    prog = C.grouped_brickwork_program(4, 3, 64, "dep", 0.03, seed=14, dtype="c128")
    L = oracle.run_lret(prog)
    np.testing.assert_allclose(L @ L.conj().T, ofdm.run_fdm(prog), atol=1e-12)
    prog = C.grouped_brickwork_program(5, 2, 64, "ad", 0.05, seed=15, two_qubit="zz", dtype="c128")
    L = oracle.run_lret(prog)
    np.testing.assert_allclose(L @ L.conj().T, ofdm.run_fdm(prog), atol=1e-12)


def test_grouped_truncation_error_identity():
    """Eckart-Young on a grouped truncation: ||rho' - rho~||_F^2 = sum of the squared discarded
    eigenvalues, with rho' the exact two-qubit channel image (brute force)."""
    rng = np.random.default_rng(16)
    n = 5
    L = rand_L(rng, n, 4)
    ops = C.grouped_channel(C.depolarizing(0.05), C.amplitude_damping(0.1))
    Lp = kraus_expand(L, n, 1, ops, 3)
    rho_p = sum(full_matrix(n, (1, 3), E) @ (L @ L.conj().T) @ full_matrix(n, (1, 3), E).conj().T for E in ops)
    Ln, info = compress(Lp, 6, renorm=0)
    lam = np.sort(np.linalg.eigvalsh(rho_p))[::-1]
    assert abs(np.linalg.norm(rho_p - Ln @ Ln.conj().T) ** 2 - np.sum(lam[6:] ** 2)) < 1e-14


def test_sparse_initial_state():
    n = 6
    idx, amp = C.ghz_init(n)
    L = init_sparse(n, idx, amp)
    P = oracle.probabilities(L)
    assert P[0] == pytest.approx(0.5) and P[-1] == pytest.approx(0.5) and abs(P.sum() - 1) < 1e-15
    np.testing.assert_allclose(oracle.expect_zz(P, n), np.ones(n - 1), atol=1e-15)
    xall = (1 << n) - 1
    assert abs(oracle.expect_pauli(L, n, xall, 0) - 1.0) < 1e-15       # <X...X> = 1 on GHZ
    # noiseless evolution from a sparse state equals the statevector from the same state
    rng = np.random.default_rng(17)
    idx = np.array([3, 17, 40, 63], dtype=np.uint64)
    amp = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    amp /= np.linalg.norm(amp)
    prog = C.cfg1_program(n=n, r=8, layers=3, p=0.0)
    prog.ops = [op for op in prog.ops if isinstance(op, C.Gate)]
    prog.init = (idx, amp)
    psi = ofdm.run_sv(prog)
    L = oracle.run_lret(prog)
    np.testing.assert_allclose(L[:, 0], psi, atol=1e-14)
    # and with noise, LRET (no truncation) equals the exact evolution from that state
    prog = C.cfg1_program(n=5, r=32, layers=3, p=0.02)
    prog.init = (np.array([1, 30], dtype=np.uint64), np.array([0.6, 0.8j]))
    L = oracle.run_lret(prog)
    np.testing.assert_allclose(L @ L.conj().T, ofdm.run_fdm(prog), atol=1e-12)


def test_intermediate_rank_rule():
    # V_I^3 = N (A V)^3 / M
    assert intermediate_rank(8, 4, 10, 1) == pytest.approx((8 * 40 ** 3) ** (1 / 3))
    assert intermediate_rank(6, 16, 2, 2) == pytest.approx((3 * 32 ** 3) ** (1 / 3))


def test_switch_to_full_rank_evolution():
    """The switch happens at the first channel whose intermediate rank reaches 2^N; from there the
    run is the exact evolution, so when nothing was truncated before the switch the result is the
    full-rank run itself."""
    # n = 3: a 4-operator channel on one column has V_I = 3^(1/3) * 4 = 5.8 < 8; on two columns 11.5
    prog = C.cfg1_program(n=3, r=8, layers=2, p=0.05)
    rho, at = run_lret_switching(prog)
    kr = [i for i, op in enumerate(prog.ops) if isinstance(op, C.Kraus)]
    assert at == kr[1]
    np.testing.assert_allclose(rho, ofdm.run_fdm(prog), atol=1e-13)
    # n = 8 with r = 8: V_I = 8^(1/3) * 4 * 8 = 64 < 256 never switches, LRET result returned
    prog = C.cfg1_program(n=8, r=8, layers=2, p=0.01)
    rho, at = run_lret_switching(prog)
    assert at == -1
    L = oracle.run_lret(prog)
    np.testing.assert_allclose(rho, L @ L.conj().T, atol=1e-14)
    # a switch after a truncation: n = 4, r = 3, the first compression keeps 3 of 4 columns, so the
    # second channel has V_I = 4^(1/3) * 4 * 3 = 19 >= 16.  From there the evolution is exact and
    # CPTP, so the result is a density matrix within the trace-norm bound 2 delta of the one
    # truncation (renormalised) from the exact run.
    prog = C.cfg1_program(n=4, r=3, layers=3, p=0.05)
    rho, at = run_lret_switching(prog)
    kr = [i for i, op in enumerate(prog.ops) if isinstance(op, C.Kraus)]
    assert at == kr[1]
    first = C.Program(prog.n, prog.ops[: kr[1]], prog.r, prog.dtype, prog.m_max)
    log = []
    oracle.run_lret(first, log=log)
    assert len(log) == 1 and log[0]["k"] == 3 and log[0]["discarded"] > 1e-6
    ev = np.linalg.eigvalsh(0.5 * (rho + rho.conj().T))
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-15 and ev.min() > -1e-14 and abs(np.trace(rho) - 1) < 1e-13
    dist = np.sum(np.abs(np.linalg.eigvalsh(rho - ofdm.run_fdm(prog))))
    assert 0 < dist <= 2 * log[0]["discarded"] + 1e-12
