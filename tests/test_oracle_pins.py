"""Pins of the CPU oracle against things other than itself (no GPU).

Every oracle function is checked against an independent construction: Kronecker / explicit-loop
brute force, closed forms of the channels (Sec. III.A), Theorem 1 (App. B) against an explicit
eigendecomposition of rho, the Eckart-Young truncation identities (Sec. II.B), Grover's closed
form (Sec. III.C) and exact agreement with full-rank evolution when r >= rank.
"""
import numpy as np
import pytest

import oracle
from oracle import fdm as ofdm
from oracle.lret import compress, kraus_expand, run_lret
from workloads import circuits as C


# ---------------------------------------------------------------- independent brute-force helpers
def full_matrix(n, qubits, U):
    """Explicit 2^n x 2^n matrix of a k-qubit gate, built by looping over basis pairs."""
    D = 2 ** n
    M = np.zeros((D, D), dtype=np.complex128)
    mask = sum(1 << q for q in qubits)
    for x in range(D):
        i = sum(((x >> q) & 1) << j for j, q in enumerate(qubits))
        for xp in range(D):
            if (x & ~mask) != (xp & ~mask):
                continue
            ip = sum(((xp >> q) & 1) << j for j, q in enumerate(qubits))
            M[xp, x] = U[ip, i]
    return M


def kron_1q(n, q, U):
    return np.kron(np.kron(np.eye(2 ** (n - 1 - q)), U), np.eye(2 ** q))


def pauli_full(n, xmask, zmask):
    M = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):            # kron order: most significant qubit first
        b = ((xmask >> q) & 1, (zmask >> q) & 1)
        P = {(0, 0): C.I2, (1, 0): C.X, (0, 1): C.Z, (1, 1): C.Y}[b]
        M = np.kron(M, P)
    return M


def rand_L(rng, n, V):
    L = rng.standard_normal((2 ** n, V)) + 1j * rng.standard_normal((2 ** n, V))
    return L / np.linalg.norm(L)


def rand_u(rng, k):
    a = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
    q, _ = np.linalg.qr(a)
    return q


def trace_norm(A):
    return float(np.sum(np.abs(np.linalg.eigvalsh(0.5 * (A + A.conj().T)))))


# ---------------------------------------------------------------- pin 1: gates
def test_full_matrix_matches_kron_convention():
    rng = np.random.default_rng(0)
    U = rand_u(rng, 1)
    for q in range(4):
        np.testing.assert_allclose(full_matrix(4, (q,), U), kron_1q(4, q, U), atol=0)


@pytest.mark.parametrize("qubits", [(0,), (3,), (4,), (0, 1), (1, 0), (0, 4), (3, 1), (2, 3)])
def test_gate_vs_bruteforce(qubits):
    rng = np.random.default_rng(len(qubits) * 10 + qubits[0])
    n = 5
    L = rand_L(rng, n, 3)
    U = rand_u(rng, len(qubits))
    got = oracle.apply_gate(L, n, qubits, U)
    np.testing.assert_allclose(got, full_matrix(n, qubits, U) @ L, atol=1e-14)
    # L^H L is invariant under a unitary gate
    np.testing.assert_allclose(got.conj().T @ got, L.conj().T @ L, atol=1e-14)


def test_named_gates():
    # CNOT(c=0 -> t=1) maps |c=1,t=0> (x=1) to x=3
    v = np.zeros((4, 1), complex); v[1] = 1
    out = oracle.apply_gate(v, 2, (0, 1), C.CNOT)
    assert abs(out[3, 0] - 1) < 1e-15
    # rotations: R_P(theta) = exp(-i theta P / 2)
    for f, P in ((C.rx, C.X), (C.ry, C.Y), (C.rz, C.Z)):
        th = 0.731
        w, V = np.linalg.eigh(P)
        ref = V @ np.diag(np.exp(-0.5j * th * w)) @ V.conj().T
        np.testing.assert_allclose(f(th), ref, atol=1e-15)
    # Haar SU(2) draws are unitary with unit determinant
    rng = np.random.Generator(np.random.PCG64(1))
    U = C.haar_su2(rng)
    np.testing.assert_allclose(U @ U.conj().T, np.eye(2), atol=1e-15)
    assert abs(np.linalg.det(U) - 1) < 1e-14


def test_diag_weight_vs_bruteforce():
    rng = np.random.default_rng(3)
    n = 5
    L = rand_L(rng, n, 2)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, n + 1))
    D = np.diag([ph[bin(x).count("1")] for x in range(2 ** n)])
    np.testing.assert_allclose(oracle.apply_diag_weight(L, n, ph), D @ L, atol=1e-15)


# ---------------------------------------------------------------- pins 2-3, 7-8: channels
CHANNELS = {"dep": C.depolarizing(0.013), "ad": C.amplitude_damping(0.021),
            "deph": C.phase_flip(0.017), "bitflip": C.bit_flip(0.011)}


@pytest.mark.parametrize("name", list(CHANNELS))
def test_kraus_completeness_and_trace(name):
    ops = CHANNELS[name]
    np.testing.assert_allclose(sum(E.conj().T @ E for E in ops), np.eye(2), atol=1e-15)
    rng = np.random.default_rng(5)
    n = 4
    L = rand_L(rng, n, 3)
    Lp = kraus_expand(L, n, 2, ops)
    assert Lp.shape == (2 ** n, 3 * len(ops))
    assert abs(np.trace(Lp.conj().T @ Lp) - np.trace(L.conj().T @ L)) < 1e-14


@pytest.mark.parametrize("name", list(CHANNELS))
def test_kraus_expansion_vs_superoperator(name):
    ops = CHANNELS[name]
    rng = np.random.default_rng(6)
    n, q = 4, 1
    L = rand_L(rng, n, 3)
    rho = L @ L.conj().T
    ref = sum(full_matrix(n, (q,), E) @ rho @ full_matrix(n, (q,), E).conj().T for E in ops)
    Lp = kraus_expand(L, n, q, ops)
    np.testing.assert_allclose(Lp @ Lp.conj().T, ref, atol=1e-14)
    np.testing.assert_allclose(ofdm.fdm_channel(rho, n, q, ops), ref, atol=1e-14)


def test_fdm_gate_vs_bruteforce():
    rng = np.random.default_rng(7)
    n = 4
    L = rand_L(rng, n, 4)
    rho = L @ L.conj().T
    U = rand_u(rng, 2)
    Uf = full_matrix(n, (3, 1), U)
    np.testing.assert_allclose(ofdm.fdm_gate(rho, n, (3, 1), U), Uf @ rho @ Uf.conj().T, atol=1e-14)


def test_depolarizing_closed_form():
    """(1-p) rho + p/3 sum sigma rho sigma = (1 - 4p/3) rho + (4p/3) Tr(rho) I/2 (Sec. III.A.1):
    the Bloch vector shrinks by (1 - 4p/3) per application."""
    rng = np.random.default_rng(8)
    p = 0.07
    L = rand_L(rng, 1, 2)
    rho = L @ L.conj().T
    ref = (1 - 4 * p / 3) * rho + (4 * p / 3) * np.trace(rho) * np.eye(2) / 2
    Lp = kraus_expand(L, 1, 0, C.depolarizing(p))
    np.testing.assert_allclose(Lp @ Lp.conj().T, ref, atol=1e-15)
    # product state on 3 qubits, channel on every qubit, r >= 2^n so LRET is exact
    prog = C.Program(3, [C.Gate((q,), C.haar_su2(np.random.Generator(np.random.PCG64(q))))
                         for q in range(3)], r=8)
    bloch0 = []
    for q in range(3):
        U = prog.ops[q].u
        v = U[:, 0]
        bloch0.append(np.real(np.conj(v) @ C.Z @ v))
    for _ in range(4):
        for q in range(3):
            prog.ops.append(C.Kraus(q, C.depolarizing(p)))
            prog.ops.append(C.Compress(8, 0.0, 0, 0))
    L = run_lret(prog)
    z = oracle.expect_z(oracle.probabilities(L), 3)
    np.testing.assert_allclose(z, np.array(bloch0) * (1 - 4 * p / 3) ** 4, atol=1e-13)


def test_amplitude_damping_and_phase_flip_closed_forms():
    g, p, k = 0.03, 0.02, 7
    ops = [C.Gate((0,), C.X)]
    for _ in range(k):
        ops += [C.Kraus(0, C.amplitude_damping(g)), C.Compress(2, 0.0, 0, 0)]
    L = run_lret(C.Program(1, ops, r=2))
    assert abs(oracle.probabilities(L)[1] - (1 - g) ** k) < 1e-14
    ops = [C.Gate((0,), C.H)]
    for _ in range(k):
        ops += [C.Kraus(0, C.phase_flip(p)), C.Compress(2, 0.0, 0, 0)]
    L = run_lret(C.Program(1, ops, r=2))
    x = oracle.expect_pauli(L, 1, 1, 0).real
    assert abs(x - (1 - 2 * p) ** k) < 1e-14


# ---------------------------------------------------------------- pins 4-5: Theorem 1, truncation
def test_theorem1_spectrum():
    rng = np.random.default_rng(9)
    n, V = 5, 12
    Lp = rand_L(rng, n, V)
    G = Lp.conj().T @ Lp
    lam_G = np.sort(np.linalg.eigvalsh(G))[::-1]
    lam_rho = np.sort(np.linalg.eigvalsh(Lp @ Lp.conj().T))[::-1]
    np.testing.assert_allclose(lam_G, lam_rho[:V], atol=1e-14)
    assert np.max(np.abs(lam_rho[V:])) < 1e-14
    # u_D = B u_M is an eigenvector of B B^H with the same eigenvalue
    w, U = np.linalg.eigh(G)
    u = Lp @ U[:, -1]
    np.testing.assert_allclose((Lp @ Lp.conj().T) @ u, w[-1] * u, atol=1e-13)


@pytest.mark.parametrize("renorm", [0, 1])
def test_compress_eckart_young(renorm):
    rng = np.random.default_rng(10 + renorm)
    n, V, k = 5, 16, 5
    Lp = rand_L(rng, n, V)
    rho = Lp @ Lp.conj().T
    Lnew, info = compress(Lp, k, 0.0, 0, renorm)
    assert info["k"] == k and Lnew.shape == (2 ** n, k)
    rt = Lnew @ Lnew.conj().T
    # direct truncation of rho's own eigendecomposition (no Theorem 1)
    w, U = np.linalg.eigh(rho)
    w, U = w[::-1], U[:, ::-1]
    direct = (U[:, :k] * w[:k]) @ U[:, :k].conj().T
    delta = float(np.sum(w[k:]))
    assert abs(info["discarded"] - delta) < 1e-14
    if renorm:
        direct = direct / np.sum(w[:k])
        assert abs(np.trace(rt).real - 1) < 1e-14
        assert abs(trace_norm(rho - rt) - 2 * delta) < 1e-13
    else:
        np.testing.assert_allclose(np.linalg.norm(rho - rt) ** 2, np.sum(w[k:] ** 2), rtol=1e-10)
        assert abs(trace_norm(rho - rt) - delta) < 1e-13
    np.testing.assert_allclose(rt, direct, atol=1e-14)
    # new columns are orthogonal with norms^2 = c^2 lambda_i
    c2 = 1.0 / np.sum(w[:k]) if renorm else 1.0
    np.testing.assert_allclose(Lnew.conj().T @ Lnew, np.diag(c2 * w[:k]), atol=1e-14)
    assert np.min(np.linalg.eigvalsh(rt)) > -1e-14
    assert np.linalg.matrix_rank(rt, tol=1e-12) <= k


def test_select_rank_rules():
    lam = np.array([0.5, 0.3, 0.1, 0.1, 0.05, 0.05 - 1e-9, 0.0])
    tr = float(lam.sum())
    assert oracle.select_rank(lam, tr, 10, 0.0, 0) == 7
    assert oracle.select_rank(lam, tr, 3, 0.0, 0) == 3
    # eps: smallest k with kept >= (1 - eps) tr
    assert oracle.select_rank(lam, tr, 10, 0.15, 0) == 4      # 0.5+0.3+0.1+0.1 = 1.0 >= 0.935
    assert oracle.select_rank(lam, tr, 10, 0.25, 0) == 3      # 0.9 >= 0.825
    # cluster: a cut inside the 0.1/0.1 tie moves up; a near-tie within tau moves too
    assert oracle.select_rank(lam, tr, 3, 0.0, 1) == 2
    assert oracle.select_rank(lam, tr, 5, 0.0, 1) == 4
    # beyond the Gram order the spectrum continues with zeros: keeping all N columns, the cut
    # against lambda_{N+1} = 0 drops a last eigenvalue within tau Tr G of zero (here the exact
    # zero; the next gap, 0.05 - 1e-9 against 0, stops it), and padding the spectrum with zeros
    # changes nothing
    assert oracle.select_rank(lam, tr, 10, 0.0, 1) == 6
    tiny = np.array([0.6, 0.4 - 5e-7, 5e-7])
    assert oracle.select_rank(tiny, 1.0, 3, 0.0, 1) == 2
    assert oracle.select_rank(tiny, 1.0, 3, 0.0, 0) == 3
    for r in (2, 3, 5):
        padded = np.concatenate([tiny, np.zeros(6)])
        assert oracle.select_rank(padded, 1.0, r, 0.0, 1) == oracle.select_rank(tiny, 1.0, r, 0.0, 1)


# ---------------------------------------------------------------- pins 6, 9: whole path vs FDM
def test_lret_equals_fdm_when_rank_suffices():
    prog = C.cfg1_program(n=4, r=16, layers=4, p=0.02)
    L = run_lret(prog)
    rho = ofdm.run_fdm(prog)
    np.testing.assert_allclose(L @ L.conj().T, rho, atol=1e-13)


def test_lret_equals_fdm_cfg1_full_rank():
    prog = C.cfg1_program(r=64, layers=3)
    L = run_lret(prog)
    rho = ofdm.run_fdm(prog)
    np.testing.assert_allclose(L @ L.conj().T, rho, atol=1e-12)


@pytest.mark.parametrize("renorm", [0, 1])
def test_tracenorm_bound_vs_fdm(renorm):
    """CPTP maps contract the trace norm, so ||rho_LRET - rho_FDM||_1 <= sum_s e_s with
    e_s = delta_s (renorm off) or 2 delta_s (renorm on)."""
    prog = C.cfg1_program(n=5, r=3, layers=4, p=0.03, renorm=renorm)
    log = []
    L = run_lret(prog, log=log)
    rho = ofdm.run_fdm(prog)
    bound = (2 if renorm else 1) * sum(i["discarded"] for i in log)
    err = trace_norm(L @ L.conj().T - rho)
    assert bound > 1e-4           # truncation really happened
    assert err <= bound + 1e-12
    P = oracle.probabilities(L)
    assert np.sum(np.abs(P - np.real(np.diag(rho)))) <= bound + 1e-12


def test_distortion_definition():
    a = np.array([0.5, 0.5]); b = np.array([0.6, 0.4]); c = np.array([1.0, 0.0])
    assert abs(oracle.distortion(a, b, c) - 0.2 / 0.8) < 1e-15
    assert oracle.distortion(b, b, c) == 0.0


# ---------------------------------------------------------------- pin 10: Grover closed form
def test_grover_closed_form():
    n, t = 8, 3
    prog = C.cfg2_program(n=n, r=4, iterations=t, p=0.0)
    M = 1 + n + n * (n - 1) // 2
    theta = np.arcsin(np.sqrt(M / 2 ** n))
    p_good = np.sin((2 * t + 1) * theta) ** 2
    w = np.array([bin(x).count("1") for x in range(2 ** n)])
    ref = np.where(w <= 2, p_good / M, (1 - p_good) / (2 ** n - M))
    psi = ofdm.run_sv(prog)
    np.testing.assert_allclose(np.abs(psi) ** 2, ref, atol=1e-14)
    L = run_lret(prog)
    np.testing.assert_allclose(oracle.probabilities(L), ref, atol=1e-14)


# ---------------------------------------------------------------- pins 11-12: outputs
def test_pauli_vs_bruteforce():
    rng = np.random.default_rng(11)
    n = 4
    L = rand_L(rng, n, 3)
    rho = L @ L.conj().T
    for xm, zm in [(0, 0), (1, 0), (0, 2), (5, 5), (6, 3), (15, 9), (8, 8)]:
        got = oracle.expect_pauli(L, n, xm, zm)
        ref = np.trace(rho @ pauli_full(n, xm, zm))
        assert abs(got - ref) < 1e-14
        assert abs(got.imag) < 1e-14
    assert abs(oracle.expect_pauli(L, n, 0, 0) - np.trace(rho)) < 1e-15


def test_probabilities_and_z():
    rng = np.random.default_rng(12)
    n = 5
    L = rand_L(rng, n, 4)
    P = oracle.probabilities(L)
    np.testing.assert_allclose(P, np.real(np.diag(L @ L.conj().T)), atol=1e-16)
    assert np.all(P >= 0) and abs(P.sum() - np.trace(L.conj().T @ L).real) < 1e-15
    z = oracle.expect_z(P, n)
    zz = oracle.expect_zz(P, n)
    for i in range(n):
        assert abs(z[i] - oracle.expect_pauli(L, n, 0, 1 << i).real) < 1e-15
    for i in range(n - 1):
        assert abs(zz[i] - oracle.expect_pauli(L, n, 0, 3 << i).real) < 1e-15


def test_sampling_rule():
    rng = np.random.default_rng(13)
    P = rng.random(37); P /= P.sum() * 1.3           # trace below one on purpose
    u = rng.random(500)
    got = oracle.sample_inverse_cdf(P, u)
    tot = P.sum()
    for uj, g in zip(u, got):
        acc, ref = 0.0, None
        for x, px in enumerate(P):
            acc += px
            if acc > uj * tot:
                ref = x
                break
        assert g == ref
    # chi-square plausibility for 1e4 draws
    u = np.random.Generator(np.random.PCG64(3003)).random(10000)
    s = oracle.sample_inverse_cdf(P, u)
    counts = np.bincount(s.astype(np.int64), minlength=P.size)
    exp = 10000 * P / tot
    chi2 = np.sum((counts - exp) ** 2 / exp)
    assert chi2 < P.size + 6 * np.sqrt(2 * P.size)
