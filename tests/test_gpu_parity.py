"""GPU parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances: complex128 bulk <= 1e-10; complex64 bulk (FP32 gate sweeps and FP32-MFMA Gram /
projection, FP64 eigensolve) <= 1e-5 absolute on probabilities and observables, the target of
the method's precision split.  Elementwise comparison of L is only meaningful before the first
compression (afterwards L is defined up to L -> L Q); later checks compare rho, Prob and
expectation values.
"""
import sys

import numpy as np
import pytest

import oracle
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


def dtype_of(lr, name):
    return lr.C64 if name == "c64" else lr.C128


def run_gpu(lr, prog, L0=None, flags=0):
    dm = lr.LowRankDM(prog.n, prog.r, dtype_of(lr, prog.dtype), prog.m_max, flags)
    if L0 is not None:
        dm.set_L(L0)
    lr.run_program(dm, prog)
    return dm


def cast_input(L, dtype):
    return L.astype(np.complex64).astype(np.complex128) if dtype == "c64" else L


def rand_unitary(rng, k):
    a = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def mixed_gate_program(n, r, seed, count=40, dtype="c64"):
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(count):
        kind = rng.integers(0, 8)
        q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
        if kind == 0:
            ops.append(C.Gate((q0,), C.haar_su2(np.random.Generator(np.random.PCG64(int(rng.integers(1 << 30)))))))
        elif kind == 1:
            ops.append(C.Gate((q0, q1), C.CNOT))
        elif kind == 2:
            ops.append(C.Gate((q0, q1), C.CZ, diagonal=True))
        elif kind == 3:
            ops.append(C.Gate((q0, q1), rand_unitary(rng, 2)))
        elif kind == 4:
            ops.append(C.Gate((q0,), C.rz(rng.uniform(-3, 3))))
        elif kind == 5:
            ops.append(C.Gate((q0,), [C.S, C.T, C.X, C.Y, C.H][int(rng.integers(0, 5))]))
        elif kind == 6:
            ops.append(C.DiagWeight(np.exp(1j * rng.uniform(0, 2 * np.pi, n + 1))))
        else:
            ops.append(C.Gate((q0, q1), C.SWAP))
    return C.Program(n, ops, r, dtype, 2, "mixed")


# ------------------------------------------------------------------------------- gate sweeps
@pytest.mark.parametrize("dtype,n,r", [("c64", 7, 8), ("c128", 7, 8), ("c64", 11, 64), ("c128", 9, 32)])
def test_gate_sweeps_elementwise(lr, dtype, n, r):
    _say(f"[gates] dtype={dtype} n={n} r={r}")
    prog = mixed_gate_program(n, r, seed=n * 100 + r, count=60, dtype=dtype)
    L0 = cast_input(C.random_orthogonal_factor(n, r, seed=7 + n), dtype)
    dm = run_gpu(lr, prog, L0)
    got = dm.get_L()[:, :r]
    ref = oracle.run_lret(prog, L0)
    tol = 2e-6 if dtype == "c64" else 1e-13
    assert np.max(np.abs(got - ref)) < tol
    dm.close()


def phase_gate_program(n, r, seed, count=80, dtype="c64"):
    """One-qubit gates and diagonal gates only, so that every gate pass runs in register phases:
    CZ, Z(x)Z-type sign patterns, diagonals with some phases exactly 1, controlled phases, Z, S,
    T and Rz, on random qubits (register bits, thread bits and tile bits of a pass)."""
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(count):
        kind = int(rng.integers(0, 8))
        q0, q1 = (int(x) for x in rng.choice(n, 2, replace=False))
        if kind <= 1:
            ops.append(C.Gate((q0,), C.haar_su2(np.random.Generator(np.random.PCG64(int(rng.integers(1 << 30)))))))
        elif kind == 2:
            ops.append(C.Gate((q0, q1), C.CZ, diagonal=True))
        elif kind == 3:
            ops.append(C.Gate((q0, q1), np.diag(rng.choice([-1.0, 1.0], 4)).astype(np.complex128), diagonal=True))
        elif kind == 4:
            ops.append(C.Gate((q0, q1), np.diag([1, 1, 1, np.exp(1j * rng.uniform(-3, 3))]), diagonal=True))
        elif kind == 5:
            ops.append(C.Gate((q0,), [C.Z, C.S, C.T, C.rz(rng.uniform(-3, 3))][int(rng.integers(0, 4))]))
        elif kind == 6:
            ops.append(C.Gate((q0, q1), np.diag([1.0, -1.0, 1.0, 1.0]).astype(np.complex128), diagonal=True))
        else:
            ops.append(C.Gate((q0,), [C.H, C.X][int(rng.integers(0, 2))]))
    return C.Program(n, ops, r, dtype, 2, "phases")


@pytest.mark.parametrize("dtype,n,r", [("c64", 7, 8), ("c64", 8, 64), ("c64", 11, 64), ("c128", 8, 32),
                                       ("c128", 10, 32)])
def test_register_phase_passes_elementwise(lr, dtype, n, r):
    """Passes of one-qubit and diagonal gates (the register-phase form of a gate pass), with the
    diagonal qubits in every combination of register, thread and tile bits, element by element
    against the oracle's gate contractions (Eq. "low rank evolution G")."""
    _say(f"[phase gates] dtype={dtype} n={n} r={r}")
    prog = phase_gate_program(n, r, seed=n * 31 + r, dtype=dtype)
    L0 = cast_input(C.random_orthogonal_factor(n, r, seed=11 + n), dtype)
    dm = run_gpu(lr, prog, L0)
    got = dm.get_L()[:, :r]
    ref = oracle.run_lret(prog, L0)
    tol = 2e-6 if dtype == "c64" else 1e-13
    err = float(np.max(np.abs(got - ref)))
    _say(f"  max|dL| {err:.2e}")
    assert err < tol
    dm.close()


# ------------------------------------------------------------------------------- one compression
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("chan", ["ad", "dep", "deph", "none"])
@pytest.mark.parametrize("plain", [0, 1])
def test_single_compress(lr, dtype, chan, plain):
    n, r, q = 8, 16, 3
    _say(f"[compress] dtype={dtype} chan={chan} plain={plain}")
    ops = {"ad": C.amplitude_damping(0.05), "dep": C.depolarizing(0.03), "deph": C.phase_flip(0.04)}
    L0 = cast_input(C.random_orthogonal_factor(n, r, seed=11, decay=0.7), dtype)
    prog_ops = []
    if chan != "none":
        prog_ops.append(C.Kraus(q, ops[chan]))
    prog_ops.append(C.Compress(r - 3, 0.0, 0, 1))
    prog = C.Program(n, prog_ops, r, dtype, 4)
    dm = lr.LowRankDM(n, r, dtype_of(lr, dtype), 4, lr.FLAG_PLAIN if plain else 0)
    dm.set_L(L0)
    if chan != "none":
        dm.apply_kraus(q, ops[chan])
    info = dm.compress(r - 3, info=True)
    log = []
    Lref = oracle.run_lret(prog, L0, log=log)
    L = dm.get_L()
    rho, rho_ref = L @ L.conj().T, Lref @ Lref.conj().T
    tol = 2e-6 if dtype == "c64" else 1e-12
    assert np.max(np.abs(rho - rho_ref)) < tol
    assert info["rank"] == log[0]["k"]
    assert abs(info["discarded"] - log[0]["discarded"]) < (1e-6 if dtype == "c64" else 1e-12)
    assert abs(info["trace_before"] - log[0]["trace"]) < (1e-6 if dtype == "c64" else 1e-12)
    # the new columns are orthogonal with squared norms c^2 lambda_i (Theorem 1)
    G = L.conj().T @ L
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < (1e-6 if dtype == "c64" else 1e-13)
    dm.close()


# ------------------------------------------------------------------------------- whole circuits
def test_cfg1_complex128(lr):
    prog = C.cfg1_program()
    _say(f"[cfg1] n={prog.n} r={prog.r} layers={prog.layers}")
    dm = run_gpu(lr, prog)
    P = dm.probabilities().cpu().numpy()
    z, zz, tr = dm.expect_z()
    L = oracle.run_lret(prog)
    Pref = oracle.probabilities(L)
    assert np.max(np.abs(P - Pref)) < 1e-10
    assert np.max(np.abs(z - oracle.expect_z(Pref, prog.n))) < 1e-10
    assert abs(tr - 1.0) < 1e-12
    dm.close()


def test_full_rank_equals_fdm(lr):
    """r >= rank: the truncation keeps everything and LRET is the exact evolution."""
    prog = C.cfg1_program(n=5, r=32, layers=3)
    _say("[full-rank] n=5 r=32 c128")
    dm = run_gpu(lr, prog)
    L = dm.get_L()
    rho = ofdm.run_fdm(prog)
    assert np.max(np.abs(L @ L.conj().T - rho)) < 1e-10
    dm.close()


@pytest.mark.parametrize("plain", [0, 1])
def test_cfg3_small(lr, plain):
    prog = C.cfg3_program(n=10, r=32, layers=3)
    _say(f"[cfg3-small] n=10 r=32 layers=3 plain={plain}")
    dm = run_gpu(lr, prog, flags=lr.FLAG_PLAIN if plain else 0)
    P = dm.probabilities().cpu().numpy()
    z, zz, tr = dm.expect_z()
    L = oracle.run_lret(prog)
    Pref = oracle.probabilities(L)
    assert np.max(np.abs(P - Pref)) < 1e-5
    assert np.max(np.abs(zz - oracle.expect_zz(Pref, prog.n))) < 1e-5
    assert abs(tr - 1.0) < 1e-5
    dm.close()


@pytest.mark.parametrize("chans", [[("ad", 0.05), ("deph", 0.04)], [("ad", 0.03), ("dep", 0.02), ("deph", 0.01)]])
def test_chained_compressions_complex128(lr, chans):
    """Consecutive channels on one qubit reuse the split view (Gram W^H S W, composed projection):
    complex128 agrees with the oracle's step-by-step run to 1e-10, and an output between the two
    channels (which materialises the intermediate factor) changes nothing."""
    prog = C.brickwork_program(7, 2, 16, chans, seed=91, dtype="c128")
    _say(f"[chain c128] chans={chans}")
    dm = run_gpu(lr, prog)
    P = dm.probabilities().cpu().numpy()
    Pref = oracle.probabilities(oracle.run_lret(prog))
    assert np.max(np.abs(P - Pref)) < 1e-10
    # the same program with a sync after every compression (no chaining)
    dm2 = lr.LowRankDM(prog.n, prog.r, lr.C128, prog.m_max)
    for op in prog.ops:
        lr.run_program(dm2, C.Program(prog.n, [op], prog.r, prog.dtype, prog.m_max, "one", 0))
        if isinstance(op, C.Compress):
            dm2.synchronize()
    P2 = dm2.probabilities().cpu().numpy()
    assert np.max(np.abs(P2 - Pref)) < 1e-10
    dm.close()
    dm2.close()


@pytest.mark.parametrize("n,r,chans", [(10, 64, [("ad", 0.002), ("deph", 0.001)]),
                                       (9, 32, [("dep", 0.003)])])
def test_largest_gram_order(lr, n, r, chans):
    """m r_pad = 128: the largest Gram matrix the eigensolver takes."""
    prog = C.brickwork_program(n, 2, r, chans, seed=77)
    _say(f"[N=128] n={n} r={r} chans={chans}")
    dm = run_gpu(lr, prog)
    P = dm.probabilities().cpu().numpy()
    Pref = oracle.probabilities(oracle.run_lret(prog))
    assert np.max(np.abs(P - Pref)) < 1e-5
    dm.close()


def test_cfg3_full_size_first_layers(lr):
    """Full cfg3 size (n = 20, r = 64) in the benchmark's launch configuration: properties that
    hold at any size (unit trace, Prob >= 0, |<ZZ>| <= 1, run-to-run determinism)."""
    prog = C.cfg3_program(layers=2)
    _say("[cfg3-full] n=20 r=64 layers=2")
    dm = run_gpu(lr, prog)
    z, zz, tr = dm.expect_z()
    P = dm.probabilities().cpu().numpy()
    assert abs(tr - 1.0) < 1e-5
    assert P.min() > -1e-7 and abs(P.sum() - 1.0) < 1e-5
    assert np.all(np.abs(zz) <= 1 + 1e-6)
    dm2 = run_gpu(lr, prog)
    z2, zz2, tr2 = dm2.expect_z()
    assert np.array_equal(zz, zz2)
    dm.close(); dm2.close()


def test_cfg2_small_cluster_policy(lr):
    prog = C.cfg2_program(n=10, r=16, iterations=3, p=0.001)
    _say("[cfg2-small] n=10 r=16 it=3 tie=cluster")
    dm = run_gpu(lr, prog)
    P = dm.probabilities().cpu().numpy()
    Pref = oracle.probabilities(oracle.run_lret(prog))
    assert np.max(np.abs(P - Pref)) < 1e-5
    dm.close()


def test_grover_noiseless_closed_form(lr):
    n, t = 12, 4
    prog = C.cfg2_program(n=n, r=8, iterations=t, p=0.0)
    _say("[grover] n=12 p=0")
    dm = run_gpu(lr, prog)
    P = dm.probabilities().cpu().numpy()
    M = 1 + n + n * (n - 1) // 2
    th = np.arcsin(np.sqrt(M / 2 ** n))
    pg = np.sin((2 * t + 1) * th) ** 2
    w = np.array([bin(x).count("1") for x in range(2 ** n)])
    ref = np.where(w <= 2, pg / M, (1 - pg) / (2 ** n - M))
    assert np.max(np.abs(P - ref)) < 1e-6
    dm.close()


# ------------------------------------------------------------------------------- outputs
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_pauli_and_z(lr, dtype):
    n, r = 9, 16
    _say(f"[pauli] dtype={dtype}")
    L0 = cast_input(C.random_orthogonal_factor(n, r, seed=5), dtype)
    dm = lr.LowRankDM(n, r, dtype_of(lr, dtype), 2)
    dm.set_L(L0)
    xm, zm, cf, _ = C.random_pauli_sum(n, terms=80, max_weight=4, seed=9)
    got = dm.expect_pauli(xm, zm)
    ref = np.array([oracle.expect_pauli(L0, n, x, z).real for x, z in zip(xm, zm)])
    tol = 2e-6 if dtype == "c64" else 1e-13
    assert np.max(np.abs(got - ref)) < tol
    e = dm.expect_pauli(xm, zm, cf, summed=True)
    assert abs(e - float(np.sum(cf * ref))) < 20 * tol
    z, zz, tr = dm.expect_z()
    P = oracle.probabilities(L0)
    assert np.max(np.abs(z - oracle.expect_z(P, n))) < tol
    assert np.max(np.abs(zz - oracle.expect_zz(P, n))) < tol
    dm.close()


def test_sampling_inverse_cdf(lr):
    n, r = 12, 8
    _say("[sample]")
    L0 = C.random_orthogonal_factor(n, r, seed=21).astype(np.complex128)
    dm = lr.LowRankDM(n, r, lr.C128, 2)
    dm.set_L(L0)
    u = C.sample_uniforms(10000, 3003)
    got = dm.sample(u)
    P = oracle.probabilities(L0)
    ref = oracle.sample_inverse_cdf(P, u)
    cdf = np.cumsum(P)
    mism = np.nonzero(got != ref)[0]
    for j in mism:   # only allowed where u lies on a CDF step up to rounding of the running sums
        assert np.min(np.abs(cdf - u[j] * cdf[-1])) < 1e-12
    assert mism.size <= 2
    dm.close()


def test_run_twice_bitwise(lr):
    prog = C.cfg3_program(n=11, r=32, layers=2)
    _say("[determinism]")
    a = run_gpu(lr, prog)
    b = run_gpu(lr, prog)
    assert np.array_equal(a.get_L(), b.get_L())
    a.close(); b.close()


def test_error_paths(lr):
    dm = lr.LowRankDM(6, 8, lr.C64, 2)
    with pytest.raises(lr.LrdmError) as e:
        dm.apply_gate((0,), np.array([[1, 1], [0, 1]]))
    assert e.value.status == 1
    with pytest.raises(lr.LrdmError) as e:
        dm.apply_gate((0, 0), np.eye(4))
    assert e.value.status == 1
    with pytest.raises(lr.LrdmError) as e:
        dm.apply_kraus(1, np.stack([C.I2, C.X]))   # incomplete: sum E^H E = 2 I
    assert e.value.status == 1
    with pytest.raises(lr.LrdmError):
        dm.compress(9)
    dm.apply_kraus(1, C.amplitude_damping(0.1))
    with pytest.raises(lr.LrdmError) as e:
        dm.apply_gate((0,), C.H)
    assert e.value.status == 5
    with pytest.raises(lr.LrdmError) as e:
        dm.expect_z()
    assert e.value.status == 5
    dm.compress(8)
    z, _, tr = dm.expect_z()
    assert abs(tr - 1) < 1e-6
    dm.close()


@pytest.mark.parametrize("plain", [0, 1])
def test_non_finite_factor_poisons_the_handle(lr, plain):
    """A NaN in the factor reaches the Gram matrix: the eigensolver reports it (LRDM_E_EIG at the
    first call that synchronises), and every later call on the handle returns LRDM_E_STATE.
    Every loop of the eigensolver is bounded independently of the values, so the kernels end."""
    n, r = 8, 8
    _say(f"[nan] plain={plain}")
    L0 = C.random_orthogonal_factor(n, r, seed=3).astype(np.complex64)
    L0[17, 2] = np.nan
    dm = lr.LowRankDM(n, r, lr.C64, 2, lr.FLAG_PLAIN if plain else 0)
    dm.set_L(L0)
    dm.apply_kraus(3, C.amplitude_damping(0.1))
    with pytest.raises(lr.LrdmError) as e:
        dm.compress(r, info=True)
    assert e.value.status == 4
    with pytest.raises(lr.LrdmError) as e:
        dm.expect_z()
    assert e.value.status == 5
    with pytest.raises(lr.LrdmError) as e:
        dm.apply_gate((0,), C.H)
    assert e.value.status == 5
    dm.close()
    # without info, the error surfaces at the next synchronising output call
    dm = lr.LowRankDM(n, r, lr.C64, 2, lr.FLAG_PLAIN if plain else 0)
    dm.set_L(L0)
    dm.apply_kraus(5, C.phase_flip(0.1))
    dm.compress(r)
    with pytest.raises(lr.LrdmError) as e:
        dm.expect_z()
    assert e.value.status == 4
    with pytest.raises(lr.LrdmError) as e:
        dm.synchronize()
    assert e.value.status == 5
    dm.close()
    # a fresh handle is unaffected
    dm = lr.LowRankDM(n, r, lr.C64, 2)
    dm.apply_gate((0,), C.H)
    z, _, tr = dm.expect_z()
    assert abs(tr - 1.0) < 1e-6
    dm.close()
