"""GPU parity of the reverse sweep (energy gradients) against the FP64 oracle.

Tolerances: complex128 bulk <= 1e-9 on gradients; complex64 bulk <= 1e-4 absolute on gradients
(FP32 products over the 2^n rows, FP64 small matrices) and <= 1e-5 on the energy.  The
truncation adjoint is compared through a gauge-invariant loss: both sides differentiate
l(L) = Tr(H rho_n(L)), whose gradient with respect to the pre-channel factor is unique.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import grad as OG
from oracle.lret import compress, kraus_expand
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


def _dt(lr, name):
    return lr.C64 if name == "c64" else lr.C128


def _rand_factor(rng, n, r, dtype):
    L = rng.standard_normal((2 ** n, r)) + 1j * rng.standard_normal((2 ** n, r))
    L /= np.linalg.norm(L)
    return L.astype(np.complex64).astype(np.complex128) if dtype == "c64" else L


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_pauli_sum_apply(lr, dtype):
    _say(f"pauli_apply {dtype}")
    n, r = 7, 8
    rng = np.random.default_rng(1)
    L = _rand_factor(rng, n, r, dtype)
    xm, zm, co, _ = C.random_pauli_sum(n, terms=40, max_weight=4, seed=3)
    src = lr.LowRankDM(n, r, _dt(lr, dtype), 2)
    dst = lr.LowRankDM(n, r, _dt(lr, dtype), 2)
    src.set_L(L)
    dst.apply_pauli_sum_from(src, xm, zm, co)
    got = dst.get_L()[:, :r]
    ref = OG.apply_pauli_sum(L, n, xm, zm, co)
    tol = 1e-5 if dtype == "c64" else 1e-12
    assert np.max(np.abs(got - ref)) <= tol * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_pauli_overlap_complex(lr, dtype):
    _say(f"pauli_overlap {dtype}")
    n, r = 7, 8
    rng = np.random.default_rng(2)
    A, B = _rand_factor(rng, n, r, dtype), _rand_factor(rng, n, r, dtype)
    xm, zm, _, _ = C.random_pauli_sum(n, terms=30, max_weight=3, seed=4)
    ha, hb = lr.LowRankDM(n, r, _dt(lr, dtype), 2), lr.LowRankDM(n, r, _dt(lr, dtype), 2)
    ha.set_L(A)
    hb.set_L(B)
    got = ha.pauli_overlap(hb, xm, zm)
    ref = np.array([np.vdot(A, OG.apply_pauli_sum(B, n, [x], [z], [1.0])) for x, z in zip(xm, zm)])
    tol = 1e-6 if dtype == "c64" else 1e-13
    np.testing.assert_allclose(got, ref, atol=tol)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("chan,renorm,r_in,r_keep", [("dep", 1, 8, 5), ("dep", 0, 8, 8), ("ad", 1, 16, 9),
                                                      ("deph", 1, 6, 3), ("ad", 0, 3, 8)])
def test_compress_adjoint_single(lr, dtype, chan, renorm, r_in, r_keep):
    """Gradient of l(L) = Tr(H rho_n) through one channel + compression on qubit 3."""
    _say(f"compress_adjoint {dtype} {chan} renorm={renorm} r_in={r_in} r_keep={r_keep}")
    n, q = 8, 3
    ops = {"dep": C.depolarizing(0.05), "ad": C.amplitude_damping(0.3), "deph": C.phase_flip(0.2)}[chan]
    m = ops.shape[0]
    r_max = max(r_in, r_keep)   # m * r_pad <= 64 for every case here
    rng = np.random.default_rng(7)
    L = _rand_factor(rng, n, r_in, dtype)
    xm, zm, co, _ = C.random_pauli_sum(n, terms=25, max_weight=3, seed=9)
    # oracle: d/dL Tr(H rho_n(L)) = sum_a E_a^H Abar_a
    A = kraus_expand(L, n, q, ops)
    Ln, info = compress(A, r_keep, renorm=renorm)
    Abar = OG.compress_adjoint(A, OG.apply_pauli_sum(Ln, n, xm, zm, co), r_keep, renorm=renorm)
    from oracle.linalg import apply_gate
    c = L.shape[1]
    ref = sum(apply_gate(Abar[:, a * c:(a + 1) * c], n, (q,), E.conj().T) for a, E in enumerate(ops))
    # GPU
    dt = _dt(lr, dtype)
    dm = lr.LowRankDM(n, r_max, dt, m)
    bar = lr.LowRankDM(n, r_max, dt, m)
    import torch
    dm.set_L(L)
    x = torch.empty(dm.state.numel(), dtype=torch.uint8, device=dm.device)
    rec = torch.empty(dm.record_bytes(), dtype=torch.uint8, device=dm.device)
    rank = dm.checkpoint(x)
    dm.apply_kraus(q, ops)
    dm.compress_record(r_keep, rec, renorm=renorm)
    bar.apply_pauli_sum_from(dm, xm, zm, co)
    bar.compress_adjoint(x, rec, q, ops)
    got = bar.get_L()[:, :c]
    assert rank == r_in
    assert np.all(np.abs(bar.get_L()[:, c:]) <= 1e-6)
    tol = 2e-4 if dtype == "c64" else 1e-9
    err = np.max(np.abs(got - ref)) / max(1.0, np.max(np.abs(ref)))
    _say(f"  max rel err {err:.2e}")
    assert err <= tol


def _small_problem(seed, n, layers):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-np.pi, np.pi, size=(layers, n, 2))
    xm, zm, co, _ = C.random_pauli_sum(n, terms=30, max_weight=4, seed=seed)
    return theta, xm, zm, co


@pytest.mark.parametrize("dtype,renorm", [("c128", 1), ("c64", 1), ("c64", 0)])
def test_energy_gradient_small_ansatz(lr, dtype, renorm):
    from paper_2009_06657_amd.adjoint import EnergyGradient

    _say(f"energy_grad small {dtype} renorm={renorm}")
    n, r, layers = 6, 4, 3
    theta, xm, zm, co = _small_problem(5, n, layers)
    make = lambda t: C.cfg4_program(t, n=n, r=r, p=0.02, dtype=dtype, renorm=renorm)  # noqa: E731
    E_ref, g_ref = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    eng = EnergyGradient(n, r, 4, xm, zm, co, dtype=_dt(lr, dtype))
    E = eng.forward(make(theta))
    g = eng.backward(theta.size)
    etol, gtol = (1e-5, 1e-4) if dtype == "c64" else (1e-10, 1e-9)
    _say(f"  |dE| {abs(E - E_ref):.2e}  max|dg| {np.max(np.abs(g - g_ref)):.2e}")
    assert abs(E - E_ref) <= etol
    np.testing.assert_allclose(g, g_ref, atol=gtol)
    # a second call on the same engine gives the same numbers (deterministic kernels)
    E2 = eng.forward(make(theta))
    g2 = eng.backward(theta.size)
    assert E2 == E and np.array_equal(g2, g)


def test_gradient_mixed_program(lr):
    """Fixed gates (H, CNOT, SWAP, CZ), a Hamming-weight phase, three channel types and
    RX/RY/RZ angles interleaved with the channels."""
    from paper_2009_06657_amd.adjoint import EnergyGradient

    _say("energy_grad mixed program")
    n, r = 6, 4
    rng = np.random.default_rng(8)
    theta = rng.uniform(-np.pi, np.pi, size=6)
    xm, zm, co, _ = C.random_pauli_sum(n, terms=20, max_weight=3, seed=8)
    phase = np.exp(1j * rng.uniform(0, 2 * np.pi, size=n + 1))

    def make(t):
        ops = [C.Gate((0,), C.H, False, "h"),
               C.Gate((1,), C.rx(t[0]), False, "rx", (0, "X")),
               C.Gate((2,), C.ry(t[1]), False, "ry", (1, "Y")),
               C.Gate((0, 1), C.CNOT, False, "cnot"),
               C.Gate((4,), C.H, False, "h"),
               C.DiagWeight(phase),
               C.Kraus(1, C.amplitude_damping(0.2), "ad"), C.Compress(r, 0.0, 0, 1),
               C.Gate((0,), C.rz(t[2]), False, "rz", (2, "Z")),
               C.Gate((1, 2), C.CZ, True, "cz"),
               C.Gate((2,), C.rx(t[3]), False, "rx", (3, "X")),
               C.Kraus(2, C.depolarizing(0.1), "dep"), C.Compress(r, 0.0, 0, 1),
               C.LayerEnd(0),
               C.Gate((0,), C.ry(t[4]), False, "ry", (4, "Y")),
               C.Gate((5, 0), C.SWAP, False, "swap"),
               C.Gate((1,), C.rz(t[5]), False, "rz", (5, "Z")),
               C.Kraus(0, C.phase_flip(0.15), "deph"), C.Compress(r, 0.0, 0, 1),
               C.Kraus(5, C.amplitude_damping(0.1), "ad"), C.Compress(r, 0.0, 0, 1),
               C.LayerEnd(1)]
        return C.Program(n, ops, r, "c128", 4, "mixed", 2)

    E_ref, g_ref = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    eng = EnergyGradient(n, r, 4, xm, zm, co, dtype=lr.C128)
    E = eng.forward(make(theta))
    g = eng.backward(theta.size)
    assert abs(E - E_ref) <= 1e-10
    np.testing.assert_allclose(g, g_ref, atol=1e-9)


def test_gradient_store_all_matches_rerun(lr):
    """Keeping every channel's input and record (the default budget) and re-running each layer
    in the reverse sweep (store_all_bytes=0) give bit-identical energies and gradients, both
    matching the oracle; the first layer ends with gates, so its reverse sweep starts from the
    restored checkpoint of the next layer."""
    from paper_2009_06657_amd.adjoint import EnergyGradient

    _say("energy_grad store-all vs re-run")
    n, r = 6, 4
    rng = np.random.default_rng(21)
    theta = rng.uniform(-np.pi, np.pi, size=5)
    xm, zm, co, _ = C.random_pauli_sum(n, terms=20, max_weight=3, seed=21)

    def make(t):
        ops = [C.Gate((0,), C.H, False, "h"),
               C.Gate((1,), C.rx(t[0]), False, "rx", (0, "X")),
               C.Kraus(1, C.amplitude_damping(0.2), "ad"), C.Compress(r, 0.0, 0, 1),
               C.Gate((2,), C.ry(t[1]), False, "ry", (1, "Y")),
               C.Gate((1, 2), C.CZ, True, "cz"),
               C.Gate((0,), C.rz(t[2]), False, "rz", (2, "Z")),
               C.LayerEnd(0),
               C.Kraus(0, C.depolarizing(0.1), "dep"), C.Compress(r, 0.0, 0, 1),
               C.Gate((3,), C.rx(t[3]), False, "rx", (3, "X")),
               C.Kraus(3, C.phase_flip(0.15), "deph"), C.Compress(r, 0.0, 0, 1),
               C.Gate((4,), C.ry(t[4]), False, "ry", (4, "Y")),
               C.LayerEnd(1)]
        return C.Program(n, ops, r, "c128", 4, "mixed", 2)

    E_ref, g_ref = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    keep = EnergyGradient(n, r, 4, xm, zm, co, dtype=lr.C128)
    rerun = EnergyGradient(n, r, 4, xm, zm, co, dtype=lr.C128, store_all_bytes=0)
    Ea = keep.forward(make(theta))
    ga = keep.backward(theta.size)
    Eb = rerun.forward(make(theta))
    gb = rerun.backward(theta.size)
    assert keep._all and not rerun._all
    assert Ea == Eb and np.array_equal(ga, gb)
    assert abs(Ea - E_ref) <= 1e-10
    np.testing.assert_allclose(ga, g_ref, atol=1e-9)
    keep.close()
    rerun.close()


def test_ansatz_full_size_against_finite_differences(lr):
    """n=12, r=16, 8 layers, 200 Pauli terms, complex64 bulk: energy and all 192 derivatives
    against the oracle's central differences (h = 1e-4) stored in tests/golden/cfg4_grad.json."""
    from paper_2009_06657_amd.adjoint import EnergyGradient

    with open(GOLDEN) as f:
        gold = json.load(f)
    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    _say("energy_grad n=12 r=16 8 layers")
    eng = EnergyGradient(12, 16, 4, xm, zm, co, dtype=lr.C64)
    E = eng.forward(C.cfg4_program(theta))
    g = eng.backward(theta.size)
    err_e = abs(E - gold["energy"])
    err_g = np.max(np.abs(g - np.array(gold["grad_fd"])))
    _say(f"  |dE| {err_e:.2e}  max|dg| vs FD {err_g:.2e}")
    assert err_e <= 1e-5
    assert err_g <= 1e-4


def test_autograd_function(lr):
    import torch

    from paper_2009_06657_amd.adjoint import EnergyGradient, make_noisy_energy

    _say("autograd function")
    n, r, layers = 5, 4, 2
    theta, xm, zm, co = _small_problem(13, n, layers)
    make = lambda t: C.cfg4_program(t, n=n, r=r, p=0.02, dtype="c128")  # noqa: E731
    eng = EnergyGradient(n, r, 4, xm, zm, co, dtype=lr.C128)
    NoisyEnergy = make_noisy_energy()
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    E = NoisyEnergy.apply(th, eng, make)
    (2.0 * E).backward()
    E_ref, g_ref = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    assert abs(float(E) - E_ref) <= 1e-10
    np.testing.assert_allclose(th.grad.numpy().reshape(-1), 2.0 * g_ref, atol=2e-9)
