"""Pins for the oracle's energy gradients (oracle/grad.py): the reverse sweep against central
finite differences, against the exact parameter-shift rule when nothing is truncated, and the
truncation adjoint against a directional difference of a single compression."""
import numpy as np
import pytest

from oracle import grad as OG
from oracle.lret import compress
from workloads import circuits as C


def _hermitian(rng, d):
    a = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    return a + a.conj().T


@pytest.mark.parametrize("renorm", [0, 1])
@pytest.mark.parametrize("r", [1, 3, 5])
def test_compress_adjoint_directional_difference(renorm, r):
    rng = np.random.default_rng(11 + r + 10 * renorm)
    A = rng.standard_normal((16, 6)) + 1j * rng.standard_normal((16, 6))
    A /= np.linalg.norm(A)
    H = _hermitian(rng, 16)
    dA = rng.standard_normal(A.shape) + 1j * rng.standard_normal(A.shape)
    dA /= np.linalg.norm(dA)

    def loss(X):
        Ln, _ = compress(X, r, renorm=renorm)
        return float(np.real(np.vdot(Ln, H @ Ln)))

    Ln, _ = compress(A, r, renorm=renorm)
    Abar = OG.compress_adjoint(A, H @ Ln, r, renorm=renorm)
    analytic = 2 * np.real(np.vdot(Abar, dA))
    # central difference with one Richardson step: the O(h^2) term cancels
    d = lambda h: (loss(A + h * dA) - loss(A - h * dA)) / (2 * h)  # noqa: E731
    h = 1e-3
    fd = (4 * d(h / 2) - d(h)) / 3
    assert abs(analytic - fd) <= 1e-8 * max(1.0, abs(fd))


def _small_problem(seed, n=4, layers=2):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-np.pi, np.pi, size=(layers, n, 2))
    xm, zm, co, _ = C.random_pauli_sum(n, terms=12, max_weight=3, seed=seed)
    return theta, xm, zm, co


@pytest.mark.parametrize("renorm", [0, 1])
def test_adjoint_matches_central_differences_with_truncation(renorm):
    theta, xm, zm, co = _small_problem(3)
    make = lambda t: C.cfg4_program(t, n=4, r=3, p=0.05, renorm=renorm)  # noqa: E731
    E, g = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    assert abs(E - OG.energy(make(theta), xm, zm, co)) < 1e-13
    fd = OG.energy_grad_fd(make, theta, xm, zm, co, h=1e-4)
    np.testing.assert_allclose(g, fd, atol=1e-7)
    assert np.max(np.abs(g)) > 1e-2   # not trivially zero


def test_adjoint_with_fixed_gates_amplitude_damping_and_weights():
    """Non-unital channel, fixed 1q/2q gates, a Hamming-weight phase, and RX/RY/RZ angles."""
    n, r = 3, 2
    rng = np.random.default_rng(8)
    theta = rng.uniform(-np.pi, np.pi, size=6)
    xm, zm, co, _ = C.random_pauli_sum(n, terms=8, max_weight=2, seed=8)
    phase = np.exp(1j * rng.uniform(0, 2 * np.pi, size=n + 1))

    def make(t):
        ops = [C.Gate((0,), C.H, False, "h"),
               C.Gate((1,), C.rx(t[0]), False, "rx", (0, "X")),
               C.Gate((2,), C.ry(t[1]), False, "ry", (1, "Y")),
               C.Gate((0, 1), C.CNOT, False, "cnot"),
               C.DiagWeight(phase),
               C.Kraus(1, C.amplitude_damping(0.2), "ad"), C.Compress(r, 0.0, 0, 1),
               C.Gate((0,), C.rz(t[2]), False, "rz", (2, "Z")),
               C.Gate((1, 2), C.CZ, True, "cz"),
               C.Gate((2,), C.rx(t[3]), False, "rx", (3, "X")),
               C.Kraus(2, C.depolarizing(0.1), "dep"), C.Compress(r, 0.0, 0, 1),
               C.Gate((0,), C.ry(t[4]), False, "ry", (4, "Y")),
               C.Gate((2, 0), C.SWAP, False, "swap"),
               C.Gate((1,), C.rz(t[5]), False, "rz", (5, "Z")),
               C.Kraus(0, C.phase_flip(0.15), "deph"), C.Compress(r, 0.0, 0, 1)]
        return C.Program(n, ops, r, "c128", 4, "mixed", 1)

    E, g = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    fd = OG.energy_grad_fd(make, theta, xm, zm, co, h=1e-4)
    np.testing.assert_allclose(g, fd, atol=1e-7)


def test_parameter_shift_is_exact_without_truncation():
    """With r = 2^n >= rank no eigenvalue mass is discarded, the map from any gate's output to E is
    linear in rho, and [E(t + pi/2) - E(t - pi/2)] / 2 is the exact derivative."""
    theta, xm, zm, co = _small_problem(21, n=3, layers=2)
    make = lambda t: C.cfg4_program(t, n=3, r=8, p=0.03)  # noqa: E731
    _, g = OG.energy_grad_adjoint(make(theta), theta.size, xm, zm, co)
    ps = OG.parameter_shift(make, theta, xm, zm, co, range(theta.size))
    np.testing.assert_allclose(g, ps, atol=1e-10)


def test_adjoint_at_full_ansatz_size_on_sampled_angles():
    """The n=12, r=16, 8-layer ansatz with the 200-term Hamiltonian: two angles (first, last)."""
    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    _, g = OG.energy_grad_adjoint(C.cfg4_program(theta), theta.size, xm, zm, co)
    idx = [0, theta.size - 1]
    fd = OG.energy_grad_fd(lambda t: C.cfg4_program(t), theta, xm, zm, co, h=1e-4, indices=idx)
    np.testing.assert_allclose(g[idx], fd[idx], atol=1e-7)
