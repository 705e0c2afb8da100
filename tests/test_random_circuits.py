"""The randomized-benchmarking circuit generator (Sec. III.A) and the oracle on its circuits, on
the CPU: structure of dense / sparse and local / global circuits, the gate set, determinism;
LRET equals the full-rank evolution when nothing is truncated, and the distortion (Sec. III)
vanishes without truncation and grows with the threshold."""
import numpy as np
import pytest

import oracle
from oracle import fdm as ofdm
from oracle.observables import distortion
from workloads import circuits as C


def _steps(prog):
    steps, cur = [], []
    for op in prog.ops:
        if isinstance(op, C.LayerEnd):
            steps.append(cur)
            cur = []
        else:
            cur.append(op)
    return steps


@pytest.mark.parametrize("kind", C.CIRCUIT_KINDS)
def test_structure(kind):
    n, depth = 9, 40
    prog = C.random_circuit(n, depth, kind, "bitflip", 0.001, 16, 1e-4, seed=11)
    steps = _steps(prog)
    assert len(steps) == depth
    n1 = n2 = nonadj = 0
    touched_total = 0
    for ops in steps:
        gates = [o for o in ops if isinstance(o, C.Gate)]
        chans = [o for o in ops if isinstance(o, C.Kraus)]
        comps = [o for o in ops if isinstance(o, C.Compress)]
        qs = [q for g in gates for q in g.qubits]
        assert len(qs) == len(set(qs))                        # one gate per qubit per step
        touched_total += len(qs)
        if kind.startswith("dense"):
            assert sorted(qs) == list(range(n))
            assert [c.qubit for c in chans] == list(range(n))
        else:
            assert [c.qubit for c in chans] == sorted(qs)      # noise only after gates
        assert len(comps) == len(chans)
        for g in gates:
            u = g.u
            assert np.allclose(u.conj().T @ u, np.eye(u.shape[0]), atol=1e-12)
            if len(g.qubits) == 2:
                n2 += 1
                nonadj += abs(g.qubits[0] - g.qubits[1]) != 1
            else:
                n1 += 1
    if kind.endswith("local"):
        assert nonadj == 0
    else:
        assert nonadj > 0
    if kind.startswith("sparse"):
        frac = touched_total / (n * depth)
        assert 0.45 < frac < 0.8
    # equal probability of a 1- or 2-qubit gate at each placement (2q placements can fail
    # for want of a partner, so 1q gates are somewhat more frequent)
    assert n2 > 0.25 * (n1 + n2)


def test_gate_set_and_determinism():
    a = C.random_circuit(8, 30, "dense-global", "dep", 0.001, 16, 1e-4, seed=4)
    b = C.random_circuit(8, 30, "dense-global", "dep", 0.001, 16, 1e-4, seed=4)
    names = {g.name for g in a.ops if isinstance(g, C.Gate)}
    assert names == {"x", "y", "z", "s", "t", "rx", "ry", "rz", "swap", "cz", "cnot"}
    assert len(a.ops) == len(b.ops)
    for x, y in zip(a.ops, b.ops):
        assert type(x) is type(y)
        if isinstance(x, C.Gate):
            assert x.qubits == y.qubits and np.array_equal(x.u, y.u)
    quiet = C.random_circuit(8, 30, "dense-global", "dep", 0.001, 16, 1e-4, seed=4, noise=False)
    ga = [g for g in a.ops if isinstance(g, C.Gate)]
    gq = [g for g in quiet.ops if isinstance(g, C.Gate)]
    assert len(ga) == len(gq) and all(np.array_equal(x.u, y.u) for x, y in zip(ga, gq))
    assert not any(isinstance(o, (C.Kraus, C.Compress)) for o in quiet.ops)


@pytest.mark.parametrize("kind", C.CIRCUIT_KINDS)
@pytest.mark.parametrize("channel", ["dep", "bitflip", "ad"])
def test_lret_equals_fdm_without_truncation(kind, channel):
    """r = 2^n and eps = 0: every compression keeps the whole spectrum."""
    n = 4
    prog = C.random_circuit(n, 4, kind, channel, 0.05, 2 ** n, 0.0, seed=5)
    rho = ofdm.run_fdm(prog)
    L = oracle.run_lret(prog)
    assert np.max(np.abs(L @ L.conj().T - rho)) < 1e-12


def test_distortion_vanishes_and_grows():
    n, depth = 6, 8
    base = dict(n=n, depth=depth, kind="dense-local", channel="dep", p=0.01, r=2 ** n, seed=9)
    exact = np.real(np.diag(ofdm.run_fdm(C.random_circuit(eps=0.0, **base))))
    quiet = np.real(np.diag(ofdm.run_fdm(C.random_circuit(eps=0.0, noise=False, **base))))
    d = []
    for eps in (0.0, 1e-4, 1e-3, 1e-2):
        P = oracle.probabilities(oracle.run_lret(C.random_circuit(eps=eps, **base)))
        d.append(distortion(P, exact, quiet))
    assert d[0] < 1e-10
    assert 0 < d[1] <= d[2] <= d[3]


def test_accuracy_host_logic():
    """Host side of the GPU distortion studies: the ratio matches the oracle's definition
    (Sec. III, Eq. "distortion"), is undefined (NaN) when noise leaves the diagonal unchanged, and
    the noiseless program keeps every gate, phase and layer marker in order while dropping the
    channels and compressions."""
    from oracle.observables import distortion as distortion_ref
    from paper_2009_06657_amd import accuracy as A

    rng = np.random.default_rng(3)
    a, b, c = (rng.dirichlet(np.ones(32)) for _ in range(3))
    assert abs(A.distortion(a, b, c) - distortion_ref(a, b, c)) <= 1e-15
    assert np.isnan(A.distortion(a, b, b))
    prog = C.random_circuit(5, 4, "sparse-local", "ad", p=0.01, r=8, eps=1e-4, seed=9)
    clean = A.noiseless_program(prog)
    kept = [op for op in prog.ops if not isinstance(op, (C.Kraus, C.Compress))]
    assert clean.ops == kept and clean.n == prog.n and clean.layers == prog.layers
    assert not any(isinstance(op, (C.Kraus, C.Compress)) for op in clean.ops)
    assert sum(isinstance(op, C.LayerEnd) for op in clean.ops) == 4


def test_depolarizing_as_three_flips_is_exact():
    """The X, Y and Z flips with a = (1 - sqrt(1 - 4p/3)) / 2, applied in turn, are the
    depolarizing channel of Sec. III.A.1: the same map on random density matrices (FP64 oracle),
    and the dep3 circuits differ from dep ones only in the channel's Kraus sets."""
    from oracle.fdm import fdm_channel

    rng = np.random.default_rng(4)
    for p in (0.001, 0.01, 0.3):
        A = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        rho = A @ A.conj().T
        rho /= np.trace(rho).real
        want = fdm_channel(rho, 2, 1, C.depolarizing(p))
        got = rho
        for ks in C.depolarizing_as_flips(p):
            got = fdm_channel(got, 2, 1, ks)
        assert np.max(np.abs(got - want)) <= 1e-15
    a = C.random_circuit(4, 3, "dense-local", "dep", p=0.01, r=8, seed=2)
    b = C.random_circuit(4, 3, "dense-local", "dep3", p=0.01, r=8, seed=2)
    assert [o.u.tobytes() for o in a.ops if isinstance(o, C.Gate)] == [o.u.tobytes() for o in b.ops if isinstance(o, C.Gate)]
    assert sum(isinstance(o, C.Kraus) for o in b.ops) == 3 * sum(isinstance(o, C.Kraus) for o in a.ops)
    assert b.m_max == 2 and a.m_max == 4
