"""Seeded synthetic circuit programs shared by the oracle, the tests and the benchmark.

This module only *describes* inputs: gate matrices, Kraus sets and the order of operations.
It performs none of the low-rank method's arithmetic (no gate application, no Gram matrix,
no eigensolve, no truncation); both the CPU oracle and the GPU library consume the same
``Program`` objects.

Conventions (readings of the paper where it is silent):
  * Qubit q is bit q of the basis index x (little-endian).
  * A k-qubit gate on ``qubits=(q0, q1)`` is a 2^k x 2^k matrix whose local index is
    ``i = b(q0) + 2*b(q1)``.
  * R_P(theta) = exp(-i theta P / 2); CZ = diag(1,1,1,-1); CNOT(c -> t) with qubits=(c, t).
  * Kraus operators are passed with their probabilities folded in, E_a = sqrt(p_a) K_a
    (Eq. "low rank evolution K", Sec. II.A).
  * Channels: depolarizing and bit/phase flip as defined in Sec. III.A.1 and III.A.3;
    amplitude damping with the daggers restored, rho -> E0 rho E0^H + E1 rho E1^H (Sec. III.A.3).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ----------------------------------------------------------------------------------------------
# Program IR
# ----------------------------------------------------------------------------------------------


@dataclasses.dataclass
class Gate:
    qubits: Tuple[int, ...]
    u: np.ndarray  # (2^k, 2^k) complex128
    diagonal: bool = False
    name: str = ""
    param: Optional[Tuple[int, str]] = None  # (angle index, axis) for parametrised rotations


@dataclasses.dataclass
class DiagWeight:
    """L[x,:] *= phase[popcount(x)]; phase has n+1 unit-modulus entries."""
    phase: np.ndarray


@dataclasses.dataclass
class Kraus:
    qubit: int
    ops: np.ndarray  # (m, 2, 2) complex128, E_a = sqrt(p_a) K_a; (m, 4, 4) with qubit2
    name: str = ""
    qubit2: int = -1  # second qubit of a two-qubit channel (local index b(qubit) + 2 b(qubit2))

    @property
    def qubits(self) -> Tuple[int, ...]:
        return (self.qubit,) if self.qubit2 < 0 else (self.qubit, self.qubit2)


@dataclasses.dataclass
class Compress:
    r: int
    eps: float = 0.0
    tie: int = 0      # 0 = plain (eigensolver order), 1 = cluster (gap-separated cut)
    renorm: int = 1   # 1 = rescale kept eigenvalues to unit trace


@dataclasses.dataclass
class LayerEnd:
    """Marks the end of one noisy circuit layer (gates + channels); carries no arithmetic."""
    index: int


@dataclasses.dataclass
class Program:
    n: int
    ops: list
    r: int
    dtype: str = "c64"        # bulk precision: "c64" complex FP32, "c128" complex FP64
    m_max: int = 4
    name: str = ""
    layers: int = 0
    meta: dict = dataclasses.field(default_factory=dict)
    # initial state: None = |0...0>; else (indices, amplitudes) of a sparse superposition
    # sum_i a_i |x_i> (unit norm), the other initial states Algorithm 1 admits (Sec. II.D)
    init: Optional[Tuple[np.ndarray, np.ndarray]] = None

    def n_compress(self) -> int:
        return sum(isinstance(o, Compress) for o in self.ops)


# ----------------------------------------------------------------------------------------------
# Gate and channel matrices (inputs; definitions only)
# ----------------------------------------------------------------------------------------------

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def rx(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(theta: float) -> np.ndarray:
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(theta: float) -> np.ndarray:
    return np.array([[np.exp(-0.5j * theta), 0], [0, np.exp(0.5j * theta)]], dtype=np.complex128)


CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
# local index i = b(control) + 2*b(target): flip target when control is 1 -> swap i=1 and i=3
CNOT = np.array([[1, 0, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0], [0, 1, 0, 0]], dtype=np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def haar_su2(rng: np.random.Generator) -> np.ndarray:
    """Uniform point (a, b) on S^3 from a normalised 4-d Gaussian; U = [[a, -b*], [b, a*]]."""
    g = rng.standard_normal(4)
    g /= np.linalg.norm(g)
    a = g[0] + 1j * g[1]
    b = g[2] + 1j * g[3]
    return np.array([[a, -np.conj(b)], [b, np.conj(a)]], dtype=np.complex128)


def depolarizing(p: float) -> np.ndarray:
    """(1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z)  (Sec. III.A.1)."""
    return np.stack([np.sqrt(1 - p) * I2, np.sqrt(p / 3) * X, np.sqrt(p / 3) * Y, np.sqrt(p / 3) * Z])


def bit_flip(p: float) -> np.ndarray:
    """(1-p) rho + p X rho X  (Sec. III.A.3)."""
    return np.stack([np.sqrt(1 - p) * I2, np.sqrt(p) * X])


def phase_flip(p: float) -> np.ndarray:
    """(1-p) rho + p Z rho Z: the U = Z member of the anisotropic family of Sec. III.A.3.
    Used as the reading of 'dephasing p'."""
    return np.stack([np.sqrt(1 - p) * I2, np.sqrt(p) * Z])


def amplitude_damping(g: float) -> np.ndarray:
    """E0 = diag(1, sqrt(1-g)), E1 = [[0, sqrt(g)], [0, 0]]  (Sec. III.A.3)."""
    e0 = np.array([[1, 0], [0, np.sqrt(1 - g)]], dtype=np.complex128)
    e1 = np.array([[0, np.sqrt(g)], [0, 0]], dtype=np.complex128)
    return np.stack([e0, e1])


PAULI_LIST = (I2, X, Y, Z)


def depolarizing2(p: float) -> np.ndarray:
    """Two-qubit depolarizing channel (1-p) rho + p/15 sum_{P != I (x) I} P rho P over the 15
    non-identity two-qubit Pauli products (16 Kraus operators, 4 x 4, local index b(q0) +
    2 b(q1))."""
    ops = []
    for a in range(4):
        for b in range(4):
            w = np.sqrt(1 - p) if (a == 0 and b == 0) else np.sqrt(p / 15)
            ops.append(w * np.kron(PAULI_LIST[b], PAULI_LIST[a]))
    return np.stack(ops)


def correlated_dephasing(p: float) -> np.ndarray:
    """(1-p) rho + p (Z (x) Z) rho (Z (x) Z): a two-qubit channel with two Kraus operators."""
    return np.stack([np.sqrt(1 - p) * np.eye(4, dtype=np.complex128), np.sqrt(p) * np.kron(Z, Z)])


def grouped_channel(ops0: np.ndarray, ops1: np.ndarray) -> np.ndarray:
    """The product of a channel on q0 and one on q1 as a single two-qubit Kraus set
    {E_a (x) F_b} (Sec. II.C: a Kraus layer decomposed into groups of M = 2 qubits, truncated
    once per group); local index b(q0) + 2 b(q1), so the matrix of E (on q0) and F (on q1) is
    kron(F, E)."""
    return np.stack([np.kron(F, E) for E in ops0 for F in ops1])


def ghz_init(n: int):
    """(|0...0> + |1...1>) / sqrt(2) as a sparse initial state."""
    return (np.array([0, 2 ** n - 1], dtype=np.uint64), np.array([1, 1], dtype=np.complex128) / np.sqrt(2.0))


def grover_oracle_phase(n: int, max_weight: int = 2) -> np.ndarray:
    """Phase -1 on basis states of Hamming weight <= max_weight (the 'good' set of Sec. III.C)."""
    w = np.arange(n + 1)
    return np.where(w <= max_weight, -1.0, 1.0).astype(np.complex128)


def zero_flip_phase(n: int) -> np.ndarray:
    """Phase -1 on |0...0> only (the reflection inside the diffusion operator)."""
    ph = np.ones(n + 1, dtype=np.complex128)
    ph[0] = -1.0
    return ph


# ----------------------------------------------------------------------------------------------
# Program builders
# ----------------------------------------------------------------------------------------------


def _g1(q, u, name="", param=None):
    return Gate((q,), np.asarray(u, dtype=np.complex128), False, name, param)


def _g2(q0, q1, u, name="", diagonal=False):
    return Gate((q0, q1), np.asarray(u, dtype=np.complex128), diagonal, name)


def brickwork_program(n: int, layers: int, r: int, channels: Sequence[Tuple[str, float]],
                      seed: int, dtype: str = "c64", eps: float = 0.0, tie: int = 0,
                      renorm: int = 1, name: str = "brickwork") -> Program:
    """Layer l: Haar SU(2) on every qubit, then CZ on (2i, 2i+1) for even l or (2i+1, 2i+2) for
    odd l (open boundary); then for each qubit in ascending order, each listed channel followed
    by a compression to rank r."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list = []
    for l in range(layers):
        for q in range(n):
            ops.append(_g1(q, haar_su2(rng), "su2"))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            ops.append(_g2(a, a + 1, CZ, "cz", diagonal=True))
        for q in range(n):
            for ch, p in channels:
                ops.append(Kraus(q, _channel(ch, p), ch))
                ops.append(Compress(r, eps, tie, renorm))
        ops.append(LayerEnd(l))
    m_max = max(_channel(ch, p).shape[0] for ch, p in channels) if channels else 1
    return Program(n, ops, r, dtype, m_max, name, layers)


def grouped_brickwork_program(n: int, layers: int, r: int, channel: str, p: float, seed: int,
                              dtype: str = "c64", eps: float = 0.0, tie: int = 0, renorm: int = 1,
                              two_qubit: str = "") -> Program:
    """Brickwork gates as in brickwork_program, then the layer's noise in groups of M = 2
    qubits (q, q+1) for q = 0, 2, 4, ...: the product of the one-qubit channel on both qubits as
    one two-qubit Kraus set, followed by one compression per group (Sec. II.C).  With two_qubit
    = "dep2" or "zz", that two-qubit channel replaces the product on each pair."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list = []
    one = _channel(channel, p) if channel else None
    m_max = 1
    for l in range(layers):
        for q in range(n):
            ops.append(_g1(q, haar_su2(rng), "su2"))
        start = 0 if l % 2 == 0 else 1
        for a in range(start, n - 1, 2):
            ops.append(_g2(a, a + 1, CZ, "cz", diagonal=True))
        for q in range(0, n - 1, 2):
            if two_qubit == "dep2":
                ks = depolarizing2(p)
            elif two_qubit == "zz":
                ks = correlated_dephasing(p)
            else:
                ks = grouped_channel(one, one)
            m_max = max(m_max, ks.shape[0])
            ops.append(Kraus(q, ks, two_qubit or f"{channel}x{channel}", q + 1))
            ops.append(Compress(r, eps, tie, renorm))
        if n % 2 == 1 and one is not None:
            ops.append(Kraus(n - 1, one, channel))
            ops.append(Compress(r, eps, tie, renorm))
        ops.append(LayerEnd(l))
    return Program(n, ops, r, dtype, m_max, "grouped-brickwork", layers,
                   {"channel": channel, "p": p, "two_qubit": two_qubit})


GATES_1Q = ("X", "Y", "Z", "S", "T", "RX", "RY", "RZ")
GATES_2Q = ("SWAP", "CZ", "CNOT")
CIRCUIT_KINDS = ("dense-local", "dense-global", "sparse-local")


def random_circuit(n: int, depth: int, kind: str = "dense-local", channel: str = "dep",
                   p: float = 0.001, r: int = 32, eps: float = 1e-4, seed: int = 0,
                   dtype: str = "c64", sparsity: float = 0.5, tie: int = 0, renorm: int = 1,
                   noise: bool = True) -> Program:
    """Randomized-benchmarking circuits (Sec. III.A): gates drawn uniformly from X, Y, Z, S, T,
    RX, RY, RZ (angles U(0, 2 pi)) and SWAP, CZ, CNOT (random control/target order), a 1- or a
    2-qubit gate with equal probability at every placement.  Time step t walks the qubits in
    ascending order; a qubit not yet used in the step gets a 2-qubit gate with probability 1/2
    when a partner is free (dense-local / sparse-local: the next qubit; dense-global: any free
    qubit), else a 1-qubit gate.  Dense circuits place a gate on every qubit at every step; in
    sparse ones a free qubit starts no gate with probability sparsity (it can still be taken as
    the partner of the qubit before it).  Noise: the channel on
    every qubit after each step (dense) or only on the qubits a gate touched (sparse), each
    followed by a compression (rank cap r, threshold eps).  noise=False gives the same gates
    without channels (the noiseless reference)."""
    if kind not in CIRCUIT_KINDS:
        raise ValueError(f"kind must be one of {CIRCUIT_KINDS}")
    rng = np.random.Generator(np.random.PCG64(seed))
    one = {"X": X, "Y": Y, "Z": Z, "S": S, "T": T}
    ops: list = []
    for t in range(depth):
        free = set(range(n))
        touched = []
        for q in range(n):
            if q not in free:
                continue
            if kind.startswith("sparse") and rng.random() < sparsity:
                continue
            free.discard(q)
            partner = -1
            if rng.random() < 0.5:
                if kind.endswith("local"):
                    partner = q + 1 if (q + 1) in free else -1
                else:
                    cand = sorted(free)
                    partner = int(cand[rng.integers(len(cand))]) if cand else -1
            if partner >= 0:
                free.discard(partner)
                g = GATES_2Q[int(rng.integers(len(GATES_2Q)))]
                a, b = (q, partner) if rng.random() < 0.5 else (partner, q)
                if g == "SWAP":
                    ops.append(_g2(a, b, SWAP, "swap"))
                elif g == "CZ":
                    ops.append(_g2(a, b, CZ, "cz", diagonal=True))
                else:
                    ops.append(_g2(a, b, CNOT, "cnot"))
                touched += [q, partner]
            else:
                g = GATES_1Q[int(rng.integers(len(GATES_1Q)))]
                if g in one:
                    ops.append(_g1(q, one[g], g.lower()))
                else:
                    theta = float(rng.uniform(0.0, 2.0 * np.pi))
                    ops.append(_g1(q, {"RX": rx, "RY": ry, "RZ": rz}[g](theta), g.lower()))
                touched.append(q)
        if noise:
            for q in (sorted(touched) if kind.startswith("sparse") else range(n)):
                for ks in _channels(channel, p):
                    ops.append(Kraus(q, ks, channel))
                    ops.append(Compress(r, eps, tie, renorm))
        ops.append(LayerEnd(t))
    m_max = max(ks.shape[0] for ks in _channels(channel, p)) if noise else 1
    return Program(n, ops, r, dtype, m_max, f"random-{kind}", depth,
                   {"kind": kind, "channel": channel, "p": p, "eps": eps, "seed": seed})


def _channel(ch: str, p: float) -> np.ndarray:
    return {"dep": depolarizing, "bitflip": bit_flip, "deph": phase_flip,
            "ad": amplitude_damping}[ch](p)


def pauli_flip(P: np.ndarray, a: float) -> np.ndarray:
    """(1 - a) rho + a P rho P for a Pauli P."""
    return np.stack([np.sqrt(1 - a) * I2, np.sqrt(a) * P])


def depolarizing_as_flips(p: float) -> List[np.ndarray]:
    """The depolarizing channel as three two-operator channels, X, Y and Z flips with the same
    probability a.  Pauli channels compose by multiplying their Pauli eigenvalues: a flip about P
    keeps P and scales the two others by 1 - 2a, so the three flips scale each of X, Y, Z by
    (1 - 2a)^2; depolarizing scales each by 1 - 4p/3, hence a = (1 - sqrt(1 - 4p/3)) / 2."""
    a = 0.5 * (1.0 - np.sqrt(1.0 - 4.0 * p / 3.0))
    return [pauli_flip(X, a), pauli_flip(Y, a), pauli_flip(Z, a)]


def _channels(ch: str, p: float) -> List[np.ndarray]:
    """The channel as a list of Kraus sets applied in turn, each followed by a compression:
    "dep3" is depolarizing written as three flips (two operators each, so a rank cap up to 64
    fits the order-128 eigensolver; three truncations instead of one)."""
    if ch == "dep3":
        return depolarizing_as_flips(p)
    return [_channel(ch, p)]


def cfg1_program(n: int = 6, r: int = 13, layers: int = 20, p: float = 0.0033, seed: int = 1001,
                 dtype: str = "c128", renorm: int = 1) -> Program:
    """Haar SU(2) on every qubit, CNOT ladder 0->1->...->n-1, depolarizing after each layer on
    every qubit with a compression after each channel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ops: list = []
    for l in range(layers):
        for q in range(n):
            ops.append(_g1(q, haar_su2(rng), "su2"))
        for q in range(n - 1):
            ops.append(_g2(q, q + 1, CNOT, "cnot"))
        for q in range(n):
            ops.append(Kraus(q, depolarizing(p), "dep"))
            ops.append(Compress(r, 0.0, 0, renorm))
        ops.append(LayerEnd(l))
    return Program(n, ops, r, dtype, 4, "cfg1", layers, {"outputs": ["probs", "z"]})


def cfg2_program(n: int = 14, r: int = 32, iterations: int = 6, p: float = 0.001,
                 dtype: str = "c64", tie: int = 1, renorm: int = 1) -> Program:
    """Grover search for states of Hamming weight <= 2 (Sec. III.C): [H^n] followed by
    `iterations` x [oracle, H^n, |0..0> flip, H^n]; every one of these layers is followed by
    depolarizing noise on every qubit with a compression after each channel."""
    ops: list = []
    layer = 0

    def hlayer():
        for q in range(n):
            ops.append(_g1(q, H, "h"))

    def noise():
        nonlocal layer
        if p > 0:
            for q in range(n):
                ops.append(Kraus(q, depolarizing(p), "dep"))
                ops.append(Compress(r, 0.0, tie, renorm))
        ops.append(LayerEnd(layer))
        layer += 1

    hlayer(); noise()
    for _ in range(iterations):
        ops.append(DiagWeight(grover_oracle_phase(n))); noise()
        hlayer(); noise()
        ops.append(DiagWeight(zero_flip_phase(n))); noise()
        hlayer(); noise()
    return Program(n, ops, r, dtype, 4, "cfg2", layer, {"outputs": ["probs"]})


def cfg3_program(n: int = 20, r: int = 64, layers: int = 40, gamma: float = 0.002,
                 p_deph: float = 0.001, seed: int = 1003, dtype: str = "c64") -> Program:
    """Random brickwork; amplitude damping then dephasing on every qubit, compressing after
    each channel."""
    prog = brickwork_program(n, layers, r, [("ad", gamma), ("deph", p_deph)], seed, dtype,
                             name="cfg3")
    prog.m_max = 2
    prog.meta["outputs"] = ["zz", "samples"]
    prog.meta["samples"] = 10_000
    prog.meta["sample_seed"] = 3003
    return prog


def cfg4_angles(n: int = 12, layers: int = 8, seed: int = 1004) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-np.pi, np.pi, size=(layers, n, 2))


def cfg4_program(theta: np.ndarray, n: int = 12, r: int = 16, p: float = 0.002,
                 dtype: str = "c64", renorm: int = 1) -> Program:
    """Layer l: RY(theta[l,q,0]) then RZ(theta[l,q,1]) on every qubit (emitted as the RY layer
    followed by the RZ layer, the same unitary since gates on different qubits commute), CZ
    ladder (q, q+1), depolarizing on every qubit with a compression after each channel."""
    layers = theta.shape[0]
    ops: list = []
    for l in range(layers):
        for q in range(n):
            ops.append(_g1(q, ry(theta[l, q, 0]), "ry", ((l * n + q) * 2 + 0, "Y")))
        for q in range(n):
            ops.append(_g1(q, rz(theta[l, q, 1]), "rz", ((l * n + q) * 2 + 1, "Z")))
        for q in range(n - 1):
            ops.append(_g2(q, q + 1, CZ, "cz", diagonal=True))
        for q in range(n):
            ops.append(Kraus(q, depolarizing(p), "dep"))
            ops.append(Compress(r, 0.0, 0, renorm))
        ops.append(LayerEnd(l))
    return Program(n, ops, r, dtype, 4, "cfg4", layers, {"outputs": ["energy", "grad"]})


def random_pauli_sum(n: int, terms: int = 200, max_weight: int = 4, seed: int = 1004):
    """Distinct Pauli strings: weight ~ U{1..max_weight}, support uniform without replacement,
    factors uniform in {X, Y, Z}, coefficients N(0, 1).  Returns (xmask, zmask, coeff, labels)
    with Y = both bits set."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    seen = set()
    xs, zs, cs, labels = [], [], [], []
    while len(xs) < terms:
        w = int(rng.integers(1, max_weight + 1))
        support = rng.choice(n, size=w, replace=False)
        kinds = rng.integers(0, 3, size=w)
        xm = zm = 0
        lab = ["I"] * n
        for q, k in zip(support, kinds):
            ch = "XYZ"[k]
            lab[q] = ch
            if ch in "XY":
                xm |= 1 << int(q)
            if ch in "YZ":
                zm |= 1 << int(q)
        if (xm, zm) in seen:
            continue
        seen.add((xm, zm))
        xs.append(xm); zs.append(zm); cs.append(float(rng.standard_normal())); labels.append("".join(lab))
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
            np.array(cs, dtype=np.float64), labels)


def cfg5_instances(count: int = 256, base_seed: int = 5000):
    """Uneven serving mix: n ~ U{8..16}, r ~ U{8,16,32}, depth ~ U{10..30}, p ~ U(1e-4, 5e-3)."""
    progs = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + i))
        n = int(rng.integers(8, 17))
        r = int(rng.choice([8, 16, 32]))
        depth = int(rng.integers(10, 31))
        p = float(rng.uniform(1e-4, 5e-3))
        prog = brickwork_program(n, depth, r, [("dep", p)], base_seed + 100000 + i, "c64",
                                 name=f"cfg5[{i}]")
        prog.meta["outputs"] = ["z"]
        progs.append(prog)
    return progs


def sample_uniforms(count: int, seed: int) -> np.ndarray:
    """Uniforms in [0, 1) consumed by inverse-CDF sampling on both sides."""
    return np.random.Generator(np.random.PCG64(seed)).random(count)


def random_orthogonal_factor(n: int, r: int, seed: int, decay: float = 0.9) -> np.ndarray:
    """A unit-trace factor L (2^n x r) with orthogonal columns and geometrically decaying column
    norms: a steady-state-like input for timing and for set_L tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((2 ** n, r)) + 1j * rng.standard_normal((2 ** n, r))
    q, _ = np.linalg.qr(a)
    w = decay ** np.arange(r)
    w = w / w.sum()
    return q * np.sqrt(w)[None, :]
