"""Energy gradients of a noisy parametrised circuit through the low-rank evolution, on the GPU.

The energy is E(theta) = sum_t c_t Tr(L^H P_t L) of the final factor (Sec. II.D).  The forward
pass runs the program through the C ABI with per-layer checkpoints of L; the reverse sweep then
walks the layers backwards: it restores the layer's checkpoint, re-runs the layer (deterministic
kernels reproduce it bit for bit) keeping each channel's input factor and the compression
record, and propagates the adjoint Lbar (dE = 2 Re Tr(Lbar^H dL)) through the layer in reverse:

  * a channel + compression by lrdm_compress_adjoint (FP64 eigenvector-derivative formula on the
    small Gram matrix, bulk-precision products over the 2^n rows);
  * a gate U by applying U^H to both Lbar and L; a rotation R_P(theta) = exp(-i theta P/2)
    contributes dE/dtheta = Im Tr(Lbar^H P L) taken right after the gate (lrdm_pauli_overlap).
    Derivatives of rotations whose generator commutes with every gate between them and the
    current point are evaluated together in one overlap call.

Memory: one checkpoint per layer plus one layer's channel inputs and records; when every channel's
input and record fit in store_all_bytes, the forward pass keeps them all and the reverse sweep
re-runs nothing (each layer starts from the next layer's checkpoint, which is bit-for-bit the
state the re-run would reach).  This module only orders calls into liblrdm; every step runs in
its kernels.
"""
from __future__ import annotations

from typing import Callable, List

import numpy as np

from .lrdm import LowRankDM

_PAULI = {
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def _masks(q: int, axis: str):
    xm = (1 << q) if axis in "XY" else 0
    zm = (1 << q) if axis in "YZ" else 0
    return xm, zm


def _split_layers(program) -> List[list]:
    from workloads.circuits import LayerEnd

    layers, cur = [], []
    for op in program.ops:
        if isinstance(op, LayerEnd):
            layers.append(cur)
            cur = []
        else:
            cur.append(op)
    if cur:
        layers.append(cur)
    return layers


class EnergyGradient:
    """Forward energy and reverse-sweep gradient for programs of one shape (n, r, m_max).

    make_program(theta) -> workloads.circuits.Program whose parametrised gates carry
    param = (index into theta.ravel(), axis)."""

    def __init__(self, n: int, r: int, m_max: int, xmask, zmask, coeff, dtype: int = 0,
                 device: str = "cuda:0", store_all_bytes: int = 8 << 30):
        import torch

        self.n, self.r, self.m_max = n, r, m_max
        self.dm = LowRankDM(n, r, dtype, m_max, device=device)
        self.bar = LowRankDM(n, r, dtype, m_max, device=device)
        self.xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        self.zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        self.coeff = np.ascontiguousarray(coeff, dtype=np.float64)
        self.rec_bytes = self.dm.record_bytes()
        self.state_bytes = self.dm.state.numel()
        self.device = torch.device(device)
        self.store_all_bytes = int(store_all_bytes)
        self._ckpt = None
        self._xbuf = None
        self._rec = None
        self._all = False
        self.program = None

    # ------------------------------------------------------------------ buffers
    def _ensure(self, n_layers: int, max_channels: int):
        import torch

        def grow(buf, count, nbytes):
            if buf is None or buf.shape[0] < count:
                return torch.empty((count, nbytes), dtype=torch.uint8, device=self.device)
            return buf

        self._ckpt = grow(self._ckpt, n_layers, self.state_bytes)
        self._xbuf = grow(self._xbuf, max(max_channels, 1), self.state_bytes)
        self._rec = grow(self._rec, max(max_channels, 1), self.rec_bytes)

    # ------------------------------------------------------------------ forward
    def _run_layer(self, ops, keep: bool, j0: int = 0):
        """Issue one layer; with keep=True save every channel's input and compression record
        (channel slots from j0 on)."""
        from workloads.circuits import Compress, DiagWeight, Gate, Kraus

        dm = self.dm
        j = j0
        for op in ops:
            if isinstance(op, Gate):
                dm.apply_gate(op.qubits, op.u)
            elif isinstance(op, DiagWeight):
                dm.apply_diagonal_weight(op.phase)
            elif isinstance(op, Kraus):
                if keep:
                    self._xrank[j] = dm.checkpoint(self._xbuf[j])
                dm.apply_kraus(op.qubit, op.ops)
            elif isinstance(op, Compress):
                dm.compress_record(op.r, self._rec[j], op.eps, op.tie, op.renorm)
                j += 1
            else:
                raise TypeError(f"unknown op {op!r}")

    def forward(self, program) -> float:
        from workloads.circuits import Compress, Kraus

        self.program = program
        self.layers = _split_layers(program)
        chans = [sum(isinstance(o, Kraus) for o in seg) for seg in self.layers]
        for seg in self.layers:
            for i, op in enumerate(seg):
                if isinstance(op, Compress) and (i == 0 or not isinstance(seg[i - 1], Kraus)):
                    raise NotImplementedError("the reverse sweep needs a Kraus channel before every compression")
        total = sum(chans)
        self._all = total * (self.state_bytes + self.rec_bytes) <= self.store_all_bytes
        slots = total if self._all else (max(chans) if chans else 1)
        self._ensure(len(self.layers), slots)
        self._xrank = [0] * max(slots, 1)
        self._ckrank = [0] * len(self.layers)
        self._j0 = [sum(chans[:l]) if self._all else 0 for l in range(len(self.layers))]
        dm = self.dm
        dm.reset()
        for l, seg in enumerate(self.layers):
            self._ckrank[l] = dm.checkpoint(self._ckpt[l])
            self._run_layer(seg, keep=self._all, j0=self._j0[l])
        self.energy = dm.expect_pauli(self.xm, self.zm, self.coeff, summed=True)
        return self.energy

    # ------------------------------------------------------------------ reverse sweep
    @staticmethod
    def _commutes(op, q: int, axis: str) -> bool:
        from workloads.circuits import DiagWeight

        if isinstance(op, DiagWeight):
            return axis == "Z"
        if q not in op.qubits:
            return True
        if len(op.qubits) == 1:
            u = np.asarray(op.u)
            P = _PAULI[axis]
            return bool(np.max(np.abs(u @ P - P @ u)) < 1e-12)
        return bool(op.diagonal) and axis == "Z"

    def _unapply(self, op):
        from workloads.circuits import DiagWeight

        if isinstance(op, DiagWeight):
            ph = np.conj(np.asarray(op.phase))
            self.dm.apply_diagonal_weight(ph)
            self.bar.apply_diagonal_weight(ph)
        else:
            ud = np.asarray(op.u).conj().T
            self.dm.apply_gate(op.qubits, ud)
            self.bar.apply_gate(op.qubits, ud)

    def _gates_backward(self, gates, grad):
        """Reverse a run of gates (forward order) on both handles, accumulating derivatives."""
        def is_param(g):
            return getattr(g, "param", None) is not None

        done = set()
        pos = len(gates)
        while pos > 0:
            batch, between = [], []
            for i in range(pos - 1, -1, -1):
                g = gates[i]
                if is_param(g) and i not in done:
                    q, axis = g.qubits[0], g.param[1]
                    if all(self._commutes(h, q, axis) for h in between):
                        batch.append(i)
                between.append(g)
            if batch:
                masks = [_masks(gates[i].qubits[0], gates[i].param[1]) for i in batch]
                ov = self.bar.pauli_overlap(self.dm, [m[0] for m in masks], [m[1] for m in masks])
                for i, v in zip(batch, ov):
                    grad[gates[i].param[0]] += float(np.imag(v))
                done.update(batch)
            nxt = max((i for i in range(pos) if is_param(gates[i]) and i not in done), default=-1)
            for i in range(pos - 1, nxt, -1):
                self._unapply(gates[i])
            pos = nxt + 1

    def backward(self, n_params: int) -> np.ndarray:
        from workloads.circuits import Compress, Kraus

        grad = np.zeros(n_params)
        self.bar.apply_pauli_sum_from(self.dm, self.xm, self.zm, self.coeff)
        last = len(self.layers) - 1
        for l in range(last, -1, -1):
            seg = self.layers[l]
            if self._all:
                # the layer's inputs and records are kept; its end state is the next checkpoint
                if l < last:
                    self.dm.restore(self._ckpt[l + 1], self._ckrank[l + 1])
            else:
                self.dm.restore(self._ckpt[l], self._ckrank[l])
                self._run_layer(seg, keep=True)
            j = self._j0[l] + sum(isinstance(o, Kraus) for o in seg)
            i = len(seg)
            while i > 0:
                op = seg[i - 1]
                if isinstance(op, Compress):
                    kr = seg[i - 2]
                    j -= 1
                    self.bar.compress_adjoint(self._xbuf[j], self._rec[j], kr.qubit, kr.ops)
                    self.dm.restore(self._xbuf[j], self._xrank[j])
                    i -= 2
                    continue
                # a maximal run of gates / diagonal weights
                k = i
                while k > 0 and not isinstance(seg[k - 1], (Compress, Kraus)):
                    k -= 1
                self._gates_backward(seg[k:i], grad)
                i = k
        self.bar.synchronize()
        return grad

    def close(self):
        self.dm.close()
        self.bar.close()


def make_noisy_energy():
    """torch.autograd.Function: E = NoisyEnergy.apply(theta, engine, make_program)."""
    import torch

    class NoisyEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, engine: EnergyGradient, make_program: Callable):
            th = theta.detach().to("cpu", torch.float64).numpy()
            E = engine.forward(make_program(th))
            ctx.engine = engine
            ctx.shape = theta.shape
            ctx.n_params = th.size
            return theta.new_tensor(E, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gE):
            g = ctx.engine.backward(ctx.n_params).reshape(ctx.shape)
            return gE * torch.as_tensor(g, dtype=torch.float64, device=gE.device), None, None

    return NoisyEnergy
