"""Energy gradients of a noisy parametrised circuit through the low-rank evolution, on the GPU.

The energy is E(theta) = sum_t c_t Tr(L^H P_t L) of the final factor (Sec. II.D).  One call of
lrdm_energy_grad (include/lrdm.h) runs the forward pass with per-layer checkpoints of L, then
the reverse sweep over the same operations in the library: the adjoint Lbar (dE = 2 Re
Tr(Lbar^H dL)) goes back through every channel + compression (FP64 eigenvector-derivative formula
on the small Gram matrix, bulk-precision products over the 2^n rows) and every gate (U^H on both
factors; a rotation R_P(theta) = exp(-i theta P/2) contributes dE/dtheta = Im Tr(Lbar^H P L)).
When every channel's input and compression record fit the byte budget they are kept from the
forward pass and nothing is re-run; otherwise each layer is re-run once from its checkpoint.

This module only converts the program (FlatProgram) and owns the device buffers.
"""
from __future__ import annotations

import ctypes
from typing import Callable

import numpy as np

from .lrdm import FlatProgram, LowRankDM, _check, _dptr


class EnergyGradient:
    """Energy and gradient for programs of one shape (n, r, m_max) and one Hamiltonian.

    Parametrised gates of the program carry param = (index into theta.ravel(), axis); the
    gradient has one entry per index."""

    def __init__(self, n: int, r: int, m_max: int, xmask, zmask, coeff, dtype: int = 0,
                 device: str = "cuda:0", store_all_bytes: int = 8 << 30):
        import torch

        self.n, self.r, self.m_max = n, r, m_max
        self.dm = LowRankDM(n, r, dtype, m_max, device=device)
        self.bar = LowRankDM(n, r, dtype, m_max, device=device)
        self.lib = self.dm.lib
        self.xm = np.ascontiguousarray(xmask, dtype=np.uint64)
        self.zm = np.ascontiguousarray(zmask, dtype=np.uint64)
        self.coeff = np.ascontiguousarray(coeff, dtype=np.float64)
        self.device = torch.device(device)
        self.store_all_bytes = int(store_all_bytes)
        self._store = None
        self._all = False
        self.energy = None
        self.grad = None

    def energy_and_grad(self, program, n_params: int | None = None):
        """(E, dE/dtheta) of `program` run from |0...0>, by lrdm_energy_grad."""
        import torch

        fp = FlatProgram(program)
        n_params = fp.n_params if n_params is None else int(n_params)
        keep_b, min_b = ctypes.c_size_t(), ctypes.c_size_t()
        _check(self.lib.lrdm_energy_grad_bytes(self.dm.h, fp.ref, ctypes.byref(keep_b), ctypes.byref(min_b)))
        want = keep_b.value if keep_b.value <= self.store_all_bytes else min_b.value
        if self._store is None or self._store.numel() < want:
            self._store = torch.empty(want, dtype=torch.uint8, device=self.device)
        E = np.zeros(1)
        g = np.zeros(max(n_params, 1))
        kept = ctypes.c_int()
        _check(self.lib.lrdm_energy_grad(self.dm.h, self.bar.h, fp.ref, None, n_params, self.xm.shape[0],
                                         self.xm.ctypes.data, self.zm.ctypes.data, self.coeff.ctypes.data,
                                         _dptr(E), _dptr(g), ctypes.c_void_p(self._store.data_ptr()), want,
                                         ctypes.byref(kept)))
        self._all = bool(kept.value)
        self.energy, self.grad = float(E[0]), g[:n_params].copy()
        return self.energy, self.grad

    # the two-step form used by the tests and the benchmark: forward computes both, backward
    # returns the gradient of that forward
    def forward(self, program) -> float:
        return self.energy_and_grad(program)[0]

    def backward(self, n_params: int) -> np.ndarray:
        g = np.zeros(n_params)
        g[: self.grad.size] = self.grad[:n_params]
        return g

    def close(self):
        self.dm.close()
        self.bar.close()


def make_noisy_energy():
    """torch.autograd.Function: E = NoisyEnergy.apply(theta, engine, make_program).  The forward
    computes the energy and, when theta requires a gradient, the gradient in the same call; the
    gradient is kept in the autograd context, so each graph node differentiates its own forward."""
    import torch

    class NoisyEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, engine: EnergyGradient, make_program: Callable):
            th = theta.detach().to("cpu", torch.float64).numpy()
            E, g = engine.energy_and_grad(make_program(th), th.size)
            ctx.save_for_backward(torch.as_tensor(g.reshape(theta.shape), dtype=torch.float64))
            return theta.new_tensor(E, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gE):
            (g,) = ctx.saved_tensors
            return gE * g.to(gE.device), None, None

    return NoisyEnergy
