"""Outputs computed from the low-rank factor (test infrastructure only).

  Prob(x) = sum_v L_{x v} conj(L_{x v})        (Sec. II.D, equation after "probability distribution")
  <O>     = Tr(L^H O L)                         (Sec. II.D)
  distortion = T(rho_LRET, rho_exact) / T(rho_exact, rho_noiseless), T(A, B) = sum_i |A_ii - B_ii|
                                                (Eq. "distortion", Sec. III; used as written)
Readings: <Z_i> = sum_x Prob(x) (1 - 2 x_i); sampling draws the smallest x whose cumulative
probability exceeds u * (total) for a supplied uniform u (the paper does not fix a sampler).
"""
from __future__ import annotations

import numpy as np

from .linalg import popcount


def probabilities(L: np.ndarray) -> np.ndarray:
    return np.sum((L * L.conj()).real, axis=1)


def expect_pauli(L: np.ndarray, n: int, xmask: int, zmask: int) -> complex:
    """Tr(L^H P L) for P = i^{|x&z|} X^xmask Z^zmask (Y where both bits are set)."""
    xmask, zmask = int(xmask), int(zmask)
    idx = np.arange(2 ** n, dtype=np.uint64)
    ny = bin(xmask & zmask).count("1")
    sign = 1.0 - 2.0 * (popcount(idx & np.uint64(zmask)) & 1)
    PL = np.empty_like(L)
    PL[(idx ^ np.uint64(xmask)).astype(np.int64)] = ((1j) ** ny) * sign[:, None] * L
    return complex(np.vdot(L, PL))


def pauli_sum_expectation(L, n, xmasks, zmasks, coeffs):
    vals = np.array([expect_pauli(L, n, x, z) for x, z in zip(xmasks, zmasks)])
    return float(np.sum(np.asarray(coeffs) * vals.real)), vals


def expect_z(P: np.ndarray, n: int) -> np.ndarray:
    x = np.arange(P.shape[0], dtype=np.int64)
    return np.array([np.sum(P * (1 - 2 * ((x >> i) & 1))) for i in range(n)])


def expect_zz(P: np.ndarray, n: int) -> np.ndarray:
    x = np.arange(P.shape[0], dtype=np.int64)
    return np.array([np.sum(P * (1 - 2 * ((x >> i) & 1)) * (1 - 2 * ((x >> (i + 1)) & 1)))
                     for i in range(n - 1)])


def sample_inverse_cdf(P: np.ndarray, u: np.ndarray) -> np.ndarray:
    """For each uniform u_j: the smallest x with CDF(x) > u_j * CDF(last)."""
    cdf = np.cumsum(P)
    idx = np.searchsorted(cdf, np.asarray(u) * cdf[-1], side="right")
    return np.minimum(idx, P.shape[0] - 1).astype(np.uint64)


def distortion(diag_lret: np.ndarray, diag_exact: np.ndarray, diag_noiseless: np.ndarray) -> float:
    return float(np.sum(np.abs(diag_lret - diag_exact)) / np.sum(np.abs(diag_exact - diag_noiseless)))
