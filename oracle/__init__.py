"""CPU FP64 oracle for low-rank density-matrix evolution with eigenvalue truncation (LRET).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import or run anything in this package; the product library never does.  It shares no
code with the GPU path: it is plain NumPy/LAPACK in complex128, written step by step from the
paper (Sec. II, Algorithm 1, Theorem 1 of Appendix B) so that each function can be checked
against the text by eye.

Modules
  linalg      -- column-wise application of a k-qubit gate (tensor contraction); popcount
  lret        -- the low-rank algorithm: gate, Kraus concatenation, eigenvalue truncation
  fdm         -- exact full-rank density-matrix evolution and the noiseless statevector
  observables -- Prob(x), Tr(L^H O L) for Pauli strings, <Z_i>, <Z_i Z_j>, sampling, distortion
  grad        -- energy gradients of a noisy ansatz: central finite differences and an FP64 adjoint

Pins (tests/test_oracle_*.py) tie every function to something other than itself: Kronecker
brute force, closed forms of the channels, Theorem 1 against an explicit eigendecomposition,
the Eckart-Young error identities, Grover's closed form and exact agreement with full rank when
r >= rank.  Functions without such a pin say "parity unpinned" in their docstring.
"""
from .linalg import apply_gate, popcount  # noqa: F401
from .lret import (run_lret, compress, kraus_expand, apply_diag_weight, init_state,  # noqa: F401
                   select_rank, TAU_CLUSTER, init_sparse, intermediate_rank, run_lret_switching)
from .fdm import run_fdm, run_sv  # noqa: F401
from .observables import (probabilities, expect_pauli, expect_z, expect_zz, sample_inverse_cdf,  # noqa: F401
                          distortion, pauli_sum_expectation)
