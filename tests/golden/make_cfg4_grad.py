"""Writes cfg4_grad.json: energy and gradient of the differentiable noisy ansatz (n=12, r=16,
8 layers of RY/RZ + CZ ladder, depolarizing p=0.002, 200-term Pauli Hamiltonian, seed 1004)
from the FP64 oracle only: the reverse sweep and central differences with h = 1e-4.

    python tests/golden/make_cfg4_grad.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import grad as OG  # noqa: E402
from workloads import circuits as C  # noqa: E402


def main():
    theta = C.cfg4_angles()
    xm, zm, co, _ = C.random_pauli_sum(12)
    E, g_adj = OG.energy_grad_adjoint(C.cfg4_program(theta), theta.size, xm, zm, co)
    g_fd = OG.energy_grad_fd(lambda t: C.cfg4_program(t), theta, xm, zm, co, h=1e-4)
    out = {"workload": "noisy RY/RZ ansatz n=12 r=16, 8 layers, depolarizing 0.002, 200 Pauli terms",
           "theta_seed": 1004, "h": 1e-4, "energy": E,
           "grad_adjoint": g_adj.tolist(), "grad_fd": g_fd.tolist(),
           "max_abs_adjoint_minus_fd": float(np.max(np.abs(g_adj - g_fd)))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg4_grad.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["energy"], out["max_abs_adjoint_minus_fd"])


if __name__ == "__main__":
    main()
