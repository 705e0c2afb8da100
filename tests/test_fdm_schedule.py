"""The full-rank comparator's host scheduler on the CPU: operator fusion (FP64 products of
operators on at most 2 index bits), pass building and register phases, checked by running the
runtime source with its device launches replaced by an interpreter of the pass descriptors
(tests/fdm_schedule/check.cpp) and comparing the state with the FP64 oracle (Eq. "full rank
evolution", Sec. II.A) to 1e-5, the same bar as the GPU parity tests."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from fdm_programs import mixed_program
from oracle import fdm as ofdm
from workloads import circuits as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_06657_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime.h"):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path_factory.mktemp("fdm") / "check")
    cmd = [gxx, "-O1", "-std=c++20", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           os.path.join(ROOT, "tests", "fdm_schedule", "check.cpp"), "-o", exe,
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def _write(prog, path):
    with open(path, "w") as f:
        f.write(f"{prog.n}\n")
        for op in prog.ops:
            if isinstance(op, C.Gate):
                u = np.asarray(op.u, dtype=complex)
                f.write("G %d %s %s\n" % (len(op.qubits), " ".join(map(str, op.qubits)),
                                          " ".join("%.17g %.17g" % (z.real, z.imag) for z in u.ravel())))
            elif isinstance(op, C.DiagWeight):
                f.write("W %s\n" % " ".join("%.17g %.17g" % (z.real, z.imag) for z in np.asarray(op.phase, complex)))
            elif isinstance(op, C.Kraus):
                e = np.asarray(op.ops, dtype=complex)
                f.write("K %d %d %s\n" % (op.qubit, e.shape[0],
                                          " ".join("%.17g %.17g" % (z.real, z.imag) for z in e.ravel())))


def _run(checker, prog, tmp_path):
    src, out = str(tmp_path / "prog.txt"), str(tmp_path / "rho.bin")
    _write(prog, src)
    r = subprocess.run([checker, src, out], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    rho = np.fromfile(out, dtype=np.complex64).reshape(2 ** prog.n, 2 ** prog.n)
    return rho, r.stdout


@pytest.mark.parametrize("n,seed,count", [(1, 11, 60), (2, 12, 60), (3, 13, 120), (5, 15, 120),
                                          (7, 17, 160), (8, 18, 160)])
def test_schedule_mixed_program(checker, tmp_path, n, seed, count):
    """Random programs: every fusion case (diagonal with diagonal, 1-bit into 2-bit, row/column
    pairs, operators on bits that later operators share) and, from n = 7 (26-bit index, full
    13-bit tiles), the register-phase descriptors."""
    prog = mixed_program(n, seed, count)
    rho, log = _run(checker, prog, tmp_path)
    ref = ofdm.run_fdm(prog)
    assert np.max(np.abs(rho - ref)) <= 1e-5, log


def test_schedule_brickwork(checker, tmp_path):
    """The brickwork layers across a flush of 3 layers at n = 7: channels fuse with the next
    layer's single-qubit gates."""
    prog = C.cfg3_program(n=7, r=64, layers=3)
    rho, log = _run(checker, prog, tmp_path)
    ref = ofdm.run_fdm(prog)
    assert np.max(np.abs(rho - ref)) <= 1e-5, log
    assert abs(np.trace(rho).real - 1) <= 1e-5


def test_schedule_hamming_weight_phase(checker, tmp_path):
    """Noisy Grover at n = 7 (Sec. III.C): each Hamming-weight phase flushes the queued passes
    and runs as its own sweep, so order with the fused gates and channels is kept."""
    prog = C.cfg2_program(n=7, r=16, iterations=2, p=0.003)
    rho, log = _run(checker, prog, tmp_path)
    ref = ofdm.run_fdm(prog)
    assert np.max(np.abs(rho - ref)) <= 1e-5, log
