"""Batched serving (many handles of uneven n and r in one captured hipGraph): every instance
equals its unbatched run bit for bit when both issue the same launches (same kernels, tiles and
reduction order), within 1e-6 on Prob and <Z_i> when the unbatched run chains consecutive
compressions on one qubit (the batch issues every compression separately), and matches the FP64
oracle within the complex64 tolerance (1e-5 on <Z_i>)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import circuits as C

pytestmark = pytest.mark.gpu


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


def _mix(count, seed, n_range=(5, 10), depth_range=(2, 4)):
    """Brickwork instances with uneven n, r, depth and channels (depolarizing, or amplitude
    damping + dephasing)."""
    rng = np.random.default_rng(seed)
    progs = []
    for i in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        r = int(rng.choice([8, 16, 32]))
        depth = int(rng.integers(depth_range[0], depth_range[1] + 1))
        if i % 3 == 2:
            chans = [("ad", float(rng.uniform(0.001, 0.01))), ("deph", float(rng.uniform(0.001, 0.01)))]
        else:
            chans = [("dep", float(rng.uniform(1e-4, 5e-3)))]
        progs.append(C.brickwork_program(n, depth, r, chans, seed=900 + i))
    return progs


def _chains(p):
    """True when the program has two channels on one qubit with nothing but a compression between."""
    prev = None
    for op in p.ops:
        if isinstance(op, C.Kraus):
            if prev is not None and prev == op.qubit:
                return True
            prev = op.qubit
        elif not isinstance(op, C.Compress):
            prev = None
    return False


def _run_unbatched(lr, progs):
    out = []
    for p in progs:
        dm = lr.LowRankDM(p.n, p.r, lr.C64, p.m_max)
        lr.run_program(dm, p)
        z, _, tr = dm.expect_z()
        out.append((dm.get_L(), z, tr, dm.probabilities().cpu().numpy()))
        dm.close()
    return out


def _run_batched(lr, progs, replays=1):
    hs = [lr.LowRankDM(p.n, p.r, lr.C64, p.m_max) for p in progs]
    b = lr.Batch(hs)
    with b.recording():
        for dm, p in zip(hs, progs):
            dm.reset()
            lr.run_program(dm, p)
    results = []
    for _ in range(replays):
        b.launch()
        done, total = b.times()
        res = []
        for dm in hs:
            dm.synchronize()
            z, _, tr = dm.expect_z()
            res.append((dm.get_L(), z, tr, dm.probabilities().cpu().numpy()))
        results.append((res, done, total))
    steps, launches = b.info()
    b.close()
    return results, steps, launches


def test_batch_equals_unbatched_bitwise(lr):
    progs = _mix(24, 5)
    _say(f"batch of {len(progs)}: n {[p.n for p in progs]} r {[p.r for p in progs]}")
    ref = _run_unbatched(lr, progs)
    results, steps, launches = _run_batched(lr, progs, replays=2)
    _say(f"  steps {steps} launches {launches}")
    nchain = 0
    for rep, (res, done, total) in enumerate(results):
        for i, ((La, za, ta, Pa), (Lb, zb, tb, Pb)) in enumerate(zip(ref, res)):
            if _chains(progs[i]):
                nchain += 1
                assert np.max(np.abs(Pa - Pb)) <= 1e-6, f"instance {i} differs (replay {rep})"
                assert np.max(np.abs(za - zb)) <= 1e-6
            else:
                assert np.array_equal(La, Lb), f"instance {i} differs (replay {rep})"
                assert np.array_equal(za, zb)
        assert total > 0 and np.all(done > 0) and np.all(done <= total + 1e-9)
        # an instance with more compressions never finishes before one with fewer
        ncomp = np.array([p.n_compress() for p in progs])
        order = np.argsort(ncomp, kind="stable")
        assert np.all(np.diff(done[order]) >= -1e-9)
    assert 0 < nchain < 2 * len(progs)   # both kinds of instance occur
    # two replays of the graph are identical
    for (La, za, _, _), (Lb, zb, _, _) in zip(results[0][0], results[1][0]):
        assert np.array_equal(La, Lb) and np.array_equal(za, zb)


def test_batch_matches_oracle(lr):
    progs = _mix(6, 11, n_range=(5, 7), depth_range=(2, 3))
    results, _, _ = _run_batched(lr, progs)
    res = results[0][0]
    for p, (_, z, tr, _) in zip(progs, res):
        L = oracle.run_lret(p)
        P = oracle.probabilities(L)
        zr = oracle.expect_z(P, p.n)
        err = np.max(np.abs(z - zr))
        _say(f"  n={p.n} r={p.r} max|dZ| {err:.2e}")
        assert err <= 1e-5
        assert abs(tr - 1.0) <= 1e-5


def test_batch_errors(lr):
    a = lr.LowRankDM(5, 8, lr.C64, 4)
    b = lr.Batch([a])
    b.begin()
    a.apply_gate((0,), C.H)
    with pytest.raises(lr.LrdmError):
        a.expect_z()          # outputs are not available while recording
    a.apply_kraus(1, C.depolarizing(0.01))
    with pytest.raises(lr.LrdmError):
        b.end()               # the program ends with an uncompressed channel
    b.close()
    a2 = lr.LowRankDM(5, 8, lr.C64, 4)
    plain = lr.LowRankDM(5, 8, lr.C64, 4, lr.FLAG_PLAIN)
    with pytest.raises(lr.LrdmError):
        lr.Batch([a2, plain])
    c128 = lr.LowRankDM(5, 8, lr.C128, 4)
    with pytest.raises(lr.LrdmError):
        lr.Batch([c128])
    with pytest.raises(lr.LrdmError):
        lr.Batch([a2, a2])
