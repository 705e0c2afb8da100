"""lrdm_expect_z_noalloc (no handle, no workspace: the kernels' scratch is a library-owned device
array per GPU) against lrdm_expect_z on the same factor: two calls in a row, the second with a
smaller input, in both bulk precisions.  The two paths run the same kernels with the same split,
so the results agree bit for bit (stricter than the 1e-5 / 1e-10 bars)."""
import sys

import numpy as np
import pytest

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


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_expect_z_matches_handle_path(lr, dtype):
    dt = lr.C64 if dtype == "c64" else lr.C128
    for n, r in ((14, 32), (9, 16)):   # the second call has the smaller input
        _say(f"[noalloc] {dtype} n={n} r={r}")
        prog = C.cfg3_program(n=n, r=r, layers=2, dtype=dtype)
        dm = lr.LowRankDM(n, r, dt, prog.m_max)
        lr.run_program(dm, prog)
        z, zz, tr = dm.expect_z()
        z2, zz2, tr2 = lr.lrdm.expect_z_noalloc(dm.state.data_ptr(), n, dm.ld, dm.ld, dt, dm.stream)
        assert np.array_equal(z, z2) and np.array_equal(zz, zz2) and tr == tr2
        assert abs(tr - 1.0) < 1e-5
        dm.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(lr):
    import torch

    buf = torch.zeros(1024, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(lr.LrdmError) as e:
        lr.lrdm.expect_z_noalloc(buf.data_ptr(), 21, 8, 8, lr.C64)
    assert e.value.status == 6
    assert "n <= 20" in str(e.value)
    with pytest.raises(lr.LrdmError) as e:
        lr.lrdm.expect_z_noalloc(buf.data_ptr(), 4, 8, 9, lr.C64)
    assert e.value.status == 1
