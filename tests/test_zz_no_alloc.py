"""lb_read_fields_noalloc against lb_read_fields, through the C ABI.

The no-allocation readout must give the same fields bit for bit (the same
kernel reads the same populations; only where its output is staged
differs), allocate nothing through the handle's allocator, and stay correct
over consecutive calls that share its fixed device array: a box of several
chunks first, then a smaller one of a single chunk, whose stale contents
from the first call must not leak into its result.
"""
import numpy as np
import pytest

from tests.test_gpu_parity import gpu, note

pytestmark = pytest.mark.gpu


def _scene(lbsq, shape, storage, layout, steps):
    s = lbsq.Sim(shape, storage=storage, layout=layout)
    c = np.array(shape, dtype=float) / 2.0
    s.add_squirmer(c + (0.3, -0.2, 0.1), (0.6, 0.0, 0.8), min(shape) / 6.0, B1=5e-3, beta=-2.0)
    s.step(steps)
    return s


@pytest.mark.parametrize("storage,layout", [("f32", "inplace"), ("f16", "ab")])
def test_noalloc_readout_matches_and_allocates_nothing(storage, layout):
    lbsq = gpu()
    # 104 x 96 x 64 = 638,976 cells: two chunks of the 508,160-cell array;
    # then 40 x 36 x 30: one chunk
    for shape, steps in (((104, 96, 64), 13), ((40, 36, 30), 7)):
        note("no-alloc readout %s %s %s" % (shape, storage, layout))
        s = _scene(lbsq, shape, storage, layout, steps)
        s.sync()
        before = s._mem.nalloc
        rho_n, u_n, own_n = s.fields_noalloc()
        assert s._mem.nalloc == before, "the no-allocation readout called the allocator"
        rho, u, own = s.fields()
        assert s._mem.nalloc > before  # the plain readout stages through the allocator
        assert np.array_equal(own_n, own)
        assert np.array_equal(rho_n, rho)
        assert np.array_equal(u_n, u)
        fl = own == 0
        assert fl.sum() > 0.9 * own.size and np.abs(u[:, fl]).max() > 0.0
        s.close()


def test_noalloc_readout_rejects_null_buffers():
    import ctypes as C
    lbsq = gpu()
    s = _scene(lbsq, (24, 24, 24), "f32", "inplace", 2)
    L = lbsq.load()
    rho = np.empty(s.n)
    assert L.lb_read_fields_noalloc(s.h, None, rho.ctypes.data_as(C.POINTER(C.c_double)), None) == lbsq.LB_EINVAL
    assert L.lb_read_fields_noalloc(None, None, None, None) == lbsq.LB_EINVAL
    s.close()
