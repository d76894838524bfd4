"""rfm_jtmul_noalloc (the J^T y entry point that allocates nothing) against rfm_jtmul on the same
inputs: two calls in a row, the second on a smaller problem, so the fixed scratch is reused with a
smaller layout after a larger one.

The device buffers come from the HIP runtime the library itself is linked with (looked up by its
soname once the library is loaded), not from torch: torch's wheel carries a HIP runtime of its own
under the same soname, and whichever of the two is loaded first serves both, so a test that brings
torch in after the library has run would drive torch on a runtime it was not built with."""
import ctypes as C
import sys

import numpy as np
import pytest

import rfm_workloads as W

pytestmark = pytest.mark.gpu

_H2D, _D2H = 1, 2


def _announce(msg):
    sys.stdout.write(f"\n[gpu-test] {msg}\n")
    sys.stdout.flush()


def _hip():
    import paper_2510_04170_amd as R
    R.lib()
    h = C.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    h.hipFree.argtypes = [C.c_void_p]
    h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    for f in (h.hipMalloc, h.hipFree, h.hipMemcpy, h.hipDeviceSynchronize):
        f.restype = C.c_int
    return h


class _DevBuf:
    """A float64 device buffer with the two methods the binding reads (data_ptr, is_contiguous)."""
    is_cuda = True

    def __init__(self, hip, host):
        self.hip, self.n = hip, host.size
        self.p = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.p), max(8 * self.n, 8)) == 0
        host = np.ascontiguousarray(host, dtype=np.float64)
        assert hip.hipMemcpy(self.p, host.ctypes.data, 8 * self.n, _H2D) == 0
        assert hip.hipDeviceSynchronize() == 0

    def data_ptr(self):
        return self.p.value

    def is_contiguous(self):
        return True

    def numpy(self):
        out = np.empty(self.n)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(out.ctypes.data, self.p, 8 * self.n, _D2H) == 0
        return out

    def free(self):
        assert self.hip.hipFree(self.p) == 0


def test_jtmul_noalloc_matches_jtmul():
    import paper_2510_04170_amd as R
    hip = _hip()
    cases = [("large", W.config2(nsub=(2, 2, 2), J=80, q=6, test_per_dim=2)),
             ("small", W.config1(nsub=(2, 2), J=30, q=8, test_per_dim=2))]
    for name, prob in cases:
        _announce(f"jtmul_noalloc {name}")
        lp = R.from_description(prob)
        rng = np.random.default_rng(4)
        lp.stage_assemble(0.1 * rng.normal(size=lp.n), 100.0)
        y = rng.normal(size=lp.m)
        ref = lp.jtmul(y)
        yd, xd = _DevBuf(hip, y), _DevBuf(hip, np.full(lp.n, np.nan))
        lp.jtmul_noalloc(yd, xd)
        got = xd.numpy()
        print(f"{name}: n {lp.n} m {lp.m}: max |noalloc - jtmul| = {np.abs(got - ref).max():.2e}")
        assert np.array_equal(got, ref)  # the same kernels in the same order
        yd.free()
        xd.free()
        lp.close()


def test_jtmul_noalloc_rejects_host_pointers_and_missing_jacobian():
    import paper_2510_04170_amd as R
    hip = _hip()
    prob = W.config1(nsub=(2, 2), J=20, q=6, test_per_dim=2)
    lp = R.from_description(prob)
    yd, xd = _DevBuf(hip, np.zeros(lp.m)), _DevBuf(hip, np.zeros(lp.n))
    with pytest.raises(R.RfmError) as ei:
        lp.jtmul_noalloc(yd, xd)                  # no Jacobian assembled yet
    assert ei.value.status == R.RFM_EINVAL
    lp.stage_assemble(np.zeros(lp.n), 100.0)
    rc = R.lib().rfm_jtmul_noalloc(lp.h, np.zeros(lp.m).ctypes.data, xd.data_ptr())
    assert rc == R.RFM_EINVAL                      # host input
    yd.free()
    xd.free()
    lp.close()
