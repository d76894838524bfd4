"""The C-ABI library loads and exports every call declared in include/rfm.h
(no compute call is made here: this host has no GPU)."""
import os
import re
import subprocess

import pytest

import paper_2510_04170_amd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "rfm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rfm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_call():
    names = _declared()
    assert len(names) >= 29
    out = subprocess.run(["nm", "-D", "--defined-only", R.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = R.lib()
    for n in names:
        assert hasattr(L, n)


def test_binding_covers_every_declared_call():
    assert set(_declared()) == set(R._SIGS)


def test_defaults_are_the_paper_values():
    o = R.default_opts()
    # Sec. 6: gamma = 3, eta = 1e-6, eps = 1e-10, tau_rel = 1e-3, m_max = 3; Sec. 5: c = 100
    assert (o.sketch_factor, o.lsqr_tol, o.outer_tol, o.tau_rel, o.m_max, o.row_scale_c) == (3.0, 1e-6, 1e-10,
                                                                                              1e-3, 3, 100.0)
    assert o.method == R.RFM_IPN and o.sketch_prec == R.RFM_PREC_F64


def test_null_handles_are_safe():
    L = R.lib()
    assert L.rfm_num_unknowns(None) == -1
    assert L.rfm_num_rows(None) == -1
    L.rfm_destroy(None)
    assert L.rfm_stage_qr(None) == R.RFM_EINVAL
    assert b"null" in L.rfm_last_error()


def test_create_rejects_bad_arguments_before_device_work():
    import ctypes as C
    L = R.lib()
    h = C.c_void_p()
    assert L.rfm_create(C.byref(h), 0, 1, 0, None) == R.RFM_EINVAL
    assert L.rfm_create(C.byref(h), 2, 9, 0, None) == R.RFM_EINVAL
    assert L.rfm_create(None, 2, 1, 0, None) == R.RFM_EINVAL


@pytest.mark.parametrize("prec,fmt", [(2, "bf16"), (3, "fp8")])
def test_sketch_table_matches_oracle(prec, fmt):
    """The library's table (host bisection on erfc, its own rounding) equals the
    oracle's (scipy's quantile function, numpy rounding) bit for bit."""
    import numpy as np
    from oracle import lowprec as L
    t = R.sketch_table(prec)
    assert np.array_equal(t, L.code_table(fmt))
    with pytest.raises(R.RfmError):
        R.sketch_table(0)
