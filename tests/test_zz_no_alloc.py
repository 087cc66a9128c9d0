"""lbm_moments_static, the entry point for callers that cannot allocate
device memory, against lbm_moments with a host destination: the same fields
bit for bit, on two calls in a row (the second for a smaller case and fewer
fields), and its size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_2408_00146_amd import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_00146_amd import lbm as L

    L.lib()
    return L


def via_moments(lbm, s, case, mask, shape):
    out = np.empty(shape, dtype=np.float64)
    rc = lbm.lib().lbm_moments(s._h, case, mask, out.ctypes.data_as(C.c_void_p), 0)
    assert rc == lbm.LBM_OK, lbm.lib().lbm_last_error()
    return out


def via_static(lbm, s, case, mask, shape):
    out = np.full(shape, np.nan, dtype=np.float64)
    rc = lbm.lib().lbm_moments_static(s._h, case, mask, out.ctypes.data_as(C.c_void_p))
    assert rc == lbm.LBM_OK, lbm.lib().lbm_last_error()
    return out


def test_static_moments_equal_moments(lbm):
    ps = [cases.channel(200, 100, 12.0, 4.0, sigma_TT=1e-3, beta_s=0.2, precision=cases.FP32),
          cases.channel(96, 48, 8.0, 4.0, sigma_TT=1e-3, beta_s=0.1, precision=cases.FP32)]
    s = lbm.Solver(ps)
    s.step(50)
    everything = (1 << 18) - 1
    a = via_static(lbm, s, 0, everything, (18, 100, 200))
    b = via_moments(lbm, s, 0, everything, (18, 100, 200))
    assert np.array_equal(a, b)
    # second call: a smaller case, six fields; the array still holds the first call's values beyond
    macro = (1 << 6) - 1
    a2 = via_static(lbm, s, 1, macro, (6, 48, 96))
    b2 = via_moments(lbm, s, 1, macro, (6, 48, 96))
    assert np.array_equal(a2, b2)
    f = s.fields_static(1)
    assert np.array_equal(f["phi"], b2[0]) and np.array_equal(f["psi"], b2[5])
    s.close()


def test_static_moments_size_limit(lbm):
    s = lbm.Solver(cases.channel(2048, 1024, 128.0, 5.0, precision=cases.FP32))
    three = 0b111  # 3 planes of 2048 x 1024 doubles: 48 MiB
    a = via_static(lbm, s, 0, three, (3, 1024, 2048))
    assert np.array_equal(a, via_moments(lbm, s, 0, three, (3, 1024, 2048)))
    out = np.empty((4, 1024, 2048))
    rc = lbm.lib().lbm_moments_static(s._h, 0, 0b1111, out.ctypes.data_as(C.c_void_p))  # 64 MiB + 0
    assert rc == lbm.LBM_OK
    out = np.empty((5, 1024, 2048))
    rc = lbm.lib().lbm_moments_static(s._h, 0, 0b11111, out.ctypes.data_as(C.c_void_p))  # 80 MiB
    assert rc == lbm.LBM_E_INVAL and b"static staging array" in lbm.lib().lbm_last_error()
    s.close()
