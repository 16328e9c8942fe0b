"""lbm_diagnostics_async, the entry point that allocates nothing (its
partial sums live in the library's static per-device scratch), against
lbm_diagnostics on the same state: two calls in a row, the second on a
smaller cavity, so the scratch holds the first call's partials when the
second starts.  Sums and the maximum must agree bitwise (same kernels, same
reduction order); Nu_vol and Re to a few ulps (the same FP64 expressions,
evaluated on the device instead of the host)."""
import ctypes as C

import numpy as np
import pytest

from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ["t", "mass", "energy", "umax", "nu_vol", "re", "nonfinite"]


def _async_diag(cav):
    import torch
    L = lbm.lib()
    out = torch.full((lbm.DIAG_VALUES,), float("nan"), dtype=torch.float64, device="cuda")
    st = L.lbm_diagnostics_async(cav._h, C.c_void_p(out.data_ptr()))
    cav._check(st)
    cav.stream.synchronize()
    return dict(zip(FIELDS, out.cpu().numpy().tolist()))


def _check(cav):
    ref = cav.diagnostics()
    got = _async_diag(cav)
    assert got["t"] == ref["t"]
    for k in ("mass", "energy", "umax", "nonfinite"):
        assert got[k] == ref[k], (k, got[k], ref[k])
    for k in ("nu_vol", "re"):
        assert abs(got[k] - ref[k]) <= 4 * np.finfo(np.float64).eps * abs(ref[k]), (k, got[k], ref[k])
    return got


def test_async_diagnostics_match_two_calls_second_smaller():
    big = lbm.Cavity(W.rayleigh_benard(2, (257, 129), ra=1e5, pr=0.71, storage="fp32"))
    big.init(5, 2e-2)
    big.step(40)
    g1 = _check(big)
    small = lbm.Cavity(W.rayleigh_benard(3, (9, 11, 13), ra=2e4, pr=0.71, storage="fp64"))
    small.init(6, 2e-2)
    small.step(17)
    g2 = _check(small)
    assert g1["mass"] != g2["mass"]
    # the first context again, after the smaller one used the scratch
    big.step(3)
    _check(big)


def test_async_diagnostics_rejects_bad_arguments():
    L = lbm.lib()
    cav = lbm.Cavity(W.rayleigh_benard(2, (17, 9), ra=1e4, pr=0.71, storage="fp32"))
    import torch
    out = torch.zeros(7, dtype=torch.float64, device="cuda")
    assert L.lbm_diagnostics_async(cav._h, C.c_void_p(out.data_ptr())) == -4  # before init
    cav.init(1, 0.0)
    assert L.lbm_diagnostics_async(cav._h, None) == -1
    host = np.zeros(7)
    assert L.lbm_diagnostics_async(cav._h, C.c_void_p(host.ctypes.data)) == -1
    assert L.lbm_diagnostics_async(None, C.c_void_p(out.data_ptr())) == -1
