"""Instability detection at sync points: a non-finite population or a node
faster than the lattice sound speed c_s = 1/sqrt(3) makes lbm_fields and
lbm_diagnostics return LBM_E_UNSTABLE (after writing their outputs), and
sets the per-cavity flag of a batch without touching the other cavities."""
import math

import numpy as np
import pytest

from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

UNSTABLE = -3


def _fast_state(n, speed):
    N = int(np.prod(n))
    u = np.zeros((2, N))
    u[0, N // 2] = speed
    return u, np.full(N, 0.5)


def test_speed_above_sound_speed_is_unstable():
    cfg = W.rayleigh_benard(2, (17, 13), ra=1e4, pr=0.71, storage="fp32")
    c = lbm.Cavity(cfg)
    u, T = _fast_state(cfg["n"][:2], 0.7)
    c.init_fields(None, u, T)
    rho, uu, TT = c.fields(check=False)
    assert abs(uu[0].ravel()[u.shape[1] // 2] - 0.7) < 1e-6  # outputs are written
    with pytest.raises(lbm.LBMError) as e:
        c.fields()
    assert e.value.status == UNSTABLE and "sound speed" in str(e.value)
    d = c.diagnostics(check=False)
    assert d["umax"] > 1 / math.sqrt(3)
    with pytest.raises(lbm.LBMError) as e:
        c.diagnostics()
    assert e.value.status == UNSTABLE
    # just below c_s: no error
    ok = lbm.Cavity(cfg)
    u, T = _fast_state(cfg["n"][:2], 0.55)
    ok.init_fields(None, u, T)
    ok.fields()
    ok.diagnostics()


def test_batch_flags_a_fast_cavity_only():
    cfgs = [W.rayleigh_benard(2, (33, 17), ra=1e4, pr=0.71, storage="fp32"),
            W.rayleigh_benard(2, (21, 21), ra=2e4, pr=0.71, storage="fp32")]
    b = lbm.Batch(cfgs)
    b.init([1, 2], [1e-2, 1e-2])
    u, T = _fast_state(cfgs[1]["n"][:2], 0.9)
    b.init_fields(1, None, u, T)
    b.step(4)
    flags = b.unstable()
    assert not flags[0] and flags[1]
