"""The paper's own cavity (Section 2.3: hot left wall, cold right wall,
adiabatic top and bottom, no-slip everywhere) run to a steady state.  The
paper prints no Nu or Re for it; what the method fixes is the steady energy
balance (heat in through the hot wall = heat out through the cold wall) and
agreement between FP32 and FP64 storage; parity with the CPU oracle over the
transient is checked in test_gpu_parity."""
import numpy as np
import pytest

from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ra", [1e4, 1e5])
def test_side_heated_steady_state(ra):
    res = {}
    for st in ("fp64", "fp32"):
        c = lbm.Cavity(W.side_heated(2, (129, 129), ra=ra, pr=0.71, storage=st))
        c.init(1, 0.0)
        nus = []
        for _ in range(12):
            c.step(25000)
            nus.append(c.nusselt())
        d = c.diagnostics()
        res[st] = (np.array(nus), d)
    nus, d = res["fp64"]
    nh, nc = nus[-1]
    print(f"side-heated 129^2 Ra {ra:g}: Nu_hot {nh:.6f} Nu_cold {nc:.6f} Re {d['re']:.4f} "
          f"max|u| {d['umax']:.5f}; FP32 Nu {res['fp32'][0][-1]}", flush=True)
    assert abs(nh - nc) / nh < 1e-4              # steady energy balance
    assert abs(nus[-1][0] - nus[-2][0]) / nh < 1e-5  # no drift left
    assert nh > 1.5                               # convection, not conduction
    n32 = res["fp32"][0][-1]
    assert abs(n32[0] - nh) / nh < 1e-4 and abs(n32[1] - nc) / nc < 1e-4
    assert abs(res["fp32"][1]["re"] - d["re"]) / d["re"] < 1e-4
