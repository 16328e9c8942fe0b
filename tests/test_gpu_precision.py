"""Storage precision from a developed state (paper_2211_03160_amd.precision)
on a small cell: 49^3, Ra 1e5, grown in FP32 until Re settles, then every
storage mode restarted from the same moments for 500 steps against FP64.

Bounds: FP32 storage rounds each population to 2^-24 relative per step, so
after 500 steps Nu and Re agree with FP64 to ~1e-6; the mixed mode (FP16 f,
FP32 g) keeps the thermal populations, hence the wall flux, in FP32 and
meets the 1e-3 Nu bound; literal FP16/BF16 lose the near-wall heat flux
(documented) and are only required to stay finite."""
import math

import pytest

from paper_2211_03160_amd import precision

pytestmark = pytest.mark.gpu


def test_developed_state_precision_small():
    res = precision.run(**precision.QUICK, log=lambda *a: print(*a, flush=True))
    m = res["modes"]
    print({k: (round(v["nu_rel_err"], 8), round(v["re_rel_err"], 8)) for k, v in m.items()}, flush=True)
    assert m["fp64"]["nu_hot"] > 1.2, "the flow must have developed convection"
    assert m["fp64"]["re"] > 0
    assert m["fp32"]["nu_rel_err"] < 1e-5 and m["fp32"]["re_rel_err"] < 1e-4
    assert m["mixed"]["nu_rel_err"] < 1e-3 and m["mixed"]["re_rel_err"] < 1e-2
    for st in ("fp16", "bf16"):
        assert math.isfinite(m[st]["nu_hot"]) and math.isfinite(m[st]["re"])
