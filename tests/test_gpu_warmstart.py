"""What the learned warm start gains over the plain run, end to end on the
GPU at a small, steady-regime size: data from the solver's own batched runs,
training with the BF16 MFMA network kernels, then plain and warm starts of
held-out cavities in one batch.  The warm start must reach a steady Nusselt
number in fewer steps and settle on the plain run's Nu."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_warm_start_saves_steps_in_the_steady_regime():
    from paper_2211_03160_amd import warmstart as WS
    out = WS.run(**WS.QUICK)
    res = out["eval"]
    print({k: v for k, v in out.items() if k not in ("eval", "loss_history")}, flush=True)
    for r in res:
        print(r, flush=True)
    assert out["loss_history"][-1] < 0.5 * out["loss_history"][0]
    pairs = [(r["steps_plain"], r["steps_warm"]) for r in res
             if r["steps_plain"] is not None and r["steps_warm"] is not None]
    assert len(pairs) >= len(res) // 2
    assert np.median([w for _, w in pairs]) < 0.7 * np.median([p for p, _ in pairs])
    assert np.median([r["nu_rel_err_warm"] for r in res]) < 0.01
    assert out["unstable_eval_runs"] == 0
