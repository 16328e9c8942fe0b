"""What the learned warm start gains over the plain run, end to end on the
GPU at a small, steady-regime size: data from the solver's own batched runs,
training with the BF16 MFMA network kernels, then plain, warm and reference
starts of held-out cavities in one batch.  The warm start must reach a
steady Nusselt number in fewer steps and settle on the reference's Nu."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(300)
def test_warm_start_saves_steps_in_the_steady_regime():
    from paper_2211_03160_amd import warmstart as WS
    out = WS.run(**WS.QUICK)
    res = out["eval"]
    print({k: v for k, v in out.items() if k not in ("eval", "loss_history", "nu_history")}, flush=True)
    for r in res:
        print(r, flush=True)
    assert out["unstable_eval_runs"] == 0
    assert out["loss_history"][-1] < 0.5 * out["loss_history"][0]
    assert out["settled_warm_1pct"] >= len(res) // 2
    assert out["median_steps_warm"] < 0.7 * out["median_steps_plain"]
    assert out["steps_saved_ci95"][0] > 0
    assert out["nu_rel_err_warm_median"] < 0.01
