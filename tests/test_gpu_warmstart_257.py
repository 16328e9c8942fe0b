"""The learned warm start at its full size: 257^2 cells, Ra 1e5..1e8 (mostly
unsteady), a 4-level U-Net with 32 base channels trained on about 2000
snapshots the solver generates, then 16 held-out cavities run plain, warm
and as an independent plain reference in one batch.  Unsteady cells are
assessed by a band sized from the reference's own fluctuation; the warm start
must reach the developed state sooner (a bootstrap interval of the steps
saved above zero), end as close to the reference's Nu as a second plain
run does, and land in the reference's state as often.  (When a chaotic
cell last leaves the band is itself random: those steps are reported, not
asserted.)"""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(400)
def test_warm_start_at_257_saves_steps_on_unsteady_cells():
    from paper_2211_03160_amd import warmstart as WS
    out = WS.run()
    res = out["eval"]
    print({k: v for k, v in out.items() if k not in ("eval", "loss_history", "nu_history")}, flush=True)
    for r in res:
        print(r, flush=True)
    assert out["H"] == 257 and out["chans"] == [32, 64, 128, 256]
    assert out["snapshots"] >= 2000 and out["cavities"] == 16
    assert out["unstable_eval_runs"] == 0
    assert out["loss_history"][-1] < 0.6 * out["loss_history"][0]
    assert out["steps_saved_reach_ci95"][0] > 0
    assert out["warm_faster_reach_fraction"] >= 0.75
    assert out["nu_rel_err_warm_median"] <= max(0.02, out["nu_rel_err_plain_median"])
    assert out["same_state_warm"] >= out["same_state_plain"] - 1
