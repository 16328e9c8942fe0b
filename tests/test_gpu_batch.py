"""GPU tests of the batched launch (lbm_batch_*): every cavity of a batch
must evolve exactly as the same cavity run alone (the per-node arithmetic is
shared), with one or several steps per launch, under every launch shape,
with and without hipGraph replay, and a diverging cavity must not disturb
the others.  One FP64 batch member is also compared with the CPU oracle."""
import numpy as np
import pytest

from oracle.lbmref import Oracle
from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu


def _small_batch(storage="fp32", dim=2):
    if dim == 2:
        return [
            W.rayleigh_benard(2, (33, 17), ra=2e4, pr=0.71, storage=storage),
            W.rayleigh_benard(2, (65, 65), ra=1e5, pr=3.0, storage=storage),
            W.side_heated(2, (41, 41), ra=1e6, storage=storage),
            W.rayleigh_benard(2, (66, 33), ra=5e4, pr=0.71, lateral="periodic", storage=storage),
            W.rayleigh_benard(2, (257, 5), ra=1e4, pr=1.5, storage=storage),
            W.rayleigh_benard(2, (3, 2), ra=1e4, pr=0.9, storage=storage),
        ]
    return [
        W.rayleigh_benard(3, (17, 19, 21), ra=1e5, pr=0.71, storage=storage),
        W.side_heated(3, (15, 15, 15), ra=1e5, storage=storage),
        W.rayleigh_benard(3, (12, 10, 9), ra=5e4, pr=0.71, lateral="periodic", storage=storage),
    ]


def _fields_equal(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def _singles(cfgs, seeds, amps, steps):
    out = []
    for c, s, a in zip(cfgs, seeds, amps):
        g = lbm.Cavity(c)
        g.init(s, a)
        g.step(steps)
        out.append((g.fields(), g.nusselt() if _has_nu(c) else None))
    return out


def _has_nu(cfg):
    return "dirichlet" in cfg["bc"]


@pytest.mark.parametrize("dim,storage", [(2, "fp32"), (2, "mixed"), (3, "fp32"), (2, "fp64")])
def test_batch_members_equal_single_runs(dim, storage):
    cfgs = _small_batch(storage, dim)
    seeds = [11 + k for k in range(len(cfgs))]
    amps = [1e-2] * len(cfgs)
    steps = 60
    ref = _singles(cfgs, seeds, amps, steps)
    b = lbm.Batch(cfgs)
    b.init(seeds, amps)
    b.step(steps)
    assert b.t == steps
    hot, cold = b.nusselt()
    for k in range(len(cfgs)):
        v = b.cavity(k)
        assert v.t == steps
        assert _fields_equal(v.fields(), ref[k][0]), k
        if ref[k][1] is not None:
            assert (hot[k], cold[k]) == ref[k][1], k
            assert v.nusselt() == ref[k][1]
        else:
            assert np.isnan(hot[k]) and np.isnan(cold[k])
    assert not b.unstable().any()


def test_batch_fp64_member_matches_oracle():
    cfgs = _small_batch("fp64", 2)
    seeds = [3] * len(cfgs)
    b = lbm.Batch(cfgs)
    b.init(seeds, [1e-2] * len(cfgs))
    b.step(150)
    for k in (1, 2):
        o = Oracle(cfgs[k])
        o.init(3, 1e-2)
        o.step(150)
        rg, ug, Tg = b.cavity(k).fields()
        ro, uo, To = o.fields()
        assert max(np.abs(rg - ro).max(), np.abs(ug - uo).max(), np.abs(Tg - To).max()) < 1e-11
        hot, cold = b.nusselt()
        nh, nc = o.nusselt()
        assert abs(hot[k] - nh) < 1e-10 and abs(cold[k] - nc) < 1e-10


@pytest.mark.parametrize("block", [128, 256, 512])
@pytest.mark.parametrize("grid_per_cu", [0, 1, 4])
def test_launch_shapes_give_identical_results(block, grid_per_cu):
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    base = lbm.Batch(cfgs)
    base.init(seeds, amps)
    base.step(25)
    b = lbm.Batch(cfgs)
    b.set_config(block=block, grid_per_cu=grid_per_cu)
    assert b.config() == {"block": block, "grid_per_cu": grid_per_cu, "graph_steps": 0, "stream_rows": 0,
                          "stream_waves": 0}
    b.init(seeds, amps)
    b.step(25)
    for k in range(len(cfgs)):
        assert _fields_equal(b.cavity(k).fields(), base.cavity(k).fields())


@pytest.mark.parametrize("spl", [3, 4])
@pytest.mark.parametrize("rows,waves", [(8, 1), (16, 2), (40, 8), (64, 4), (256, 2)])
def test_streaming_shapes_give_identical_results(spl, rows, waves):
    """The streaming kernel's segment rows and wavefronts per block (the
    autotuner's parameters) change nothing in the results."""
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    base = lbm.Batch(cfgs)
    base.steps_per_launch = 1
    base.init(seeds, amps)
    base.step(25)
    b = lbm.Batch(cfgs)
    b.steps_per_launch = spl
    b.set_config(block=256, stream_rows=rows, stream_waves=waves)
    b.init(seeds, amps)
    b.step(25)
    for k in range(len(cfgs)):
        assert _fields_equal(b.cavity(k).fields(), base.cavity(k).fields()), k
    assert np.array_equal(np.nan_to_num(b.nusselt()[0]), np.nan_to_num(base.nusselt()[0]))


def test_graph_replay_matches_eager():
    """Replays separated by the program's own work and synchronisations,
    every replay checked against the eager run."""
    import torch
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    eager = lbm.Batch(cfgs)
    graph = lbm.Batch(cfgs)
    graph.set_config(block=256, grid_per_cu=0, graph_steps=4)
    eager.init(seeds, amps)
    graph.init(seeds, amps)
    for rep in range(5):
        n = 4 if rep != 2 else 9  # 9 = two replays and one single launch
        eager.step(n)
        graph.step(n)
        x = torch.randn(1024, device="cuda")  # unrelated eager work between replays
        torch.cuda.synchronize()
        assert float((x * 0).sum()) == 0.0
        assert graph.t == eager.t
        for k in range(len(cfgs)):
            assert _fields_equal(graph.cavity(k).fields(), eager.cavity(k).fields()), (rep, k)
        assert np.array_equal(np.nan_to_num(graph.nusselt()[0]), np.nan_to_num(eager.nusselt()[0]))


def test_diverging_cavity_is_flagged_and_isolated():
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    ref = _singles(cfgs, seeds, amps, 30)
    b = lbm.Batch(cfgs)
    b.init(seeds, amps)
    bad = 1
    n = int(np.prod(cfgs[bad]["n"]))
    T = np.full(n, 0.5)
    T[n // 2] = np.nan
    b.init_fields(bad, None, np.zeros((2, n)), T)
    b.step(30)
    flags = b.unstable()
    assert flags[bad] and flags.sum() == 1
    for k in range(len(cfgs)):
        if k != bad:
            assert _fields_equal(b.cavity(k).fields(), ref[k][0]), k
    hot, _ = b.nusselt()
    assert np.isfinite(hot[0])


def test_autotuner_picks_a_candidate_and_keeps_results():
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    b = lbm.Batch(cfgs)
    b.init(seeds, amps)
    best, ms = b.tune(steps=2)
    # 12 one-step shapes, then 2/3/4/5 steps per launch (FP32) x 5 segment
    # lengths x 3 block sizes of the streaming kernel
    assert len(ms) == 12 + 60 and all(m > 0 for m in ms)
    assert best["block"] in (128, 256, 512) and best["grid_per_cu"] in (0, 2, 4, 8)
    assert b.config() == best
    spl = b.steps_per_launch
    if spl > 1:
        assert best["stream_rows"] in (16, 24, 32, 48, 64) and best["stream_waves"] in (2, 4, 8)
        assert min(ms[12:]) <= min(ms[:12])
    t = b.t
    assert t == 12 * 3 + 15 * 3 * (2 + 3 + 4 + 5)
    ref = _singles(cfgs, seeds, amps, t + 10)
    b.step(10)
    for k in range(len(cfgs)):
        assert _fields_equal(b.cavity(k).fields(), ref[k][0]), k


def test_views_refuse_stepping_and_batch_errors():
    cfgs = _small_batch("fp32", 2)
    b = lbm.Batch(cfgs)
    with pytest.raises(lbm.LBMError):
        b.step(1)  # before init
    b.init([1] * len(cfgs), [0.0] * len(cfgs))
    v = b.cavity(0)
    for call in (lambda: v.step(1), lambda: v.init(1, 0.0)):
        with pytest.raises(lbm.LBMError) as e:
            call()
        assert e.value.status == -4
    with pytest.raises(lbm.LBMError):
        b.set_config(block=100)
    with pytest.raises(lbm.LBMError):
        b.set_config(graph_steps=3)
    for bad in (dict(stream_rows=5), dict(stream_rows=300), dict(stream_waves=3), dict(stream_waves=16)):
        with pytest.raises(lbm.LBMError):
            b.set_config(**bad)
    b.step(1)
    with pytest.raises(lbm.LBMError) as e:
        b.init_fields(0, None, np.zeros((2, 33 * 17)), np.zeros(33 * 17))
    assert e.value.status == -4
    with pytest.raises(lbm.LBMError):
        lbm.Batch([W.rayleigh_benard(2, (9, 9), ra=1e4, pr=0.7, storage="fp32"),
                   W.rayleigh_benard(2, (9, 9), ra=1e4, pr=0.7, storage="fp64")])


def test_sweep_recipe_runs_and_tunes():
    """The 64-cavity sweep: all members advance; the few under-resolved ones
    (relaxation times within 1% of 1/2) may be flagged, no other."""
    cfgs, seeds = W.batched_sweep()
    b = lbm.Batch(cfgs)
    b.init(seeds, [W.NOISE] * len(cfgs))
    best, ms = b.tune(steps=2)
    b.set_config(graph_steps=10, **{k: best[k] for k in ("block", "grid_per_cu")})
    b.step(40)
    flags = b.unstable()
    taus = [lbm.derive(c) for c in cfgs]
    for k, f in enumerate(flags):
        if f:
            assert min(taus[k]["tau_f"], taus[k]["tau_g"]) < 0.51, k
    hot, cold = b.nusselt()
    ok = ~flags
    assert np.all(np.isfinite(hot[ok])) and np.all(np.isfinite(cold[ok]))
    print("sweep tune", best, ms, "flagged", int(flags.sum()), flush=True)


def test_batch_steps_per_launch_defaults_and_arguments():
    """2D batches start streaming with a single cavity's default count; 3D
    ones with one step per launch and refuse more."""
    for storage, k in (("fp32", 5), ("mixed", 4), ("fp16", 3), ("bf16", 4), ("fp64", 2)):
        assert lbm.Batch(_small_batch(storage, 2)).steps_per_launch == k, storage
    b = lbm.Batch(_small_batch("fp32", 2))
    for bad in (0, 6, -1):
        with pytest.raises(lbm.LBMError) as e:
            b.steps_per_launch = bad
        assert e.value.status == -1
    for k in (1, 2, 3, 4, 5):
        b.steps_per_launch = k
        assert b.steps_per_launch == k
    for storage in ("mixed", "fp16", "bf16"):  # five steps: FP32 storage only
        with pytest.raises(lbm.LBMError) as e:
            lbm.Batch(_small_batch(storage, 2)).steps_per_launch = 5
        assert e.value.status == -5
    b64 = lbm.Batch(_small_batch("fp64", 2))
    with pytest.raises(lbm.LBMError) as e:
        b64.steps_per_launch = 3
    assert e.value.status == -5
    b3 = lbm.Batch(_small_batch("fp32", 3))
    assert b3.steps_per_launch == 1
    with pytest.raises(lbm.LBMError) as e:
        b3.steps_per_launch = 2
    assert e.value.status == -5


@pytest.mark.parametrize("storage,spl", [(s, k) for s in ("fp32", "mixed", "fp16", "bf16") for k in (1, 2, 3, 4)]
                         + [("fp32", 5), ("fp64", 1), ("fp64", 2)])
def test_streaming_batch_members_equal_single_runs(storage, spl):
    """23 steps (launches of spl steps and single steps for the rest, spl
    changed once mid-run): every member equals its single-cavity run bit
    for bit, Nusselt numbers included."""
    cfgs = _small_batch(storage, 2)
    seeds = [5 + k for k in range(len(cfgs))]
    amps = [1e-2] * len(cfgs)
    ref = _singles(cfgs, seeds, amps, 23)
    b = lbm.Batch(cfgs)
    b.steps_per_launch = spl
    b.init(seeds, amps)
    b.step(10)
    b.steps_per_launch = {1: 4, 2: 3, 3: 4, 4: 3, 5: 2}[spl] if storage != "fp64" else 3 - spl
    b.step(13)
    assert b.t == 23
    hot, cold = b.nusselt()
    for k in range(len(cfgs)):
        assert _fields_equal(b.cavity(k).fields(), ref[k][0]), k
        if ref[k][1] is not None:
            assert (hot[k], cold[k]) == ref[k][1], k
    assert not b.unstable().any()


@pytest.mark.parametrize("spl,graph_steps", [(4, 4), (4, 6), (5, 10), (5, 12)])
def test_streaming_graph_replay_matches_eager(spl, graph_steps):
    """Graphs of multi-step launches plus single steps (6 = one launch of
    four and two single steps, which leaves the buffers swapped; 12 = two of
    five and two single steps), keyed by the parity of t and the buffer;
    each replay checked against eager."""
    import torch
    cfgs = _small_batch("fp32", 2)
    seeds = list(range(len(cfgs)))
    amps = [1e-2] * len(cfgs)
    eager = lbm.Batch(cfgs)
    graph = lbm.Batch(cfgs)
    assert eager.steps_per_launch == graph.steps_per_launch == 5
    eager.steps_per_launch = graph.steps_per_launch = spl
    graph.set_config(block=256, grid_per_cu=0, graph_steps=graph_steps)
    eager.init(seeds, amps)
    graph.init(seeds, amps)
    for rep, n in enumerate((graph_steps, 2 * graph_steps + 1, 3, graph_steps, graph_steps + 2)):
        eager.step(n)
        graph.step(n)
        x = torch.randn(1024, device="cuda")
        torch.cuda.synchronize()
        assert float((x * 0).sum()) == 0.0
        assert graph.t == eager.t
        for k in range(len(cfgs)):
            assert _fields_equal(graph.cavity(k).fields(), eager.cavity(k).fields()), (rep, k)
        assert np.array_equal(np.nan_to_num(graph.nusselt()[0]), np.nan_to_num(eager.nusselt()[0]))
