"""Two to four steps per launch (2D temporal blocking) against one step
per launch.

The streaming kernels apply the same per-node update to the same stored
values (the intermediate rows stay in registers, rounded through the storage
type), so the whole exported state -- populations, both wall-flux slots and
t -- must be bitwise identical, in every storage mode and boundary layout,
including grids narrower than one strip, grids whose rows wrap more than
once, ragged strips and segments, and step counts that the steps per launch
do not divide (which end with shorter launches), and tall grids whose
inner segments take the sweep without wall rules.  Parity of the default
(multi-step) path with the oracle is covered by test_gpu_parity."""
import numpy as np
import pytest

from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu

STORAGES = ["fp32", "fp64", "fp16", "bf16", "mixed"]
# (200, 1000): its inner strips and segments clear every wall (a strip
# needs about 116 columns to clear both x walls at four steps per launch),
# so in the walled layouts wavefronts without wall rules run next to ones
# with them; in the periodic box every unit takes the wall-free sweep
SHAPES = [(129, 129), (67, 45), (64, 19), (65, 20), (5, 7), (2, 2), (300, 3), (7, 200), (1, 33), (40, 1),
          (200, 1000)]


def _layouts(shape, storage):
    return {
        "rb": W.rayleigh_benard(2, shape, ra=5e4, pr=0.71, storage=storage),
        "side": W.side_heated(2, shape, ra=5e4, pr=0.71, storage=storage),
        "box": W.periodic_box(2, shape, nu=0.02, alpha=0.03, gbeta=1e-4, storage=storage),
    }


def _run(cfg, spl, steps, seed=9, amp=2e-2):
    c = lbm.Cavity(cfg)
    c.steps_per_launch = spl
    assert c.steps_per_launch == spl
    c.init(seed, amp)
    c.step(steps)
    return c


@pytest.mark.parametrize("storage", STORAGES)
@pytest.mark.parametrize("shape", SHAPES)
def test_multi_step_bitwise(storage, shape):
    """23 steps: 11 launches of two + one single step, 7 of three + one of
    two, 5 of four + one of three, 4 of five + one of three (FP32), against
    23 single steps (FP64: two)."""
    for name, cfg in _layouts(shape, storage).items():
        if name != "box" and min(shape) < 2:
            continue  # a walled axis needs two nodes
        one = _run(cfg, 1, 23)
        a = one.export_state()
        for spl in {"fp64": (2,), "fp32": (2, 3, 4, 5)}.get(storage, (2, 3, 4)):
            other = _run(cfg, spl, 23)
            assert one.t == other.t == 23
            b = other.export_state()
            assert len(a) == len(b)
            if a != b:
                x, y = np.frombuffer(a, np.uint8), np.frombuffer(b, np.uint8)
                bad = np.flatnonzero(x != y)
                pytest.fail(f"{name} {shape} {storage}, {spl} steps per launch: {bad.size} bytes differ, "
                            f"first at {bad[:8]}")


SHAPES3 = [(17, 19, 21), (33, 31, 50), (5, 7, 9), (40, 16, 3), (2, 2, 2), (31, 15, 100), (65, 29, 31)]


def _layouts3(shape, storage):
    return {
        "rb": W.rayleigh_benard(3, shape, ra=5e4, pr=0.71, storage=storage),
        "rb_periodic": W.rayleigh_benard(3, shape, ra=5e4, pr=0.71, lateral="periodic", storage=storage),
        "side": W.side_heated(3, shape, ra=5e4, pr=0.71, storage=storage),
        "box": W.periodic_box(3, shape, nu=0.02, alpha=0.03, gbeta=1e-4, storage=storage),
    }


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16", "mixed"])
@pytest.mark.parametrize("shape", SHAPES3)
def test_3d_two_steps_bitwise(storage, shape):
    """3D, two steps per launch (the LDS plane ring): 9 steps = 4 launches of
    two + one single step, against 9 single steps; tiles and z segments
    ragged, periodic and walled axes, every storage with FP32 arithmetic."""
    for name, cfg in _layouts3(shape, storage).items():
        if name != "box" and min(shape) < 2:
            continue
        one = _run(cfg, 1, 9)
        two = _run(cfg, 2, 9)
        assert one.t == two.t == 9
        a, b = one.export_state(), two.export_state()
        if a != b:
            x, y = np.frombuffer(a, np.uint8), np.frombuffer(b, np.uint8)
            bad = np.flatnonzero(x != y)
            pytest.fail(f"{name} {shape} {storage}: {bad.size} bytes differ, first at {bad[:8]}")
        if name == "rb":
            assert one.nusselt() == two.nusselt()


def test_two_step_after_single_steps_and_nusselt():
    """Mixing launch modes mid-run keeps the state and the flux history."""
    cfg = W.rayleigh_benard(2, (257, 129), ra=1e5, pr=0.71, storage="fp32")
    ref = _run(cfg, 1, 0)
    mix = _run(cfg, 1, 0)
    for n, spl in ((3, 2), (4, 1), (1, 3), (6, 3), (5, 2), (7, 4), (9, 3), (4, 4), (11, 5), (5, 5), (3, 5)):
        ref.step(n)
        mix.steps_per_launch = spl
        mix.step(n)
    assert ref.export_state() == mix.export_state()
    assert ref.nusselt() == mix.nusselt()


def test_steps_per_launch_arguments():
    defaults = {"fp32": 5, "mixed": 4, "fp16": 3, "bf16": 4, "fp64": 2}
    for st, k in defaults.items():
        assert lbm.Cavity(W.rayleigh_benard(2, (33, 17), ra=1e4, pr=0.71, storage=st)).steps_per_launch == k
    c2 = lbm.Cavity(W.rayleigh_benard(2, (33, 17), ra=1e4, pr=0.71, storage="fp32"))
    for bad in (0, 6, -1):
        with pytest.raises(lbm.LBMError) as e:
            c2.steps_per_launch = bad
        assert e.value.status == -1
    for st in ("fp16", "bf16", "mixed"):  # five steps: FP32 storage only
        c16 = lbm.Cavity(W.rayleigh_benard(2, (33, 17), ra=1e4, pr=0.71, storage=st))
        with pytest.raises(lbm.LBMError) as e:
            c16.steps_per_launch = 5
        assert e.value.status == -5
    c64 = lbm.Cavity(W.rayleigh_benard(2, (33, 17), ra=1e4, pr=0.71, storage="fp64"))
    for k in (3, 4, 5):
        with pytest.raises(lbm.LBMError) as e:
            c64.steps_per_launch = k
        assert e.value.status == -5
    defaults3 = {"fp32": 2, "mixed": 1, "fp16": 1, "bf16": 1, "fp64": 1}
    for st, k in defaults3.items():
        assert lbm.Cavity(W.rayleigh_benard(3, (9, 9, 9), ra=1e4, pr=0.71, storage=st)).steps_per_launch == k
    c3 = lbm.Cavity(W.rayleigh_benard(3, (9, 9, 9), ra=1e4, pr=0.71, storage="fp32"))
    for k in (3, 4, 5):
        with pytest.raises(lbm.LBMError) as e:
            c3.steps_per_launch = k
        assert e.value.status == -5
    c3.steps_per_launch = 2
    c3.steps_per_launch = 1
    c3d = lbm.Cavity(W.rayleigh_benard(3, (9, 9, 9), ra=1e4, pr=0.71, storage="fp64"))
    with pytest.raises(lbm.LBMError) as e:
        c3d.steps_per_launch = 2
    assert e.value.status == -5
    c2.steps_per_launch = 3
    assert c2.steps_per_launch == 3


# Shapes whose population arrays (f, or g in the mixed mode) exceed 4 GiB,
# which takes the streaming kernels' 64-bit addressing path: stores through
# a buffer resource based at the first tile of each row.
BIG = [("fp64", (8193, 8193)), ("fp32", (12289, 12289)), ("mixed", (14849, 14849)),
       ("fp16", (15489, 15489)), ("bf16", (15489, 15489))]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("storage,shape", BIG)
def test_multi_step_beyond_4gib_arrays(storage, shape):
    """Moments and wall fluxes agree bitwise after 7 steps with one step per
    launch and with the storage mode's default (7 = 5 + 2, 4 + 3, 3 + 3 + 1
    or 2 + 2 + 2 + 1 steps per launch)."""
    import torch
    cfg = W.rayleigh_benard(2, shape, ra=1e8, pr=0.71, storage=storage)
    N = shape[0] * shape[1]
    qf, qg = 9, 5
    ef = {"fp64": 8, "fp32": 4, "mixed": 2, "fp16": 2, "bf16": 2}[storage]
    eg = {"fp64": 8, "fp32": 4, "mixed": 4, "fp16": 2, "bf16": 2}[storage]
    assert max(N * qf * ef, N * qg * eg) > 2 ** 32  # the 64-bit path
    res = []
    for spl in (1, {"fp64": 2, "fp32": 5, "mixed": 4, "fp16": 3, "bf16": 4}[storage]):
        print(f"{storage} {shape}: {spl} steps per launch", flush=True)
        c = _run(cfg, spl, 7, amp=1e-3)
        rho = torch.empty(N, dtype=torch.float64, device="cuda")
        u = torch.empty(2 * N, dtype=torch.float64, device="cuda")
        T = torch.empty(N, dtype=torch.float64, device="cuda")
        c._check(lbm.lib().lbm_fields(c._h, rho.data_ptr(), u.data_ptr(), T.data_ptr()))
        res.append((rho, u, T, c.wall_flux()))
        del c
        torch.cuda.empty_cache()
    (r1, u1, t1, w1), (r2, u2, t2, w2) = res
    for name, a, b in (("rho", r1, r2), ("u", u1, u2), ("T", t1, t2)):
        if not torch.equal(a, b):
            bad = torch.nonzero(a != b).flatten()
            pytest.fail(f"{storage} {shape}: {name} differs at {bad.numel()} entries, first {bad[:8].tolist()}")
    assert all(np.array_equal(a, b) for a, b in zip(w1, w2))
    del res
    torch.cuda.empty_cache()
