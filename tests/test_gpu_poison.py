"""Debug mode that fills the buffer each launch writes with NaN first: every
kernel lbm_step launches (one step per launch, the 2D streaming kernel at two
to five steps, the 3D two-step kernel, with and without wall rules, every
storage mode) must write every population of every node, so a poisoned run
stays finite and bitwise equal to the normal run.  (The pull scheme reads
only the state and writes only the other buffer; a node a kernel skipped
would read as NaN in the next state.)"""
import numpy as np
import pytest

from paper_2211_03160_amd import lbm, workloads as W

pytestmark = pytest.mark.gpu


def _run(cfg, spl, steps, poison):
    c = lbm.Cavity(cfg)
    c.steps_per_launch = spl
    c.debug_poison = poison
    assert c.debug_poison == poison
    c.init(1234, 1e-3)
    c.step(steps)
    return c


def _check(cfg, spl, steps, what):
    a = _run(cfg, spl, steps, False)
    b = _run(cfg, spl, steps, True)
    d = b.diagnostics()
    assert d["nonfinite"] == 0, (what, d)
    x, y = a.export_state(), b.export_state()
    if x != y:
        bad = np.flatnonzero(np.frombuffer(x, np.uint8) != np.frombuffer(y, np.uint8))
        pytest.fail(f"{what}: {bad.size} bytes differ, first at {bad[:8]}")


SPL2 = {"fp32": (1, 2, 3, 4, 5), "mixed": (1, 2, 3, 4), "fp16": (1, 2, 3, 4), "bf16": (1, 2, 3, 4), "fp64": (1, 2)}


@pytest.mark.parametrize("storage", list(SPL2))
def test_poison_2d_every_launch_mode(storage):
    # (200, 97): strips that clear the x walls beside ones that do not, a
    # ragged last strip and segment; periodic box: every strip wall-free
    layouts = {"rb": W.rayleigh_benard(2, (200, 97), ra=1e5, pr=0.71, storage=storage),
               "side": W.side_heated(2, (131, 70), ra=1e5, pr=0.71, storage=storage),
               "box": W.periodic_box(2, (96, 33), nu=0.02, alpha=0.03, gbeta=1e-4, storage=storage)}
    for name, cfg in layouts.items():
        for spl in SPL2[storage]:
            _check(cfg, spl, 2 * spl + 1, f"2d {name} {storage} spl {spl}")


@pytest.mark.parametrize("storage,spl", [("fp32", 1), ("fp32", 2), ("bf16", 2), ("fp16", 1), ("mixed", 2),
                                         ("fp64", 1)])
def test_poison_3d(storage, spl):
    # 65 x 33 x 40: several tiles and z segments, wall-free blocks inside
    layouts = {"rb": W.rayleigh_benard(3, (65, 33, 40), ra=5e4, pr=0.71, storage=storage),
               "box": W.periodic_box(3, (34, 17, 12), nu=0.02, alpha=0.03, gbeta=1e-4, storage=storage)}
    for name, cfg in layouts.items():
        _check(cfg, spl, 5, f"3d {name} {storage} spl {spl}")


def test_poison_argument_checks():
    c = lbm.Cavity(W.rayleigh_benard(2, (17, 9), ra=1e4, pr=0.71, storage="fp32"))
    assert c.debug_poison is False
    with pytest.raises(lbm.LBMError) as e:
        lib = lbm.lib()
        c._check(lib.lbm_set_debug_poison(c._h, 2))
    assert e.value.status == -1
