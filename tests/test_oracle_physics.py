"""Physics pins of the FP64 oracle: results the method fixes exactly or
that have closed forms, independent of the oracle's own arithmetic.

* conduction: the linear profile between isothermal walls is a fixed point
  of stream + anti-bounce-back (Section 2.2) for any rates and a_T, so the
  wall Nusselt number is exactly 1 and the fluid stays at rest;
* energy: sum T changes per step by exactly the anti-bounce-back link flux;
* mass: sum rho is conserved in closed and periodic boxes, and a uniform
  force adds exactly sum F to the momentum per step;
* plane Poiseuille flow between half-way bounce-back walls (Section 2.2) is
  reproduced exactly by the two-rate operator with Lambda = 3/16;
* shear and thermal waves decay at nu k^2 and alpha k^2 to second order;
* Rayleigh-Benard onset between rigid plates at Ra_c = 1707.76;
* odd grids (Section 2.3) remove the period-two lattice mode.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import lbmref
from paper_2211_03160_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dim,n,a_t,q_e,q_nu", [
    (2, (16, 32), None, None, None),
    (2, (9, 20), 0.0, 0.6, 1.7),
    (2, (8, 11), -3.0, 1.3, 0.4),
    (3, (5, 6, 12), None, None, None),
    (3, (4, 5, 9), 0.5, 0.7, 1.5),
])
def test_conduction_is_exact(dim, n, a_t, q_e, q_nu):
    cfg = W.rayleigh_benard(dim, n, ra=2e4, pr=0.71, storage="fp64", gbeta=0.0,
                            a_t=a_t, q_e=q_e, q_nu=q_nu)
    o = lbmref.Oracle(cfg)
    o.init(3, 0.0)
    o.step(400)
    _, u, T = o.fields()
    H = n[-1]
    z = np.arange(H) + 0.5
    prof = 1.0 - z / H
    Tref = prof[:, None] if dim == 2 else prof[:, None, None]
    assert np.abs(T - Tref).max() < 1e-13
    assert np.abs(u).max() < 1e-14  # rest up to rounding of the moment sums
    nh, nc = o.nusselt()
    assert abs(nh - 1) < 1e-12 and abs(nc - 1) < 1e-12


def test_conduction_side_heated_init_profile():
    cfg = W.side_heated(2, (11, 7), ra=1e5, storage="fp64")
    o = lbmref.Oracle(cfg)
    o.init(1, 0.0)
    _, _, T = o.fields()
    x = np.arange(11) + 0.5
    assert np.abs(T - (1 - x / 11)[None, :]).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_energy_identity(dim):
    n = (13, 11) if dim == 2 else (7, 6, 9)
    cfg = W.rayleigh_benard(dim, n, ra=5e4, pr=0.71, storage="fp64")
    o = lbmref.Oracle(cfg)
    o.init(42, 0.05)
    o.step(50)
    for _ in range(4):
        e0 = o.diagnostics()["energy"]
        o.step(1)
        e1 = o.diagnostics()["energy"]
        last, _ = o.wall_flux()
        assert abs(last.sum()) > 1e-6
        assert abs((e1 - e0) - last.sum()) < 1e-12 * max(1.0, abs(e0))


def test_energy_conserved_periodic_and_adiabatic():
    cfg = W.periodic_box(2, (9, 7), nu=0.05, alpha=0.04, gbeta=1e-3)
    o = lbmref.Oracle(cfg)
    rng = np.random.default_rng(1)
    o.init_fields(None, 0.01 * rng.standard_normal((2, 63)), 0.5 + 0.1 * rng.standard_normal(63))
    e0 = o.diagnostics()["energy"]
    o.step(200)
    assert abs(o.diagnostics()["energy"] - e0) < 1e-12
    cfg = W.rayleigh_benard(2, (9, 7), ra=1e4, pr=0.71, storage="fp64")
    cfg["bc"] = ("adiabatic",) * 4 + ("periodic",) * 2
    o = lbmref.Oracle(cfg)
    o.init_fields(None, 0.01 * rng.standard_normal((2, 63)), 0.5 + 0.1 * rng.standard_normal(63))
    e0 = o.diagnostics()["energy"]
    o.step(200)
    assert abs(o.diagnostics()["energy"] - e0) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_conserved_closed_box(dim):
    n = (17, 17) if dim == 2 else (7, 7, 7)
    cfg = W.rayleigh_benard(dim, n, ra=1e5, pr=0.71, storage="fp64")
    o = lbmref.Oracle(cfg)
    o.init(9, 0.05)
    m0 = o.diagnostics()["mass"]
    o.step(300)
    d = o.diagnostics()
    assert d["umax"] > 1e-5  # the flow is not at rest
    assert abs(d["mass"] - m0) / m0 < 300 * 4 * 2.2e-16 * 10


def test_uniform_force_momentum_budget():
    """Periodic box, uniform T != T0: each step adds sum F to sum j."""
    cfg = W.periodic_box(2, (6, 5), nu=0.1, alpha=0.1, gbeta=1e-3)
    o = lbmref.Oracle(cfg)
    N = 30
    o.init_fields(None, np.zeros((2, N)), np.full(N, 0.8))
    e, _, _, _ = lbmref.lattice(2, False)
    for _ in range(3):
        f0, _ = o.populations()
        o.step(1)
        f1, _ = o.populations()
        rho = f0.sum(0)
        F = rho * 1e-3 * (0.8 - 0.5)
        dj = (e[:, 1] @ f1).sum() - (e[:, 1] @ f0).sum()
        # sums of N order-one values: a few ulp per node
        assert abs(dj - F.sum()) < N * 1e-16
        assert abs((e[:, 0] @ f1).sum() - (e[:, 0] @ f0).sum()) < N * 1e-16


@pytest.mark.parametrize("dim", [2, 3])
def test_poiseuille_between_bounce_back_walls(dim):
    """Walls on the x faces, periodic along the others, uniform buoyancy
    along the gravity axis: the steady profile u(x) = g (x+1/2)(W-1/2-x)/2nu
    with walls half a link outside the first and last nodes."""
    Wd, nu, gb, dT = 15, 0.12, 1e-4, 0.1
    if dim == 2:
        n, bc = (Wd, 3), ("adiabatic", "adiabatic", "periodic", "periodic", "periodic", "periodic")
    else:
        n, bc = (Wd, 3, 3), ("adiabatic", "adiabatic", "periodic", "periodic", "periodic", "periodic")
    cfg = dict(dim=dim, n=n, bc=bc, t_wall=(0,) * 6, nu=nu, alpha=0.1, gbeta=gb,
               t_hot=1.0, t_cold=0.0)
    o = lbmref.Oracle(cfg)
    N = int(np.prod(n))
    o.init_fields(None, np.zeros((dim, N)), np.full(N, 0.5 + dT))
    o.step(6000 if dim == 2 else 5000)
    _, u, T = o.fields()
    x = np.arange(Wd)
    ref = gb * dT / (2 * nu) * (x + 0.5) * (Wd - 0.5 - x)
    prof = u[dim - 1].reshape(-1, Wd)
    assert np.abs(prof - ref[None, :]).max() / ref.max() < 1e-9
    for a in range(dim - 1):
        assert np.abs(u[a]).max() < 1e-14


def _wave_decay(dim, Nn, which, nu=0.05, alpha=0.05):
    n = (4, Nn) if dim == 2 else (4, 4, Nn)
    cfg = W.periodic_box(dim, n, nu=nu, alpha=alpha)
    o = lbmref.Oracle(cfg)
    N = int(np.prod(n))
    k = 2 * np.pi / Nn
    ax = np.arange(Nn)
    shape = o.shape
    prof = np.sin(k * ax).reshape((Nn,) + (1,) * (dim - 1))
    u = np.zeros((dim,) + shape)
    T = np.full(shape, 0.5)
    if which == "shear":
        u[0] = 1e-4 * prof
        rate = nu * k * k
    else:
        T = T + 1e-3 * prof
        rate = alpha * k * k
    o.init_fields(None, u.reshape(dim, N), T.ravel())

    def amp():
        _, uu, TT = o.fields()
        fld = uu[0] if which == "shear" else TT - 0.5
        return 2 * np.mean(fld * prof)

    o.step(int(0.1 / rate))
    a1, t1 = amp(), o.t
    o.step(int(0.5 / rate))
    a2, t2 = amp(), o.t
    return -math.log(a2 / a1) / (t2 - t1) / rate - 1


@pytest.mark.parametrize("which", ["shear", "thermal"])
def test_wave_decay_second_order(which):
    e16 = _wave_decay(2, 16, which)
    e32 = _wave_decay(2, 32, which)
    assert abs(e32) < 2e-3
    assert 3.5 < e16 / e32 < 4.5


@pytest.mark.parametrize("which", ["shear", "thermal"])
def test_wave_decay_3d(which):
    assert abs(_wave_decay(3, 32, which)) < 2e-3


def _growth(H, ra):
    Wd = 2 * H
    cfg = W.rayleigh_benard(2, (Wd, H), ra=ra, pr=0.71, lateral="periodic", storage="fp64")
    o = lbmref.Oracle(cfg)
    x = np.arange(Wd)
    y = np.arange(H)[:, None] + 0.5
    T = 1 - y / H + 1e-4 * np.sin(np.pi * y / H) * np.cos(2 * np.pi * x[None, :] / Wd)
    o.init_fields(None, np.zeros((2, Wd * H)), T.ravel())

    def amp():
        _, u, _ = o.fields()
        return math.sqrt(np.mean(u[1] ** 2))

    o.step(4000)
    a1 = amp()
    o.step(8000)
    return math.log(amp() / a1) / 8000


def test_rayleigh_benard_onset():
    gold = json.load(open(os.path.join(GOLD, "rb_onset.json")))
    rac = gold["ra_c"]
    lo, hi = 0.9 * rac, 1.1 * rac
    glo, ghi = _growth(17, lo), _growth(17, hi)
    assert glo < 0 < ghi
    crossing = lo - glo * (hi - lo) / (ghi - glo)
    assert abs(crossing / rac - 1) < 0.015


def test_odd_grid_removes_period_two_mode():
    """Section 2.3: odd node counts suppress the spurious oscillation."""
    res = {}
    for n in ((16, 32), (17, 33)):
        cfg = W.rayleigh_benard(2, n, ra=1000, pr=0.71, storage="fp64")
        o = lbmref.Oracle(cfg)
        o.init(1, 0.0)
        o.step(20000)
        last, prev = o.wall_flux()
        res[n] = (abs(last[2] - prev[2]) / abs(last[2]), o.diagnostics()["umax"], o.nusselt())
    even, odd = res[(16, 32)], res[(17, 33)]
    assert even[0] > 1e-4 and even[1] > 1e-7
    assert odd[0] < 1e-7 and odd[1] < 1e-9  # hydrostatic conduction below onset
    for nh, nc in (even[2], odd[2]):  # the two-step mean removes the mode
        assert abs(nh - 1) < 1e-9 and abs(nc - 1) < 1e-9
