"""Pins of the oracle's FP64 diagnostics (mass, energy, max |u|, the volume
Nusselt number and the Reynolds number) against values the mathematics
fixes, not the oracle's own sums.

The paper prints no Nusselt or Reynolds number (Section 2.3), so these
definitions are readings: Nu_vol = 1 + H <u_g (T - T0)> / (alpha dT) with
u_g the upward velocity, Re = sqrt(<|u|^2>) H / nu, H the node count along
gravity.  Two closed forms pin them:

* a state set by init_fields with no buoyancy, u_g = A (sin(k x) + c) and
  T = T0 + B sin(k x) with k = 2 pi / W on a periodic axis of W nodes: the
  moments of the equilibrium populations are the fields themselves, and the
  discrete means over one period are <sin> = 0, <sin^2> = 1/2, so
  <u_g (T - T0)> = A B / 2 and <|u|^2> = A^2 (1/2 + c^2);
* plane Poiseuille flow between half-way bounce-back walls, which the
  operator reproduces to 1e-9 (see test_oracle_physics): its Reynolds number
  is the root mean square of the analytic profile times H / nu.

The offset c makes <u_g> nonzero, so T in place of T - T0 changes Nu_vol;
nu differs from alpha in every case, and the expected values are computed
here from those formulas, not from the oracle.
"""
import math

import numpy as np
import pytest

from oracle import lbmref
from paper_2211_03160_amd import workloads as W


def _closed_form_state(dim, n, A, c, B, nu, alpha):
    cfg = W.periodic_box(dim, n, nu=nu, alpha=alpha, gbeta=0.0)
    o = lbmref.Oracle(cfg)
    Wd = n[0]
    x = np.arange(Wd)
    s = np.sin(2 * np.pi * x / Wd)
    shape = o.shape  # (ny, nx) or (nz, ny, nx)
    bshape = (1,) * (len(shape) - 1) + (Wd,)
    u = np.zeros((dim,) + shape)
    u[dim - 1] = (A * (s + c)).reshape(bshape)
    T0 = 0.5 * (cfg["t_hot"] + cfg["t_cold"])
    T = np.broadcast_to((T0 + B * s).reshape(bshape), shape)
    o.init_fields(None, u.reshape(dim, -1), np.ascontiguousarray(T).ravel())
    return o, cfg, T0


@pytest.mark.parametrize("dim,n", [(2, (16, 5)), (3, (8, 3, 4))])
def test_volume_nusselt_and_reynolds_closed_form(dim, n):
    A, c, B, nu, alpha = 0.01, 0.5, 0.2, 0.05, 0.04
    o, cfg, T0 = _closed_form_state(dim, n, A, c, B, nu, alpha)
    d = o.diagnostics()
    H = n[-1]  # nodes along gravity (y in 2D, z in 3D)
    dT = cfg["t_hot"] - cfg["t_cold"]
    N = int(np.prod(n))
    assert abs(d["nu_vol"] - (1.0 + H * (A * B / 2) / (alpha * dT))) < 1e-12
    assert abs(d["re"] - A * math.sqrt(0.5 + c * c) * H / nu) < 1e-12 * (A * H / nu)
    assert abs(d["umax"] - A * (1 + c)) < 1e-15  # sin reaches 1 at x = W/4
    assert abs(d["mass"] - N) < 1e-12 * N
    assert abs(d["energy"] - N * T0) < 1e-12 * N


def test_volume_nusselt_is_one_at_rest_and_tracks_the_sign():
    """A resting state gives exactly 1; the upward flow of warm fluid
    raises Nu_vol above 1, of cold fluid lowers it."""
    o, _, _ = _closed_form_state(2, (12, 4), 0.0, 0.0, 0.3, 0.05, 0.04)
    assert o.diagnostics()["nu_vol"] == 1.0
    up = _closed_form_state(2, (12, 4), 0.01, 0.0, 0.2, 0.05, 0.04)[0].diagnostics()["nu_vol"]
    down = _closed_form_state(2, (12, 4), 0.01, 0.0, -0.2, 0.05, 0.04)[0].diagnostics()["nu_vol"]
    assert up > 1.0 > down
    assert abs((up - 1.0) + (down - 1.0)) < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_reynolds_number_of_plane_poiseuille(dim):
    """Walls on the x faces, periodic along the others, uniform buoyancy
    along gravity: u(x) = g beta dT (x + 1/2)(W - 1/2 - x) / (2 nu), and
    Re = sqrt(mean_x u(x)^2) H / nu with H the node count along gravity."""
    Wd, nu, gb, dT = 15, 0.12, 1e-4, 0.1
    n = (Wd, 3) if dim == 2 else (Wd, 3, 4)
    bc = ("adiabatic", "adiabatic") + ("periodic",) * 4
    cfg = dict(dim=dim, n=n, bc=bc, t_wall=(0,) * 6, nu=nu, alpha=0.1, gbeta=gb,
               t_hot=1.0, t_cold=0.0)
    o = lbmref.Oracle(cfg)
    N = int(np.prod(n))
    o.init_fields(None, np.zeros((dim, N)), np.full(N, 0.5 + dT))
    o.step(6000 if dim == 2 else 5000)
    x = np.arange(Wd)
    prof = gb * dT / (2 * nu) * (x + 0.5) * (Wd - 0.5 - x)
    H = n[-1]
    re = math.sqrt(np.mean(prof ** 2)) * H / nu
    d = o.diagnostics()
    assert abs(d["re"] / re - 1) < 1e-9
    assert abs(d["umax"] / prof.max() - 1) < 1e-9


def test_derive_without_state_matches_create():
    """lbmref_derive gives the mapping of lbmref_create, and the free-fall
    scaling of Eqs. 2-4: nu = U H sqrt(Pr/Ra), alpha = U H / sqrt(Pr Ra),
    g beta = U^2 / (dT H)."""
    cfg = W.rayleigh_benard(2, (33, 17), ra=3e4, pr=2.0, storage="fp64")
    d = lbmref.derive(cfg)
    assert d == lbmref.Oracle(cfg).derived()
    U, H = 0.1, 17
    assert abs(d["nu"] - U * H * math.sqrt(2.0 / 3e4)) < 1e-15
    assert abs(d["alpha"] - U * H / math.sqrt(2.0 * 3e4)) < 1e-15
    assert abs(d["gbeta"] - U * U / H) < 1e-18
    with pytest.raises(lbmref.OracleError):
        lbmref.derive(dict(cfg, ra=-1.0))
