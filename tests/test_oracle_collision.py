"""Pins of the oracle's collision operators (Section 2.2, Eqs. 5-7).

With every relaxation rate equal, an MRT operator is the single-relaxation
(BGK) operator, whose textbook form needs no moment basis at all:
    f+ = f - s (f - f_eq) + (1 - s/2) F~_Guo,   g+ = g - q (g - g_eq).
The test drives one oracle step on a random periodic state, undoes the
streaming with array rolls (a pure permutation) and compares with that form.
This pins the bases, their inverses, the equilibria, the forcing moments and
the (I - S/2) factor at once.  With the default (unequal) rates it pins the
collision invariants: rho and T unchanged, momentum changed by exactly F.
"""
import numpy as np
import pytest

from oracle import lbmref

CS2 = 1.0 / 3.0


def unstream(pop, e, shape):
    """Undo a periodic pull: f+_i(x) = f_i(x + e_i, t + 1)."""
    out = np.empty_like(pop)
    axes = {0: len(shape) - 1, 1: len(shape) - 2, 2: len(shape) - 3}
    for i in range(pop.shape[0]):
        a = pop[i].reshape(shape)
        for ax in range(3):
            if e[i][ax] and axes[ax] >= 0:
                a = np.roll(a, -e[i][ax], axis=axes[ax])
        out[i] = a.ravel()
    return out


def random_state(dim, shape, rng):
    e, w, _, _ = lbmref.lattice(dim, False)
    eg, wg, _, _ = lbmref.lattice(dim, True)
    N = int(np.prod(shape))
    f = w[:, None] * (1 + 0.05 * rng.standard_normal((len(w), N)))
    g = wg[:, None] * (0.5 + 0.2 * rng.standard_normal((len(wg), N)))
    return f, g


def moments(dim, f, g, gbeta, t0):
    e, _, _, _ = lbmref.lattice(dim, False)
    rho = f.sum(0)
    j = e.T.astype(float) @ f
    T = g.sum(0)
    F = np.zeros_like(j)
    F[dim - 1] = rho * gbeta * (T - t0)  # buoyancy along +y (2D) / +z (3D)
    u = (j + 0.5 * F) / rho
    return rho, j, T, F, u


@pytest.mark.parametrize("dim", [2, 3])
def test_equal_rates_reduce_to_bgk_with_guo_forcing(dim):
    rng = np.random.default_rng(100 + dim)
    shape = (4, 5) if dim == 2 else (3, 4, 5)
    n = tuple(reversed(shape)) + ((1,) if dim == 2 else ())
    base = dict(dim=dim, n=n, bc=("periodic",) * 6, nu=0.07, alpha=0.05,
                gbeta=2e-3, t_hot=1.0, t_cold=0.0)
    d = lbmref.Oracle(base).derived()
    s, qj = d["s_nu"], d["q_j"]
    cfg = dict(base, s_e=s, s_eps=s, s_q=s, s_pi=s, s_m=s, q_e=qj, q_nu=qj)
    o = lbmref.Oracle(cfg)
    f, g = random_state(dim, shape, rng)
    o.set_populations(f, g)
    o.step(1)
    f1, g1 = o.populations()
    e, w, _, _ = lbmref.lattice(dim, False)
    eg, _, _, _ = lbmref.lattice(dim, True)
    fp = unstream(f1, e, shape)
    gp = unstream(g1, eg, shape)

    rho, j, T, F, u = moments(dim, f, g, d["gbeta"], d["t0"])
    eu = e.astype(float) @ u
    uu = (u * u).sum(0)
    feq = w[:, None] * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))
    eF = e.astype(float) @ F
    uF = (u * F).sum(0)
    guo = w[:, None] * ((eF - uF) / CS2 + eu * eF / CS2 ** 2)
    f_bgk = f - s * (f - feq) + (1 - s / 2) * guo
    assert np.abs(fp - f_bgk).max() < 2e-15

    # thermal BGK with the linear equilibrium whose moving weight is
    # omega/2 (the anti-bounce-back weight) and c_sT^2 = omega
    om = d["omega"]
    wg = np.array([1 - dim * om] + [om / 2] * (2 * dim))
    egu = eg.astype(float) @ u
    geq = wg[:, None] * T * (1 + egu / om)
    g_bgk = g - qj * (g - geq)
    assert np.abs(gp - g_bgk).max() < 2e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_default_rates_collision_invariants(dim):
    rng = np.random.default_rng(7 + dim)
    shape = (4, 5) if dim == 2 else (3, 4, 5)
    n = tuple(reversed(shape)) + ((1,) if dim == 2 else ())
    cfg = dict(dim=dim, n=n, bc=("periodic",) * 6, nu=0.02, alpha=0.03,
               gbeta=5e-3, t_hot=1.0, t_cold=0.0)
    o = lbmref.Oracle(cfg)
    d = o.derived()
    f, g = random_state(dim, shape, rng)
    o.set_populations(f, g)
    o.step(1)
    f1, g1 = o.populations()
    e, _, _, _ = lbmref.lattice(dim, False)
    eg, _, _, _ = lbmref.lattice(dim, True)
    fp = unstream(f1, e, shape)
    gp = unstream(g1, eg, shape)
    rho, j, T, F, _ = moments(dim, f, g, d["gbeta"], d["t0"])
    assert np.abs(fp.sum(0) - rho).max() < 1e-14
    assert np.abs(gp.sum(0) - T).max() < 1e-14
    jp = e.T.astype(float) @ fp
    assert np.abs(jp - (j + F)).max() < 1e-15
    # the non-conserved moments really were relaxed
    assert np.abs(fp - f).max() > 1e-3
