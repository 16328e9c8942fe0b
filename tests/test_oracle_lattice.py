"""Pins of the oracle's lattice tables against closed forms and the paper.

The oracle builds its velocity sets, weights and moment bases itself; these
tests compare what it built with facts fixed independently of it:
isotropy of the weights, orthogonality of the bases, the forcing vectors the
paper prints (Section 2.2, Eqs. 6a/6b) against Guo's velocity-space force
term, the closed-form equilibrium moments, and the anti-bounce-back weight.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import lbmref

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def guo_force(e, w, u, F):
    """Guo, Zheng & Shi (2002) force term in velocity space (no 1 - s/2)."""
    eu = e @ u
    eF = e @ F
    return w * (((e - u) @ F) / CS2 + eu * eF / CS2 ** 2)


@pytest.mark.parametrize("dim", [2, 3])
def test_flow_lattice_isotropy(dim):
    e, w, _, _ = lbmref.lattice(dim, False)
    q = len(w)
    assert q == (9 if dim == 2 else 19)
    assert abs(w.sum() - 1.0) < 1e-15
    I = np.eye(3)
    for a in range(dim):
        assert abs(w @ e[:, a]) < 1e-15
        for b in range(dim):
            assert abs(w @ (e[:, a] * e[:, b]) - CS2 * I[a, b]) < 1e-15
            for c in range(dim):
                assert abs(w @ (e[:, a] * e[:, b] * e[:, c])) < 1e-15
                for d in range(dim):
                    m4 = w @ (e[:, a] * e[:, b] * e[:, c] * e[:, d])
                    ref = CS2 ** 2 * (I[a, b] * I[c, d] + I[a, c] * I[b, d] + I[a, d] * I[b, c])
                    assert abs(m4 - ref) < 1e-15


@pytest.mark.parametrize("dim,thermal", [(2, False), (3, False), (2, True), (3, True)])
def test_opposites_and_layout(dim, thermal):
    e, _, _, _ = lbmref.lattice(dim, thermal)
    rows = {tuple(v) for v in e}
    assert len(rows) == len(e)
    for v in e:
        assert tuple(-v) in rows
    if dim == 2:
        # Section 3.1 names f_2, f_5, f_6 (and g_2) as the populations that
        # move up and f_4, f_7, f_8 (g_4) as those that move down
        up = [i for i in range(len(e)) if e[i][1] == 1]
        down = [i for i in range(len(e)) if e[i][1] == -1]
        assert up == ([2, 5, 6] if not thermal else [2])
        assert down == ([4, 7, 8] if not thermal else [4])


NORMS = {
    (2, False): [9, 36, 36, 6, 12, 6, 12, 4, 4],
    (3, False): [19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8],
    (2, True): [5, 2, 2, 20, 4],
    (3, True): [7, 2, 2, 2, 42, 12, 4],
}


@pytest.mark.parametrize("key", list(NORMS))
def test_basis_orthogonal_and_inverse(key):
    dim, thermal = key
    _, _, M, Minv = lbmref.lattice(dim, thermal)
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))  # integer-exact
    assert np.diag(G).tolist() == NORMS[key]
    # the numerically inverted basis equals the closed form M^T D^-1
    closed = M.T / np.diag(G)[None, :]
    assert np.abs(Minv - closed).max() < 1e-14
    assert np.abs(Minv @ M - np.eye(len(M))).max() < 1e-14


def _eval_entry(entry, u, F):
    names = "xyz"
    val = 0.0
    for term, coef in entry.items():
        if term == "uF":
            val += coef * (u @ F)
        elif term[0] == "F":
            val += coef * F[names.index(term[1])]
        else:
            val += coef * u[names.index(term[0])] * F[names.index(term[1].lower())]
    return val


@pytest.mark.parametrize("dim", [2, 3])
def test_paper_forcing_vectors_equal_guo_moments(dim):
    gold = json.load(open(os.path.join(GOLD, "forcing_moments.json")))
    table = gold["d2q9" if dim == 2 else "d3q19"]
    e, w, M, _ = lbmref.lattice(dim, False)
    rng = np.random.default_rng(5)
    for _ in range(5):
        u = np.zeros(3)
        F = np.zeros(3)
        u[:dim] = rng.uniform(-0.1, 0.1, dim)
        F[:dim] = rng.uniform(-1e-3, 1e-3, dim)
        mf = M @ guo_force(e.astype(float), w, u, F)
        ref = np.array([_eval_entry(t, u, F) for t in table])
        assert np.abs(mf - ref).max() < 1e-17
        if dim == 2:
            printed = _eval_entry(gold["paper_as_printed_d2q9_last"], u, F)
            assert abs(mf[8] - printed) > 1e-8  # the printed entry is not the xy moment


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments_closed_form(dim):
    e, w, M, _ = lbmref.lattice(dim, False)
    rng = np.random.default_rng(11)
    rho = 1.03
    u = np.zeros(3)
    u[:dim] = rng.uniform(-0.08, 0.08, dim)
    eu = e @ u
    uu = u @ u
    feq = w * rho * (1 + eu / CS2 + eu ** 2 / (2 * CS2 ** 2) - uu / (2 * CS2))
    m = M @ feq
    ux, uy, uz = u
    if dim == 2:
        ref = [rho, rho * (-2 + 3 * uu), rho * (1 - 3 * uu), rho * ux, -rho * ux,
               rho * uy, -rho * uy, rho * (ux ** 2 - uy ** 2), rho * ux * uy]
    else:
        ref = [rho, rho * (-11 + 19 * uu), rho * (3 - 5.5 * uu), rho * ux,
               -2 / 3 * rho * ux, rho * uy, -2 / 3 * rho * uy, rho * uz,
               -2 / 3 * rho * uz, rho * (3 * ux ** 2 - uu), -0.5 * rho * (3 * ux ** 2 - uu),
               rho * (uy ** 2 - uz ** 2), -0.5 * rho * (uy ** 2 - uz ** 2),
               rho * ux * uy, rho * uy * uz, rho * ux * uz, 0, 0, 0]
    assert np.abs(m - np.array(ref)).max() < 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_thermal_weights_match_anti_bounce_back_omega(dim):
    """The ABB weight omega of Section 2.2 is twice the moving weight of
    the thermal equilibrium the oracle builds from n_eq, for every a_T."""
    gold = json.load(open(os.path.join(GOLD, "anti_bounce_back.json")))
    spec = gold["omega"]["d2q5" if dim == 2 else "d3q7"]
    for a_t in gold["a_t_samples"]:
        cfg = dict(dim=dim, n=(3, 3, 3 if dim == 3 else 1), bc=("periodic",) * 6,
                   nu=0.1, alpha=0.1, gbeta=0.0, a_t=a_t, t_hot=1.0, t_cold=0.0)
        o = lbmref.Oracle(cfg)
        d = o.derived()
        omega = (spec["num"] + a_t) / spec["den"]
        assert abs(d["omega"] - omega) < 1e-15
        # rest-state equilibrium: T = 1, u = 0
        N = o.N
        o.init_fields(None, np.zeros((dim, N)), np.ones(N))
        _, g = o.populations()
        moving = g[1:, 0]
        assert np.abs(moving - omega / 2).max() < 1e-15
        assert abs(g[0, 0] - (1 - omega / 2 * (2 * dim))) < 1e-15
        assert abs(d["cs2_t"] - omega) < 1e-15  # c_sT^2 = 2 w = omega


def test_splitmix64_published_outputs():
    gold = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    state = gold["seed"]
    for hexval in gold["outputs"]:
        assert lbmref.splitmix64(state) == int(hexval, 16)
        state = (state + 0x9E3779B97F4A7C15) & ((1 << 64) - 1)


def test_paper_roofline_arithmetic():
    """Section 3.1 derives its bandwidth roofline from values per node."""
    gold = json.load(open(os.path.join(GOLD, "paper_performance.json")))
    for key in ("2d", "3d"):
        mlups = gold["a100_bandwidth_gb_s"] * 1e9 / (
            gold["values_per_node"][key] * gold["bytes_per_value"] * 1e6)
        assert abs(mlups - gold["roofline_mlups"][key]) < 0.05
        frac = gold["measured_mlups"][key] / gold["roofline_mlups"][key]
        assert frac > 0.76  # the ">76%" of the abstract
