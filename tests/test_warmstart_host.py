"""Host-side logic of the warm-start evaluation on synthetic Nusselt records:
the settling criterion, the assessment against an independent reference run and
the bootstrap intervals.  No GPU is touched."""
import math

import numpy as np

from paper_2211_03160_amd import warmstart as WS


def test_steps_to_steady_on_a_clean_exponential():
    # Nu(t) = 1 + exp(-t/tau), sampled every `every` steps: the window mean
    # over [i, i + w) is 1 + exp(-i/tau) (1 - exp(-w/tau)) / (w (1 - exp(-1/tau)))
    # in record units; it first stays within tol once that excess <= tol
    every, tau, w, tol = 10, 50.0, 20, 0.01
    i = np.arange(2000)
    h = 1.0 + np.exp(-i / tau)
    got = WS.steps_to_steady(h, every, 1.0, w, tol)
    k = (1 - math.exp(-w / tau)) / (w * (1 - math.exp(-1 / tau)))
    first = math.ceil(tau * math.log(k / tol))
    assert got == (first + w) * every
    # never inside the band: None; shorter than a window: None
    assert WS.steps_to_steady(h + 1.0, every, 1.0, w, tol) is None
    assert WS.steps_to_steady(h[:w - 1], every, 1.0, w, tol) is None


def test_assess_widens_the_band_for_a_fluctuating_reference():
    rng = np.random.default_rng(3)
    n, w, tail = 1200, 50, 360
    # steady cell: tiny noise, band stays at 1%
    ref = 4.0 + 1e-4 * rng.standard_normal(n)
    r = WS.assess(ref.copy(), ref.copy(), ref, 100, w, tail)
    assert r["band"] == 0.01 and r["same_state_plain"] and r["steps_plain"] == w * 100
    # unsteady cell: red noise whose window means wander by several percent
    x = np.zeros(n)
    for k in range(1, n):
        x[k] = 0.98 * x[k - 1] + 0.05 * rng.standard_normal()
    ref = 10.0 + x
    _, sem, spread = WS.tail_stats(ref, w, tail)
    r = WS.assess(np.roll(ref, 400), np.roll(ref, 800), ref, 100, w, tail)
    assert math.isclose(r["band"], max(0.01, 3 * math.hypot(spread, sem)))
    assert r["band"] > 0.01


def test_assess_flags_another_state_and_a_faster_start():
    rng = np.random.default_rng(5)
    n, w, tail = 1000, 40, 300
    t = np.arange(n)
    noise = lambda: 0.02 * rng.standard_normal(n)
    ref = 5.0 + noise()
    plain = 5.0 + 2.0 * np.exp(-t / 150.0) + noise()
    warm = 5.0 + 2.0 * np.exp(-t / 15.0) + noise()
    other = 4.0 + noise()  # a second roll state, 20% lower
    r = WS.assess(plain, warm, ref, 500, w, tail)
    assert r["same_state_plain"] and r["same_state_warm"]
    assert r["steps_warm"] < r["steps_plain"]
    assert r["steps_warm_1pct"] is not None
    r2 = WS.assess(plain, other, ref, 500, w, tail)
    assert not r2["same_state_warm"] and r2["steps_warm"] is None
    assert abs(r2["nu_rel_err_warm"] - 0.2) < 0.01
    s = WS.summarize([dict(r, ra=1e5, pr=1.0), dict(r2, ra=1e6, pr=2.0)], n * 500, 0)
    assert s["cavities"] == 2 and s["same_state_warm"] == 1 and s["settled_warm"] == 1
    # the never-settled warm run counts as the horizon
    assert s["median_steps_warm"] == 0.5 * (r["steps_warm"] + n * 500)


def test_median_ci_brackets_the_median():
    rng = np.random.default_rng(0)
    v = rng.standard_normal(16) + 3.0
    m, lo, hi = WS.median_ci(v, np.random.default_rng(1))
    assert lo <= m <= hi and m == np.median(v)
    assert WS.median_ci([2.0] * 8, np.random.default_rng(1)) == (2.0, 2.0, 2.0)
    assert WS.median_ci([], np.random.default_rng(1)) == (None, None, None)
