"""Learned warm start for Rayleigh-Benard cavities.

A U-Net (paper_2211_03160_amd.nn, BF16 MFMA kernels) maps the conduction
state of a cavity and its parameters (log Ra, Pr, aspect ratio) to a
developed convective state (T, u_x, u_y).  The lattice Boltzmann run then
starts from that state (lbm_batch_init_fields) instead of from conduction
plus noise.  Training data are snapshots of the developed flow produced by
the solver itself (batched runs); the plain run from the conduction state
is both the fallback and the yardstick.  Every held-out cavity runs three
times: plain, warm, and plain again with another noise seed (the reference,
so that neither assessed run is compared with its own record).  The
evaluation counts the steps each start needs until the windowed mean of the
wall Nusselt number stays inside a band around the reference's long-time
mean (1%, wider for unsteady cells by their measured fluctuation), and the
error of each start's long-time Nu against the reference, each as a median
over the held-out cavities with a 95% bootstrap interval.

Grids: the network sees every second node of the cavity (H = 2 Hc - 1 nodes
become Hc), zero-padded to a multiple of 2^(levels-1); predictions are
interpolated back to the full grid.  Large-scale rolls come in two mirror
images; snapshots are mirrored to a clockwise mean circulation so the
network learns one of them.

Usage: python -m paper_2211_03160_amd.warmstart [--quick] [--out PATH] [--profile-train STEPS]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lbm, nn
from . import workloads as W

U_FF = 0.1
CIN, COUT = 16, 16
LOGRA_MID, LOGRA_HALF = 6.5, 1.5
PR_MID, PR_HALF = 3.85, 3.15


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cavity_cfgs(count, H, ra_range, pr_range, seed, aspect=1, storage="fp32"):
    rng = np.random.default_rng(seed)
    cfgs = []
    for _ in range(count):
        ra = float(10.0 ** rng.uniform(math.log10(ra_range[0]), math.log10(ra_range[1])))
        pr = float(rng.uniform(*pr_range))
        cfgs.append(W.rayleigh_benard(2, ((H - 1) * aspect + 1, H), ra=ra, pr=pr, u_ff=U_FF,
                                      storage=storage))
    return cfgs


def coarse_shape(cfg, levels):
    nx, ny = cfg["n"][0], cfg["n"][1]
    cx, cy = (nx + 1) // 2, (ny + 1) // 2
    q = 2 ** (levels - 1)
    return cy, cx, -(-cy // q) * q, -(-cx // q) * q


def conduction(cfg):
    ny = cfg["n"][1]
    y = (np.arange(ny) + 0.5) / ny
    return np.repeat((1.0 - y)[:, None], cfg["n"][0], axis=1)


def features(cfg, levels):
    """Network input [Hp, Wp, CIN]: conduction T - 1/2, normalised log Ra,
    Pr and aspect ratio, and the inside mask, on the coarse grid."""
    cy, cx, hp, wp = coarse_shape(cfg, levels)
    x = np.zeros((hp, wp, CIN), np.float32)
    x[:cy, :cx, 0] = conduction(cfg)[::2, ::2] - 0.5
    x[:cy, :cx, 1] = (math.log10(cfg["ra"]) - LOGRA_MID) / LOGRA_HALF
    x[:cy, :cx, 2] = (cfg["pr"] - PR_MID) / PR_HALF
    x[:cy, :cx, 3] = (cfg["n"][0] - 1) / (cfg["n"][1] - 1) - 1.0
    x[:cy, :cx, 4] = 1.0
    return x


def canonical(u, T):
    """Mirror in x if the mean circulation is counter-clockwise."""
    ux, uy = u[0], u[1]
    circ = float((np.gradient(uy, axis=1) - np.gradient(ux, axis=0)).mean())
    if circ > 0:
        return np.stack([-ux[:, ::-1], uy[:, ::-1]]), T[:, ::-1]
    return u, T


def target(cfg, u, T, levels):
    """Training target [Hp, Wp, 3] (T - T_cond, u_x / U, u_y / U) and mask."""
    cy, cx, hp, wp = coarse_shape(cfg, levels)
    u, T = canonical(u, T)
    y = np.zeros((hp, wp, 3), np.float32)
    m = np.zeros((hp, wp, 3), np.float32)
    y[:cy, :cx, 0] = (T - conduction(cfg))[::2, ::2]
    y[:cy, :cx, 1] = u[0][::2, ::2] / U_FF
    y[:cy, :cx, 2] = u[1][::2, ::2] / U_FF
    m[:cy, :cx, :] = 1.0
    return y, m


def to_full(cfg, pred):
    """Coarse prediction [Hp, Wp, 3] -> full-grid (u [2][ny][nx], T)."""
    nx, ny = cfg["n"][0], cfg["n"][1]
    cy, cx = (ny + 1) // 2, (nx + 1) // 2
    p = pred[:cy, :cx, :].astype(np.float64)
    full = np.zeros((ny, nx, 3))
    full[::2, ::2] = p
    full[1::2, ::2] = 0.5 * (p[:-1] + p[1:])
    full[:, 1::2] = 0.5 * (full[:, :-1:2] + full[:, 2::2])
    T = conduction(cfg) + full[..., 0]
    u = np.stack([full[..., 1], full[..., 2]]) * U_FF
    return u, T


def generate(cfgs, seeds, steps, snap_from, snap_every, levels, graph_steps=100):
    """Run the cavities together and collect developed snapshots."""
    b = lbm.Batch(cfgs)
    b.init(seeds, [W.NOISE] * len(cfgs))
    best, _ = b.tune(steps=2)
    b.set_config(best["block"], best["grid_per_cu"], graph_steps)
    X = np.stack([features(c, levels) for c in cfgs])
    xs, ys, ms = [], [], []
    t0 = time.time()
    while b.t < steps:
        nxt = min(steps, snap_from if b.t < snap_from else b.t + snap_every)
        b.step(nxt - b.t)
        if b.t >= snap_from:
            flags = b.unstable()
            for k, c in enumerate(cfgs):
                if flags[k]:
                    continue
                _, u, T = b.cavity(k).fields()
                y, m = target(c, u, T, levels)
                xs.append(X[k])
                ys.append(y)
                ms.append(m)
            log(f"  t = {b.t}: {len(ys)} snapshots ({time.time() - t0:.1f} s)")
    return np.stack(xs), np.stack(ys), np.stack(ms), int(b.unstable().sum())


def train(X, Y, M, chans, epochs, batch, lr, seed, log_every=1):
    import torch
    net = nn.UNet(cin=CIN, cout=COUT, chans=chans, seed=seed)
    Xd = nn.to_bf16(torch.from_numpy(X).cuda())
    Yd = torch.from_numpy(Y).cuda()
    Md = torch.from_numpy(M).cuda()
    rng = np.random.default_rng(seed)
    hist = []
    S = X.shape[0]
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(S)).cuda()
        tot = 0.0
        nb = 0
        rate = lr if ep < int(0.7 * epochs) else lr * 0.3
        for i in range(0, S - batch + 1, batch):
            idx = order[i:i + batch]
            y, tape = net.forward(Xd[idx].contiguous())
            loss, dy = nn.mse(y, Yd[idx].contiguous(), Md[idx].contiguous())
            net.backward(tape, dy)
            net.adam(lr=rate)
            tot += float(loss.item())
            nb += 1
        hist.append(tot / max(nb, 1))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            log(f"  epoch {ep}: loss {hist[-1]:.5f}")
    return net, hist


def predict(net, cfgs, levels):
    import torch
    X = np.stack([features(c, levels) for c in cfgs])
    y, _ = net.forward(nn.to_bf16(torch.from_numpy(X).cuda()))
    out = nn.to_f32(y).cpu().numpy()[..., :3]
    return [to_full(c, out[k]) for k, c in enumerate(cfgs)]


def window_means(h, window):
    return np.convolve(np.asarray(h, float), np.ones(window) / window, mode="valid")


def steps_to_steady(hist, every, ref, window, tol=0.01):
    """First step after which the windowed mean of Nu stays within tol of
    ref; None if it never settles."""
    h = np.asarray(hist)
    if len(h) < window:
        return None
    ok = np.abs(window_means(h, window) - ref) <= tol * abs(ref)
    bad = np.nonzero(~ok)[0]
    first = 0 if len(bad) == 0 else bad[-1] + 1
    if first >= len(ok):
        return None
    return int((first + window) * every)


def steps_to_reach(hist, every, ref, window, tol):
    """First step at which the windowed mean of Nu is within tol of ref;
    None if it never gets there."""
    h = np.asarray(hist)
    if len(h) < window:
        return None
    ok = np.nonzero(np.abs(window_means(h, window) - ref) <= tol * abs(ref))[0]
    return None if len(ok) == 0 else int((ok[0] + window) * every)


def tail_stats(h, window, tail):
    """Long-time mean of a Nu record (its last `tail` entries), the relative
    standard error of that mean (spread of four block means) and the
    relative spread of the window means inside the tail."""
    t = np.asarray(h[-tail:], float)
    mean = float(t.mean())
    sem = float(np.std([b.mean() for b in np.array_split(t, 4)]) / 2.0) / abs(mean)
    spread = float(np.std(window_means(t, window))) / abs(mean) if len(t) >= window else 0.0
    return mean, sem, spread


def assess(plain, warm, ref_run, every, window, tail):
    """Compare a plain and a warm run of one cavity with a third, independent
    plain run (another noise seed), the reference.  The reference's
    long-time mean is the target Nu.  The band around that target is 1%, or,
    for unsteady cells whose window means wander by more than that in the
    developed state, three times the combined spread of the reference's
    window means and the error of its mean, so that the developed reference
    itself seldom leaves it.  A run reaches the developed state when its
    window mean first enters the band, and has settled once it stays inside
    (for a chaotic cell the last exit is itself a random event).  A
    run settled in the reference's state if its own long-time mean agrees
    within 1% or three combined standard errors (2D cells are multistable:
    two plain runs with different noise can end in different roll states)."""
    ref, sem_r, spread_r = tail_stats(ref_run, window, tail)
    band = max(0.01, 3.0 * math.hypot(spread_r, sem_r))
    r = {"nu_ref": ref, "nu_ref_rel_sem": sem_r, "band": band}
    for name, h in (("plain", plain), ("warm", warm)):
        mean, sem, _ = tail_stats(h, window, tail)
        err = abs(mean - ref) / abs(ref)
        r[f"nu_{name}"] = mean
        r[f"nu_rel_err_{name}"] = err
        r[f"same_state_{name}"] = bool(err <= max(0.01, 3.0 * math.hypot(sem_r, sem)))
        r[f"steps_{name}"] = steps_to_steady(h, every, ref, window, tol=band)
        r[f"steps_{name}_reach"] = steps_to_reach(h, every, ref, window, tol=band)
        r[f"steps_{name}_1pct"] = steps_to_steady(h, every, ref, window, tol=0.01)
    return r


def evaluate(net, cfgs, seeds, ref_seeds, steps, every, levels, window):
    """Three starts of every held-out cavity in one batch: plain (conduction
    + noise), warm (the network's prediction) and the reference (conduction
    + noise with another seed); Nu = (Nu_hot + Nu_cold)/2 every `every`
    steps."""
    n = len(cfgs)
    b = lbm.Batch(cfgs * 3)
    b.init(list(seeds) + list(seeds) + list(ref_seeds), [W.NOISE] * (3 * n))
    for k, (u, T) in enumerate(predict(net, cfgs, levels)):
        b.init_fields(n + k, None, u, T)
    b.set_config(256, 0, every if every % 2 == 0 else 0)
    hist = []
    t0 = time.time()
    while b.t < steps:
        b.step(every)
        hot, cold = b.nusselt()
        hist.append(0.5 * (hot + cold))
        if len(hist) % max(1, (steps // every) // 10) == 0:
            log(f"  eval t = {b.t} ({time.time() - t0:.1f} s)")
    hist = np.array(hist)  # [records][3n]
    tail = max(window, (3 * len(hist)) // 10)
    res = []
    for k in range(n):
        r = {"ra": cfgs[k]["ra"], "pr": cfgs[k]["pr"]}
        r.update(assess(hist[:, k], hist[:, n + k], hist[:, 2 * n + k], every, window, tail))
        res.append(r)
    flags = b.unstable()
    return res, int(flags.sum()), hist


def run(H=257, n_train=128, n_eval=16, steps=200000, snap_from=72000, snap_every=8000,
        chans=(32, 64, 128, 256), epochs=24, batch=16, lr=1e-3, ra_range=(1e5, 1e8),
        pr_range=(0.7, 7.0), eval_steps=600000, eval_every=500, window=100, seed=2024):
    """Defaults: the 257^2 configuration (window = 50000 steps, about 20
    free-fall times H/U)."""
    levels = len(chans)
    out = {"H": H, "chans": list(chans), "ra_range": list(ra_range), "pr_range": list(pr_range)}
    t0 = time.time()
    train_cfgs = cavity_cfgs(n_train, H, ra_range, pr_range, seed)
    X, Y, M = [], [], []
    flagged = 0
    for i in range(0, n_train, 64):
        log(f"data: cavities {i}..{min(n_train, i + 64) - 1}")
        x, y, m, f = generate(train_cfgs[i:i + 64], [seed + k for k in range(i, min(n_train, i + 64))],
                              steps, snap_from, snap_every, levels)
        X.append(x)
        Y.append(y)
        M.append(m)
        flagged += f
    X, Y, M = np.concatenate(X), np.concatenate(Y), np.concatenate(M)
    out["snapshots"] = int(X.shape[0])
    out["unstable_training_cavities"] = flagged
    out["datagen_s"] = time.time() - t0
    t1 = time.time()
    net, hist = train(X, Y, M, chans, epochs, batch, lr, seed)
    out["train_s"] = time.time() - t1
    out["loss_history"] = [round(v, 6) for v in hist]
    t2 = time.time()
    eval_cfgs = cavity_cfgs(n_eval, H, ra_range, pr_range, seed + 99991)
    res, bad, hist = evaluate(net, eval_cfgs, [seed + 5000 + k for k in range(n_eval)],
                        [seed + 7000 + k for k in range(n_eval)], eval_steps, eval_every, levels,
                        window)
    out["eval_s"] = time.time() - t2
    out["unstable_eval_runs"] = bad
    out["eval"] = res
    # Nu every eval_every steps: columns plain, warm, reference per cavity
    out["nu_history"] = [[float(f"{v:.6g}") for v in row] for row in hist.T]
    out["window_steps"] = window * eval_every
    out["horizon_steps"] = eval_steps
    out.update(summarize(res, eval_steps, seed))
    return out


def median_ci(values, rng, draws=4000, level=0.95):
    """Median and a bootstrap confidence interval over the cavities
    (percentile method, the cavities resampled with replacement)."""
    v = np.asarray(values, float)
    if len(v) == 0:
        return None, None, None
    meds = np.median(v[rng.integers(0, len(v), (draws, len(v)))], axis=1)
    lo, hi = np.quantile(meds, [(1 - level) / 2, (1 + level) / 2])
    return float(np.median(v)), float(lo), float(hi)


def summarize(res, horizon, seed):
    """Medians over the held-out cavities, each with a 95% bootstrap
    interval: steps saved by the warm start (plain minus warm steps until
    the run settles in the band, and until it first reaches it; a run that
    never does counts as the horizon) and the Nu error
    of either start against the reference; plus how many runs settled (band
    and strict 1%) and how many ended in the reference's state."""
    rng = np.random.default_rng(seed)
    cap = lambda s: horizon if s is None else s
    out = {"cavities": len(res)}
    for kind, suffix in (("", ""), ("reach", "_reach")):
        saved = [cap(r["steps_plain" + suffix]) - cap(r["steps_warm" + suffix]) for r in res]
        med, lo, hi = median_ci(saved, rng)
        tag = "_" + kind if kind else ""
        out[f"steps_saved{tag}_median"] = med
        out[f"steps_saved{tag}_ci95"] = [lo, hi]
        out[f"warm_faster{tag}_fraction"] = float(np.mean([s > 0 for s in saved])) if saved else None
    for name in ("plain", "warm"):
        out[f"median_steps_{name}"] = float(np.median([cap(r[f"steps_{name}"]) for r in res]))
        out[f"median_steps_{name}_reach"] = float(np.median([cap(r[f"steps_{name}_reach"]) for r in res]))
        out[f"settled_{name}"] = sum(r[f"steps_{name}"] is not None for r in res)
        out[f"settled_{name}_1pct"] = sum(r[f"steps_{name}_1pct"] is not None for r in res)
        m, a, z = median_ci([r[f"nu_rel_err_{name}"] for r in res], rng)
        out[f"nu_rel_err_{name}_median"] = m
        out[f"nu_rel_err_{name}_ci95"] = [a, z]
        out[f"same_state_{name}"] = int(sum(r[f"same_state_{name}"] for r in res))
    out["steps_saved_fraction"] = (1.0 - out["median_steps_warm"] / out["median_steps_plain"]
                                   if out["median_steps_plain"] else None)
    return out


def profile_train(steps=40, H=257, chans=(32, 64, 128, 256), batch=16, seed=7):
    """Time `steps` training steps of the network at the shape of the 257^2
    configuration (random BF16 inputs and targets), with HIP events, and
    count the algorithmic FLOPs of its 3x3 convolutions (forward, data
    gradient except for the first layer, weight gradient; 2 per
    multiply-add).  Returns ms per step and TFLOP/s."""
    import torch
    levels = len(chans)
    cfg = W.rayleigh_benard(2, (H, H), ra=1e6, pr=1.0)
    _, _, hp, wp = coarse_shape(cfg, levels)
    rng = np.random.default_rng(seed)
    X = nn.to_bf16(torch.from_numpy(rng.standard_normal((batch, hp, wp, CIN)).astype(np.float32)).cuda())
    Y = torch.from_numpy(rng.standard_normal((batch, hp, wp, 3)).astype(np.float32)).cuda()
    M = torch.ones_like(Y)
    net = nn.UNet(cin=CIN, cout=COUT, chans=chans, seed=seed)

    def one():
        y, tape = net.forward(X)
        loss, dy = nn.mse(y, Y, M)
        net.backward(tape, dy)
        net.adam(lr=1e-4)

    for _ in range(3):
        one()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        one()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # layer resolutions: two per encoder level, two per decoder level, the
    # output layer at full resolution
    res = [lvl for lvl in range(levels) for _ in range(2)] + \
          [lvl for lvl in range(levels - 2, -1, -1) for _ in range(2)] + [0]
    flops = 0.0
    for k, (lay, lvl) in enumerate(zip(net.layers, res)):
        mac = batch * (hp >> lvl) * (wp >> lvl) * 9 * lay["ci"] * lay["co"]
        flops += 2 * mac * (3 if k > 0 else 2)
    return {"ms_per_step": ms, "gflop_per_step": flops / 1e9, "tflops": flops / (ms * 1e-3) / 1e12,
            "batch": batch, "grid": [hp, wp], "chans": list(chans)}


QUICK = dict(H=65, n_train=64, n_eval=8, steps=40000, snap_from=16000, snap_every=2000,
             chans=(32, 64), epochs=20, batch=16, ra_range=(1e4, 1e5), eval_steps=80000,
             eval_every=200, window=16)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--profile-train", type=int, default=0, metavar="STEPS",
                    help="only time STEPS training steps of the network at the 257^2 shape")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if a.profile_train:
        print(json.dumps(profile_train(a.profile_train)), flush=True)
        return
    if a.quick:
        out = run(**QUICK)
    else:
        out = run()
    print(json.dumps({k: v for k, v in out.items() if k != "nu_history"}), flush=True)
    if a.out:
        open(a.out, "w").write(json.dumps(out))


if __name__ == "__main__":
    main()
