"""Benchmark of the fused thermal LBM step on one MI355X.

Headline: GLUPS of the FP32 fused step on the 8193 x 8193 D2Q9 + D2Q5
Rayleigh-Benard cell (Ra 1e8, Pr 0.71), W untimed warm-up steps then K timed
steps, inputs resident in HBM, in the library's default launch mode (four
steps per launch for FP32 in 2D).  GLUPS = nodes x steps / time / 1e9 (the
MLUPS definition of Section 2.3, Eq. 10, in units of 1e9).  The same JSON
line carries the roofline of the dominant kernel against HBM (the
algorithmic bytes of one launch, one read and one write of every population
of every node, over the launch's average duration from HIP events, against
the 8 TB/s peak and against the copy ceiling this GPU reaches with the
library's probe kernels, measured first), that launch's vector-ALU figures,
the Nu error of the run against an FP64 GPU run of the same steps (which
runs before the headline, with its own roofline), the other launch modes and
storage forms, the 385^3 D3Q19 + D3Q7 cell, and the FP64 CPU oracle timed
on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
       [--only NAME] [--no-cpu] [--copy-probe] [--oracle-timing]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "GLUPS & %HBM peak, FP32 vs FP16-store, 8193² D2Q9+D2Q5 / 385³ D3Q19+D3Q7"
# the kernels and their launch configuration (strip segments, steps per
# launch): HBM traffic counters are valid for this hash only
KERNEL_SOURCES = ["paper_2211_03160_amd/csrc/kernels.hpp", "paper_2211_03160_amd/csrc/lattice.hpp",
                  "paper_2211_03160_amd/csrc/stream3d.hpp", "paper_2211_03160_amd/csrc/lbm_api.hip"]
TRAFFIC_FILES = {5: os.path.join(ROOT, "profiles", "stream5_d2q9_fp32_8193_counters.txt"),
                 1: os.path.join(ROOT, "profiles", "step_d2q9_fp32_8193_counters.txt")}
TRAFFIC_FILES_3D = {2: os.path.join(ROOT, "profiles", "stream3d_d3q19_fp32_385_counters.txt"),
                    1: os.path.join(ROOT, "profiles", "step_d3q19_fp32_385_counters.txt")}
# FP32 operations per 2D lattice update in the kernels' formulation (adds,
# subtracts, multiplies and the reciprocal 1 each, fused multiply-adds 2):
# the written-out D2Q9 + D2Q5 collision with its shared terms, its moments
# and the reference-state temperature, as in the one-step kernel, which
# computes every node once (loop-invariant products of rates and constants
# not counted)
FLOPS_PER_UPDATE_2D = 148
# non-packed FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz.  The build disables packed FP32, whose dual-rate issue gives the
# published 157.3; both are reported.
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(steps_per_launch, files=TRAFFIC_FILES):
    """HBM bytes per launch of an FP32 step kernel (several steps per launch
    or one) from the committed rocprofv3 counter runs, if they were taken on
    the current kernel source."""
    path = files.get(steps_per_launch)
    if path is None or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def read_valu_instructions(steps_per_launch):
    """VALU wave instructions per launch of the multi-step FP32 kernel from
    the committed rocprofv3 run, if taken on the current kernel source at
    this many steps per launch."""
    path = os.path.join(ROOT, "profiles", "valu_d2q9_fp32_8193.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_hash() or kv.get("steps_per_launch") != str(steps_per_launch):
        return None
    try:
        return float(kv["stream_valu_instructions_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(cav, steps):
    """Average wall time per step over `steps` launches, measured with HIP
    events recorded on the stream the kernels are launched on."""
    import torch
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(cav.stream)
    cav.step(steps)
    e1.record(cav.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms


def run_case(cfg, warmup, steps, seed, noise, want_nu=True, steps_per_launch=None):
    import torch
    from paper_2211_03160_amd import lbm
    cav = lbm.Cavity(cfg)
    if steps_per_launch:
        cav.steps_per_launch = steps_per_launch
    cav.init(seed, noise)
    cav.step(warmup)
    ms = timed_steps(cav, steps)
    out = {"ms_per_step": ms, "glups": cav.N / (ms * 1e-3) / 1e9,
           "steps_per_launch": cav.steps_per_launch,
           "bytes_per_update": cav.bytes_per_update()}
    out["hbm_gbs_algorithmic"] = out["glups"] * out["bytes_per_update"]
    if want_nu:
        out["nu"] = cav.nusselt()
        d = cav.diagnostics()
        out["re"] = d["re"]
        out["umax"] = d["umax"]
    del cav
    torch.cuda.empty_cache()
    return out


def batched_sweep(K, warmup, noise):
    """Config 3: 64 ragged cavities advanced together, the launch shape and
    steps per launch chosen by the library's autotuner (one-step kernel
    shapes, and the streaming kernel at 2-5 steps per launch x segment rows
    x wavefronts per block), replayed from a hipGraph; then the same batch
    with one step per launch (the tuned one-step shape).  Both against the
    same 64 cavities run one after another in the single-cavity default
    mode and with one step per launch."""
    import torch
    from paper_2211_03160_amd import lbm, workloads as W
    cfgs, seeds = W.batched_sweep()
    nodes = sum(c["n"][0] * c["n"][1] for c in cfgs)
    graph_steps = 60  # a multiple of every steps-per-launch count

    def timed(b):
        b.step(warmup)  # captures the graph
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(K)
        e1.record(b.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    b = lbm.Batch(cfgs)
    b.init(seeds, [noise] * len(cfgs))
    best, cand_ms = b.tune(steps=3)
    spl_tuned = b.steps_per_launch
    b.set_config(**{**best, "graph_steps": graph_steps})
    ms_tuned = timed(b)
    flagged = int(b.unstable().sum())
    del b
    b = lbm.Batch(cfgs)
    b.steps_per_launch = 1
    b.init(seeds, [noise] * len(cfgs))
    b.set_config(**{**best, "graph_steps": graph_steps})
    ms_one = timed(b)
    del b
    torch.cuda.empty_cache()
    ms_seq = {"default": 0.0, "one": 0.0}
    for c, sd in zip(cfgs, seeds):
        for mode in ms_seq:
            cav = lbm.Cavity(c)
            if mode == "one":
                cav.steps_per_launch = 1
            cav.init(sd, noise)
            cav.step(8)
            ms_seq[mode] += timed_steps(cav, K) * K
            del cav
    torch.cuda.empty_cache()
    g = lambda ms: nodes * K / (ms * 1e-3) / 1e9
    return {"cavities": len(cfgs), "nodes": nodes, "steps": K, "steps_per_launch": spl_tuned,
            "glups": g(ms_tuned),
            "glups_sequential": g(ms_seq["default"]),
            "speedup_vs_sequential": ms_seq["default"] / ms_tuned,
            "glups_one_step_per_launch": g(ms_one),
            "glups_sequential_one_step_per_launch": g(ms_seq["one"]),
            "speedup_vs_sequential_one_step_per_launch": ms_seq["one"] / ms_one,
            "ms_per_step": ms_tuned / K, "config": {**best, "graph_steps": graph_steps},
            "tuner_candidates": len(cand_ms),
            "tuner_best_ms_per_step": round(min(cand_ms), 4),
            "tuner_ms_per_step": [round(m, 4) for m in cand_ms],
            "unstable_cavities": flagged}


def rel(a, b):
    return abs(a - b) / abs(b) if b else float("nan")


def nu_err(nu, ref):
    return max(rel(nu[0], ref[0]), rel(nu[1], ref[1]))


def copy_ceiling(nbytes=4 << 30, reps=5):
    """The HBM ceiling of one-pass streaming on this GPU: the library's
    probe kernels (copy, read-only, write-only; 1, 2, 4 or 8 16-byte vectors
    per thread, plain or non-temporal) over `nbytes`, each shape timed with
    HIP events on the stream it is launched on over `reps` launches after
    one untimed launch.  Returns the best GB/s of each kind and its shape;
    a copy counts its bytes twice (read and write)."""
    import torch
    from paper_2211_03160_amd import lbm
    s = torch.cuda.current_stream()
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for kind in ("copy", "read", "write"):
        best = None
        for k in (1, 2, 4, 8):
            for nt in (False, True):
                a = None if kind == "write" else src
                lbm.probe_bandwidth(kind, a, dst, nbytes, k, nt, s)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                for _ in range(reps):
                    lbm.probe_bandwidth(kind, a, dst, nbytes, k, nt, s)
                e1.record(s)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                gbs = nbytes * (2 if kind == "copy" else 1) / (ms * 1e-3) / 1e9
                if best is None or gbs > best["gbs"]:
                    best = {"gbs": round(gbs, 1), "per_thread": k, "nontemporal": nt, "ms": round(ms, 4)}
        out[kind] = best
    del src, dst
    torch.cuda.empty_cache()
    out["bytes"] = nbytes
    return out


def hbm_roofline(r, nodes, kernel, ceiling_gbs=None):
    """Roofline of a step kernel against HBM: the algorithmic bytes of one
    launch (one read and one write of every population of every node)
    divided by the launch's average duration from HIP events."""
    spl = r["steps_per_launch"]
    launch_s = r["ms_per_step"] * spl * 1e-3
    per_node = r["bytes_per_update"] * spl
    gbs = nodes * per_node / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(gbs / PEAK_HBM_GBS, 4), "kernel": kernel, "steps_per_launch": spl,
           "launch_ms": round(launch_s * 1e3, 4), "bytes_per_node_per_launch": per_node,
           "bytes_per_lattice_update": r["bytes_per_update"]}
    if ceiling_gbs:
        out["copy_ceiling_gbs"] = ceiling_gbs
        out["frac_of_copy_ceiling"] = round(gbs / ceiling_gbs, 4)
    return out


def cpu_baseline(cfg2d, budget_s=12.0):
    """The FP64 oracle, as it stands, on a strip of the headline cell: the
    full 8193-node rows, 65 rows high, same walls and parameters; steps run
    until ~budget_s of wall time."""
    from oracle.lbmref import Oracle, threads
    cfg = dict(cfg2d)
    cfg["n"] = (cfg2d["n"][0], 65, 1)
    # keep the transport coefficients of the full cell (the oracle's own
    # parameter mapping)
    from oracle.lbmref import derive
    d = derive(cfg2d)
    cfg.update(nu=d["nu"], alpha=d["alpha"], gbeta=d["gbeta"])
    o = Oracle(cfg)
    o.init(1234, 1e-3)
    o.step(1)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and steps < 2000:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    nodes = cfg["n"][0] * cfg["n"][1]
    return {"value": nodes * steps / dt / 1e9, "unit": "GLUPS", "cores": threads(),
            "kind": "oracle",
            "sample": f"FP64 oracle on a {cfg['n'][0]}x{cfg['n'][1]} strip of the 8193^2 cell "
                      f"(same rows, walls and lattice parameters), {steps} steps in {dt:.1f} s"}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_timing():
    """The FP64 oracle timed in full: C0 (129^2, all 5000 steps), the C1 and
    C2 shapes (3 steps after 1 warm-up), each on all host threads and, for
    C0 and a C1 strip, on one thread.  Host memory: ~15 GB (C1) and ~24 GB
    (C2) of FP64 populations."""
    from oracle.lbmref import Oracle, set_threads, threads
    from paper_2211_03160_amd import workloads as W
    all_threads = threads()
    out = {"cpu": cpu_model(), "threads": all_threads, "cases": []}

    def timed(name, cfg, warm, steps, nthreads):
        set_threads(nthreads)
        o = Oracle(cfg)
        o.init(W.SEED, W.NOISE)
        if warm:
            o.step(warm)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        n = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
        r = {"case": name, "nodes": n, "steps": steps, "threads": nthreads, "seconds": round(dt, 3),
             "mlups": round(n * steps / dt / 1e6, 3)}
        log("oracle", json.dumps(r))
        out["cases"].append(r)
        del o

    c0 = W.C0["cfg"]
    timed("C0 129^2 D2Q9+D2Q5, 5000 steps", c0, 0, W.C0["steps"], all_threads)
    timed("C0 129^2, 200 steps", c0, 0, 200, 1)
    strip = dict(W.C1["cfg"])
    strip["n"] = (8193, 65, 1)
    from oracle.lbmref import derive
    d = derive(W.C1["cfg"])
    strip.update(nu=d["nu"], alpha=d["alpha"], gbeta=d["gbeta"], storage="fp64")
    timed("C1 strip 8193x65, 3 steps", strip, 1, 3, 1)
    timed("C1 8193^2 D2Q9+D2Q5, 3 steps", W.with_storage(W.C1["cfg"], "fp64"), 1, 3, all_threads)
    timed("C2 385^3 D3Q19+D3Q7, 3 steps", W.with_storage(W.C2["cfg"], "fp64"), 1, 3, all_threads)
    set_threads(0)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--quick", action="store_true", help="headline only, no variants")
    ap.add_argument("--only", default=None, help="comma-separated case names: run those and exit")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three 1 GiB probe copies (for counter calibration)")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="time the FP64 oracle on C0 in full and the C1/C2 shapes, then exit")
    args = ap.parse_args()
    if args.oracle_timing:
        print(json.dumps(oracle_timing()), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the fused step has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2211_03160_amd import lbm, workloads as W
    lbm.lib()  # fails loudly if the HIP library is not built
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    c1 = W.C1
    cfg32 = c1["cfg"]
    seed, noise = c1["seed"], c1["noise"]
    K, Wm = args.steps, args.warmup

    cases = {
        "rb2d_8193_fp32": (cfg32, Wm, K),
        "rb2d_8193_fp32_1": (cfg32, Wm, K),
        "rb2d_8193_fp32_2": (cfg32, Wm, K),
        "rb2d_8193_fp64": (W.with_storage(cfg32, "fp64"), Wm, K),
        "rb2d_8193_fp16": (W.with_storage(cfg32, "fp16"), Wm, K),
        "rb2d_8193_bf16": (W.with_storage(cfg32, "bf16"), Wm, K),
        "rb2d_8193_mixed": (W.with_storage(cfg32, "mixed"), Wm, K),
        "rb3d_385_fp32": (W.C2["cfg"], 5, W.C2["steps"]),
        "rb3d_385_fp32_1": (W.C2["cfg"], 5, W.C2["steps"]),
        "rb3d_385_fp64": (W.with_storage(W.C2["cfg"], "fp64"), 5, W.C2["steps"]),
        "rb3d_385_fp16": (W.with_storage(W.C2["cfg"], "fp16"), 5, W.C2["steps"]),
        "rb3d_385_bf16": (W.with_storage(W.C2["cfg"], "bf16"), 5, W.C2["steps"]),
        "rb3d_385_mixed": (W.with_storage(W.C2["cfg"], "mixed"), 5, W.C2["steps"]),
    }

    if args.copy_probe:
        # a plain copy of known size for counter calibration: 1 GiB read and
        # 1 GiB written by the library's probe kernel (4 vectors per thread)
        x = torch.ones(1 << 30, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            lbm.probe_bandwidth("copy", x, y, 1 << 30, 4, False, torch.cuda.current_stream())
        torch.cuda.synchronize()
        del x, y
        log("copy probe: 3 x 1 GiB probe copies done")

    if args.only:
        for name in args.only.split(","):
            cfg, w, k = cases[name]
            spl = {"_1": 1, "_2": 2}.get(name[-2:])
            r = run_case(cfg, min(w, args.warmup), min(k, args.steps), seed, noise, want_nu=False,
                         steps_per_launch=spl)
            log(name, json.dumps(r))
        return

    # The copy ceiling and the FP64 reference run first, so the headline is
    # not the process's first GPU work.
    ceil = copy_ceiling()
    log("copy ceiling", json.dumps(ceil))
    ref64 = run_case(cases["rb2d_8193_fp64"][0], Wm, K, seed, noise)
    log("fp64", json.dumps(ref64))
    log(f"headline: 8193^2 D2Q9+D2Q5 FP32, warmup {Wm}, timed {K}")
    head = run_case(cfg32, Wm, K, seed, noise)
    log("fp32", json.dumps(head))

    # The dominant kernel: several steps per launch (K and W are multiples
    # of the steps per launch, so every timed launch is one).  Its
    # algorithmic HBM traffic is one read and one write of all populations
    # per node and launch: 112 B per node, 22.4 B per lattice update at five
    # steps.  The same launch's vector-ALU figures stand beside it.
    N = cfg32["n"][0] * cfg32["n"][1]
    spl = head["steps_per_launch"]
    kname = f"lbm::stream_kernel<StF32, 4, true, {spl}, 0>" if spl > 1 else "lbm::step_kernel<2, StF32>"
    roofline = hbm_roofline(head, N, kname, ceil["copy"]["gbs"])
    roofline["traffic"] = read_traffic(spl)
    launch_s = roofline["launch_ms"] * 1e-3
    if spl > 1:
        tflops = head["glups"] * FLOPS_PER_UPDATE_2D / 1e3
        # VALU issue slots the launch uses: instructions x 4 cycles per
        # SIMD over 1024 SIMDs at 2.4 GHz, during the HIP-event launch time
        insts = read_valu_instructions(spl)
        roofline["valu"] = {
            "flops_per_lattice_update": FLOPS_PER_UPDATE_2D, "achieved_tflops": round(tflops, 2),
            "peak_tflops": PEAK_FP32_PACKED_TFLOPS, "frac": round(tflops / PEAK_FP32_PACKED_TFLOPS, 4),
            "peak_nonpacked_tflops": PEAK_FP32_TFLOPS, "frac_nonpacked": round(tflops / PEAK_FP32_TFLOPS, 4),
            "issue_frac": round(insts * 4 / 1024 / 2.4e9 / launch_s, 4) if insts else None}
    ref64["roofline"] = hbm_roofline(ref64, N, f"lbm::stream_kernel<StF64, 4, false, {ref64['steps_per_launch']}, 1>",
                                     ceil["copy"]["gbs"])

    variants = {"rb2d_8193_fp64": {**ref64}}
    for k, name in ((1, "one"), (2, "two")):
        r = run_case(cfg32, Wm, K, seed, noise, want_nu=False, steps_per_launch=k)
        r["hbm_frac"] = r["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
        variants[f"rb2d_8193_fp32_{name}_step{'s' if k > 1 else ''}_per_launch"] = r
        log(f"fp32 {name} step(s) per launch", json.dumps(r))
    if not args.quick:
        for name in ("rb2d_8193_fp16", "rb2d_8193_bf16", "rb2d_8193_mixed"):
            cfg, w, k = cases[name]
            r = run_case(cfg, w, k, seed, noise)
            r["nu_rel_err_vs_fp64"] = nu_err(r["nu"], ref64["nu"])
            variants[name] = r
            log(name, json.dumps(r))
        N3 = 385 ** 3
        ref3 = run_case(cases["rb3d_385_fp64"][0], 5, W.C2["steps"], W.C2["seed"], W.C2["noise"])
        ref3["roofline"] = hbm_roofline(ref3, N3, "lbm::step_kernel<3, StF64>", ceil["copy"]["gbs"])
        variants["rb3d_385_fp64"] = ref3
        log("rb3d_385_fp64", json.dumps(ref3))
        for name in ("rb3d_385_fp32", "rb3d_385_fp16", "rb3d_385_bf16", "rb3d_385_mixed"):
            cfg, w, k = cases[name]
            r = run_case(cfg, w, k, W.C2["seed"], W.C2["noise"])
            r["nu_rel_err_vs_fp64"] = nu_err(r["nu"], ref3["nu"])
            r["re_rel_err_vs_fp64"] = rel(r["re"], ref3["re"])
            r["hbm_frac"] = r["hbm_gbs_algorithmic"] / PEAK_HBM_GBS
            st = {"rb3d_385_fp32": "StF32", "rb3d_385_fp16": "StF16", "rb3d_385_bf16": "StBF16",
                  "rb3d_385_mixed": "StMix"}[name]
            k3 = f"lbm::stream3_kernel<{st}>" if r["steps_per_launch"] == 2 else f"lbm::step_kernel<3, {st}>"
            r["roofline"] = hbm_roofline(r, N3, k3, ceil["copy"]["gbs"])
            if name == "rb3d_385_fp32":
                r["roofline"]["traffic"] = read_traffic(r["steps_per_launch"], TRAFFIC_FILES_3D)
            variants[name] = r
            log(name, json.dumps(r))

        bs = batched_sweep(W.C3["steps"], W.C3["warmup"], W.C3["noise"])
        variants["batch64_rb2d_fp32"] = bs
        log("batch64_rb2d_fp32", json.dumps(bs))

        # the paper's own cavity (side-heated, Section 2.3) at its 2D size
        sh = run_case(W.side_heated(2, (8193, 8193), ra=1e8, storage="fp32"), Wm, K, seed, noise)
        variants["sh2d_8193_fp32"] = sh
        log("sh2d_8193_fp32", json.dumps(sh))

        # learned warm start at 257^2: a 4-level, 32-base U-Net trained on
        # about 2000 snapshots of Ra 1e5..1e8 cells, assessed on 16 held-out
        # cavities against independent plain runs (data, training and
        # evaluation all on the GPU, about 80 s)
        from paper_2211_03160_amd import warmstart as WS
        ws = WS.run()
        variants["warmstart_rb2d_257"] = {k: v for k, v in ws.items() if k not in ("eval", "loss_history", "nu_history")}
        log("warmstart_rb2d_257", json.dumps(variants["warmstart_rb2d_257"]))

    cpu = None if args.no_cpu else cpu_baseline(cfg32)
    if cpu:
        log("cpu baseline", json.dumps(cpu))

    for v in variants.values():
        for k in list(v):
            if isinstance(v[k], float):
                v[k] = float(f"{v[k]:.6g}")
    line = {
        "metric": METRIC,
        "value": round(head["glups"], 3),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rb2d_8193x8193_d2q9_d2q5_ra1e8_pr0.71_fp32",
                   "grid": [8193, 8193], "lattice": "D2Q9+D2Q5", "storage": "fp32",
                   "ra": 1e8, "pr": 0.71, "seed": seed, "noise": noise},
        "nu": head["nu"],
        "nu_rel_err_vs_fp64": float(f"{nu_err(head['nu'], ref64['nu']):.3g}"),
        "roofline": roofline,
        "copy_ceiling": ceil,
        "cpu_baseline": cpu,
        "variants": variants,
        "context": {"paper_single_gpu_glups": {"2d_8193": 1.9312, "3d_385": 1.0424},
                    "paper_hardware": "NVIDIA A100 1555 GB/s, FP64, side-heated cavity"},
        "kernel_source_sha256": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
