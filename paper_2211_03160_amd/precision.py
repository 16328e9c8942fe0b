"""Storage precision measured from a developed convective state.

The Nusselt and Reynolds numbers of every storage mode after `steps` steps,
against FP64, all started from one developed state: the state is grown in
FP32 from conduction plus noise (lbm_init) until the Reynolds number has
settled, its moments (rho, u, T) are read back (lbm_fields), and every mode,
FP64 included as the reference, restarts from their equilibria
(lbm_init_fields).  Started from conduction, the large cells are still at
rest after a few hundred steps, so relative Re errors there are ill-
conditioned; from a developed flow they measure what the storage loses.

Usage: python -m paper_2211_03160_amd.precision [--quick] [--out PATH]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import lbm
from . import workloads as W

STORAGES = ("fp64", "fp32", "mixed", "fp16", "bf16")


def develop(cfg: dict, max_steps: int, chunk: int, seed: int, noise: float, settle: float = 0.02,
            log=print):
    """FP32 run from conduction plus noise, in chunks, until the Reynolds
    number changes by less than `settle` (relative) over two consecutive
    chunks (or max_steps).  Returns host (rho, u, T) and the (t, Re, Nu_hot,
    Nu_cold) history."""
    c = lbm.Cavity(W.with_storage(cfg, "fp32"))
    c.init(seed, noise)
    hist = []
    t0 = time.time()
    while c.t < max_steps:
        c.step(chunk)
        d = c.diagnostics()
        nh, nc = c.nusselt()
        hist.append((c.t, d["re"], nh, nc))
        log(f"  develop t = {c.t}: Re {d['re']:.4g}, Nu {nh:.5f} / {nc:.5f} ({time.time() - t0:.0f} s)")
        if len(hist) >= 3:
            r = [h[1] for h in hist[-3:]]
            if r[-1] > 0 and all(abs(r[-1] - x) <= settle * r[-1] for x in r[:-1]):
                break
    fields = c.fields()
    c.close()
    return fields, hist


def compare(cfg: dict, fields, steps: int, storages=STORAGES, log=print) -> dict:
    """Every storage mode restarted from `fields`, `steps` steps each."""
    res = {}
    for st in storages:
        c = lbm.Cavity(W.with_storage(cfg, st))
        c.init_fields(*fields)
        t0 = time.time()
        c.step(steps)
        nh, nc = c.nusselt()
        d = c.diagnostics()
        res[st] = {"nu_hot": nh, "nu_cold": nc, "re": d["re"], "umax": d["umax"]}
        log(f"  {st}: Nu {nh:.7f} / {nc:.7f}, Re {d['re']:.6g} ({time.time() - t0:.1f} s)")
        c.close()
    ref = res["fp64"]
    for st, r in res.items():
        r["nu_rel_err"] = max(abs(r["nu_hot"] - ref["nu_hot"]) / abs(ref["nu_hot"]),
                              abs(r["nu_cold"] - ref["nu_cold"]) / abs(ref["nu_cold"]))
        r["re_rel_err"] = abs(r["re"] - ref["re"]) / abs(ref["re"])
    return res


def run(cfg: dict, max_develop: int, chunk: int, steps: int, seed: int = W.SEED, noise: float = W.NOISE,
        storages=STORAGES, log=print) -> dict:
    fields, hist = develop(cfg, max_develop, chunk, seed, noise, log=log)
    res = compare(cfg, fields, steps, storages, log=log)
    return {"grid": list(cfg["n"][:cfg["dim"]]), "ra": cfg["ra"], "pr": cfg["pr"],
            "developed_at": hist[-1][0], "develop_history": hist, "steps": steps, "modes": res}


QUICK = dict(cfg=W.rayleigh_benard(3, (49, 49, 49), ra=1e5, pr=0.71, storage="fp32"),
             max_develop=20000, chunk=1000, steps=500)
FULL = dict(cfg=W.C2["cfg"], max_develop=60000, chunk=3000, steps=W.C2["steps"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="49^3 Ra 1e5 instead of 385^3 Ra 1e7")
    ap.add_argument("--out", default=None, help="write the result as JSON")
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    res = run(**(QUICK if args.quick else FULL), log=log)
    line = json.dumps(res)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
