"""CPU checks of the C ABI library: it loads, exports every entry point the
header declares, validates parameters, and was compiled with tables that
satisfy the same pins as the oracle's (checked here without a GPU)."""
import json
import math
import os
import re

import numpy as np
import pytest

from oracle import lbmref
from paper_2211_03160_amd import build as hip_build
from paper_2211_03160_amd import lbm, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(hip_build.LIB):
        hip_build.build()


def header_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_entry_point():
    from paper_2211_03160_amd import nn
    names = header_functions()
    assert len(names) >= 40
    assert sorted(names) == sorted(lbm.EXPORTS + nn.NN_EXPORTS)
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert b"gfx950" in L.lbm_version()


def test_library_is_built_for_gfx950_only():
    out = os.popen(f"/opt/rocm/llvm/bin/clang-offload-bundler --list --type=o "
                   f"--input={hip_build.LIB} 2>/dev/null").read()
    if out.strip():
        targets = [t for t in out.split() if "amdgcn" in t]
        assert targets and all("gfx950" in t for t in targets), out


@pytest.mark.parametrize("cfg", [W.C0["cfg"], W.C1["cfg"], W.C2["cfg"],
                                 W.side_heated(3, (17, 17, 17), ra=1e5),
                                 W.periodic_box(2, (8, 8), nu=0.1, alpha=0.07, gbeta=1e-3, a_t=0.3)])
def test_derived_parameters_agree_with_oracle(cfg):
    g = lbm.derive(cfg)
    o = lbmref.Oracle(cfg) if np.prod(cfg["n"]) < 3e6 else None
    ref = o.derived() if o else None
    if ref is None:  # too large for a CPU allocation here: compare closed forms
        H = cfg["n"][cfg["dim"] - 1]
        ref = {"nu": cfg["u_ff"] * H * math.sqrt(cfg["pr"] / cfg["ra"]),
               "alpha": cfg["u_ff"] * H / math.sqrt(cfg["pr"] * cfg["ra"]),
               "gbeta": cfg["u_ff"] ** 2 / ((cfg["t_hot"] - cfg["t_cold"]) * H)}
    for k, v in ref.items():
        assert abs(g[k] - v) <= 1e-14 * max(1.0, abs(v)), (k, g[k], v)


def test_config_zero_lattice_parameters():
    """The 129^2, Ra 1e5, Pr 0.71, U 0.1 cell in lattice units."""
    d = lbm.derive(W.C0["cfg"])
    assert abs(d["nu"] - 0.034373) < 1e-6 and abs(d["tau_f"] - 0.60312) < 1e-5
    assert abs(d["alpha"] - 0.048413) < 1e-6 and abs(d["tau_g"] - 0.69365) < 1e-5
    assert abs(d["gbeta"] - 7.752e-5) < 1e-8


BAD = [
    dict(dim=4),
    dict(n=(0, 5, 1)),
    dict(n=(5, 5, 2)),
    dict(bc=("periodic", "adiabatic", "dirichlet", "dirichlet", "periodic", "periodic")),
    dict(ra=-1.0),
    dict(u_ff=0.5),
    dict(a_t=1.5),
    dict(storage=9),
    dict(nu=-0.01, alpha=0.1, gbeta=0.0),
    dict(nu=0.1, alpha=1e-12, gbeta=0.0, q_e=2.5),
    dict(n=(70000, 70000, 1)),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_parameters_rejected(bad):
    cfg = dict(W.C0["cfg"])
    cfg.update(bad)
    with pytest.raises(lbm.LBMError) as ei:
        lbm.derive(cfg)
    assert ei.value.status == -1
    assert lbm.lib().lbm_workspace_bytes(__import__("ctypes").byref(lbm.make_params(cfg))) == 0
    assert len(lbm.lib().lbm_last_error(None)) > 0


def test_bytes_per_update():
    base = W.C1["cfg"]
    assert lbm.bytes_per_update(base) == 112.0
    assert lbm.bytes_per_update(dict(base, storage="fp64")) == 224.0
    assert lbm.bytes_per_update(dict(base, storage="fp16")) == 56.0
    assert lbm.bytes_per_update(dict(base, storage="bf16")) == 56.0
    assert lbm.bytes_per_update(dict(base, storage="mixed")) == 76.0
    c3 = W.C2["cfg"]
    assert lbm.bytes_per_update(c3) == 208.0
    assert lbm.bytes_per_update(dict(c3, storage="fp16")) == 104.0
    assert lbm.bytes_per_update(dict(c3, storage="mixed")) == 132.0


def test_workspace_fits_the_large_cells():
    assert lbm.workspace_bytes(W.C1["cfg"]) < 8e9
    assert lbm.workspace_bytes(W.C2["cfg"]) < 12.5e9
    assert lbm.workspace_bytes(dict(W.C2["cfg"], storage="fp64")) < 25e9


@pytest.mark.parametrize("dim,thermal", [(2, False), (3, False), (2, True), (3, True)])
def test_kernel_tables_match_oracle_geometry(dim, thermal):
    """The kernels' own tables describe the same lattice as the oracle's:
    the same velocity set (possibly in another order), orthogonal integer
    bases spanning the same moments, and the same weights."""
    e, M, w = lbm.lattice(dim, thermal)
    eo, wo, Mo, _ = lbmref.lattice(dim, thermal)
    assert sorted(map(tuple, e)) == sorted(map(tuple, eo))
    perm = [next(j for j in range(len(eo)) if tuple(eo[j]) == tuple(v)) for v in e]
    assert np.allclose(w, wo[perm], rtol=0, atol=1e-15)
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G)))
    # row by row the kernel basis equals the oracle basis on the same velocities
    assert np.array_equal(M.astype(float), Mo[:, perm])


@pytest.mark.parametrize("dim", [2, 3])
def test_kernel_basis_reproduces_paper_forcing_vectors(dim):
    gold = json.load(open(os.path.join(GOLD, "forcing_moments.json")))
    table = gold["d2q9" if dim == 2 else "d3q19"]
    e, M, w = lbm.lattice(dim, False)
    rng = np.random.default_rng(3)
    u = np.zeros(3)
    F = np.zeros(3)
    u[:dim] = rng.uniform(-0.1, 0.1, dim)
    F[:dim] = rng.uniform(-1e-3, 1e-3, dim)
    cs2 = 1 / 3
    ef = e.astype(float)
    guo = w * (((ef - u) @ F) / cs2 + (ef @ u) * (ef @ F) / cs2 ** 2)
    mf = M @ guo
    names = "xyz"
    for k, entry in enumerate(table):
        ref = 0.0
        for term, coef in entry.items():
            if term == "uF":
                ref += coef * (u @ F)
            elif term[0] == "F":
                ref += coef * F[names.index(term[1])]
            else:
                ref += coef * u[names.index(term[0])] * F[names.index(term[1].lower())]
        assert abs(mf[k] - ref) < 1e-17


def test_bench_gpu_count_and_profile_summaries():
    """bench.py refuses more than one GPU, and the committed rocprofv3
    summaries it reports from parse into the fields of its JSON line (their
    source hash either matches the kernels or they are ignored)."""
    import subprocess
    import sys
    import bench
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
    for spl in (5, 1):
        t = bench.read_traffic(spl)
        assert t is None or 7.5e9 < t < 1.2e10, (spl, t)
    v = bench.read_valu_instructions(5)
    assert v is None or 5e8 < v < 2e9
    import glob
    streams = glob.glob(os.path.join(ROOT, "profiles", "stream*_d2q9_fp32_8193_counters.txt"))
    assert streams
    for name in [os.path.basename(p) for p in streams] + [
            "step_d2q9_fp32_8193_counters.txt", "valu_d2q9_fp32_8193.md", "memreq_d2q9_fp32_8193.md",
            "rb2d_8193_kernel_trace.md"]:
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert "rocprofv3" in text and "$REPO" in text, name
