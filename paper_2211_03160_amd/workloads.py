"""Run configurations and seeded inputs for the thermal LBM cavities.

Pure data: each recipe is a plain dict that both the GPU binding and the CPU
oracle accept.  Nothing here computes any part of the method; derived lattice
parameters (viscosity, diffusivity, relaxation rates, equilibria) are each
side's own business.

Faces are ordered -x, +x, -y, +y, -z, +z.  Gravity points along -y in 2D and
-z in 3D, so Rayleigh-Benard cells heat the bottom face (-y / -z) and cool the
top one.
"""
from __future__ import annotations

import math

PERIODIC, ADIABATIC, DIRICHLET = "periodic", "adiabatic", "dirichlet"


def rayleigh_benard(dim: int, n, ra: float, pr: float, u_ff: float = 0.1,
                    t_hot: float = 1.0, t_cold: float = 0.0,
                    lateral: str = ADIABATIC, storage: str = "fp32",
                    **extra) -> dict:
    """Closed (or laterally periodic) cell heated from below."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    if dim == 2:
        bc = (lateral, lateral, DIRICHLET, DIRICHLET, PERIODIC, PERIODIC)
        tw = (0.0, 0.0, t_hot, t_cold, 0.0, 0.0)
    else:
        bc = (lateral, lateral, lateral, lateral, DIRICHLET, DIRICHLET)
        tw = (0.0, 0.0, 0.0, 0.0, t_hot, t_cold)
    cfg = dict(dim=dim, n=n, bc=bc, t_wall=tw, ra=ra, pr=pr, u_ff=u_ff,
               t_hot=t_hot, t_cold=t_cold, storage=storage)
    cfg.update(extra)
    return cfg


def side_heated(dim: int, n, ra: float, pr: float = 0.71, u_ff: float = 0.1,
                storage: str = "fp32", **extra) -> dict:
    """The paper's cavity: hot -x wall, cold +x wall, others adiabatic."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    bc = [ADIABATIC] * 6
    bc[0] = bc[1] = DIRICHLET
    if dim == 2:
        bc[4] = bc[5] = PERIODIC
    tw = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    cfg = dict(dim=dim, n=n, bc=tuple(bc), t_wall=tw, ra=ra, pr=pr,
               u_ff=u_ff, t_hot=1.0, t_cold=0.0, storage=storage)
    cfg.update(extra)
    return cfg


def periodic_box(dim: int, n, nu: float, alpha: float, gbeta: float = 0.0,
                 storage: str = "fp64", **extra) -> dict:
    """Fully periodic box with explicit transport coefficients."""
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    cfg = dict(dim=dim, n=n, bc=(PERIODIC,) * 6, t_wall=(0.0,) * 6,
               ra=math.nan, pr=math.nan, u_ff=math.nan, t_hot=1.0,
               t_cold=0.0, nu=nu, alpha=alpha, gbeta=gbeta, storage=storage)
    cfg.update(extra)
    return cfg


# The five workloads of the benchmark suite.  Seeds default to 1234; the
# batched sweep draws per-cavity seeds 1234 + k.
SEED = 1234
NOISE = 1e-3

C0 = dict(name="rb2d_129_ra1e5", steps=5000, seed=SEED, noise=NOISE,
          cfg=rayleigh_benard(2, (129, 129), ra=1e5, pr=0.71, storage="fp64"))
C1 = dict(name="rb2d_8193_ra1e8_fp32", warmup=200, steps=1000, seed=SEED,
          noise=NOISE,
          cfg=rayleigh_benard(2, (8193, 8193), ra=1e8, pr=0.71, storage="fp32"))
C2 = dict(name="rb3d_385_ra1e7", steps=500, seed=SEED, noise=NOISE,
          cfg=rayleigh_benard(3, (385, 385, 385), ra=1e7, pr=0.71,
                              storage="fp32"))


def with_storage(cfg: dict, storage: str) -> dict:
    out = dict(cfg)
    out["storage"] = storage
    return out


def batched_sweep(count: int = 64, seed: int = SEED, storage: str = "fp32",
                  heights=(129, 257, 513, 1025), aspects=(1, 2, 4),
                  ra_range=(1e4, 1e8), pr_range=(0.7, 7.0)):
    """The batched sweep: `count` independent Rayleigh-Benard cells with
    heights drawn uniformly from `heights`, aspect ratios from `aspects`
    (width (H - 1) x aspect + 1 nodes, odd when H is odd), Ra log-uniform
    and Pr uniform over the given ranges, each with its own seed
    seed + k.  Returns (cfgs, seeds)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    cfgs, seeds = [], []
    for k in range(count):
        H = int(rng.choice(heights))
        G = int(rng.choice(aspects))
        ra = float(10.0 ** rng.uniform(math.log10(ra_range[0]), math.log10(ra_range[1])))
        pr = float(rng.uniform(*pr_range))
        cfgs.append(rayleigh_benard(2, ((H - 1) * G + 1, H), ra=ra, pr=pr, storage=storage))
        seeds.append(seed + k)
    return cfgs, seeds


C3 = dict(name="batch64_rb2d", steps=240, warmup=120, noise=NOISE, count=64, seed=SEED)
