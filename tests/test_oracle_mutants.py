"""Planted mistakes: each mutant is a plausible error (a dropped term, a
wrong sign, index or factor, a transposed operand) patched into a temporary
copy of the oracle source and compiled on the CPU.  The oracle's pin tests
must fail on every one of them; otherwise the pins would not be able to tell
a wrong oracle from a right one."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbmref.c")

MUTANTS = {
    "velocity without the half-force shift": (
        "c->u[a * N + idx] = (j[a] + 0.5 * F[a]) / rho;", "c->u[a * N + idx] = j[a] / rho;"),
    "anti-bounce-back sign": (
        "v = -v + c->omega * c->p.t_wall[face];", "v = v + c->omega * c->p.t_wall[face];"),
    "forcing without (I - S/2)": (
        "+ (1.0 - 0.5 * c->s[k]) * mf[k];", "+ mf[k];"),
    "Eq. 6a last entry as printed": (
        "mf[8] = u[0] * F[1] + u[1] * F[0];", "mf[8] = u[0] * F[0] + u[1] * F[1];"),
    "transposed basis product": (
        "acc += A[k][i] * x[i];", "acc += A[i][k] * x[i];"),
    "bounce-back to the same direction": (
        "v = src[L->opp[i] * N + idx];", "v = src[i * N + idx];"),
    "equilibrium second-order coefficient": (
        "4.5 * eu * eu", "3.0 * eu * eu"),
    "wall flux factor": (
        "- 2.0 * c->gp[out * N + idx];", "- c->gp[out * N + idx];"),
    "anti-bounce-back weight": (
        "(4.0 + c->a_t) / 10.0 : (6.0 + c->a_t) / 21.0;", "(4.0 + c->a_t) / 20.0 : (6.0 + c->a_t) / 42.0;"),
    "buoyancy without T0": (
        "F[c->gaxis] = rho * c->gbeta * (T - c->t0);", "F[c->gaxis] = rho * c->gbeta * T;"),
    "viscosity to relaxation time": (
        "double tau_f = 3.0 * c->nu + 0.5;", "double tau_f = 3.0 * c->nu + 1.0;"),
    # buoyancy acts along z only, so terms carrying F_x or F_y vanish for
    # every valid input and mutating them changes nothing; plant the error
    # on a term that carries F_z
    "Eq. 6b entry sign": (
        "mf[10] = -2.0 * u[0] * F[0] + u[1] * F[1] + u[2] * F[2];",
        "mf[10] = -2.0 * u[0] * F[0] + u[1] * F[1] - u[2] * F[2];"),
    "thermal equilibrium energy moment": (
        "neq[3] = a_t * T;", "neq[3] = a_t;"),
    "push instead of pull": (
        "s[a] = xyz[a] - L->e[i][a];", "s[a] = xyz[a] + L->e[i][a];"),
    "odd rates equal to the shear rate": (
        "8.0 * (2.0 - s_nu) / (8.0 - s_nu)", "s_nu"),
    "thermal relaxation time with the flow sound speed": (
        "double tau_g = c->alpha / cs2t + 0.5;", "double tau_g = 3.0 * c->alpha + 0.5;"),
    "3D diagonal weight": (
        "s == 1 ? 1.0 / 18.0 : 1.0 / 36.0;", "s == 1 ? 1.0 / 18.0 : 1.0 / 72.0;"),
    "gravity along x in 2D": (
        "c->gaxis = p->dim == 2 ? 1 : 2;", "c->gaxis = p->dim == 2 ? 0 : 2;"),
    "Nusselt from one step only": (
        "double q = 0.5 * (c->flux[0][face] + c->flux[1][face]);", "double q = c->flux[c->t & 1][face];"),
    "volume Nusselt number with T instead of T - T0": (
        "uT += c->u[c->gaxis * N + idx] * (c->T[idx] - c->t0);", "uT += c->u[c->gaxis * N + idx] * c->T[idx];"),
    "volume Nusselt number with the horizontal velocity": (
        "uT += c->u[c->gaxis * N + idx] * (c->T[idx] - c->t0);", "uT += c->u[0 * N + idx] * (c->T[idx] - c->t0);"),
    "volume Nusselt number with the viscosity": (
        "d->nu_vol = 1.0 + c->H * (uT / N) / (c->alpha * c->dT);", "d->nu_vol = 1.0 + c->H * (uT / N) / (c->nu * c->dT);"),
    "Reynolds number with the thermal diffusivity": (
        "d->re = sqrt(u2 / N) * c->H / c->nu;", "d->re = sqrt(u2 / N) * c->H / c->alpha;"),
    "Reynolds number without the square root": (
        "d->re = sqrt(u2 / N) * c->H / c->nu;", "d->re = (u2 / N) * c->H / c->nu;"),
    "Reynolds number with the width for H": (
        "d->re = sqrt(u2 / N) * c->H / c->nu;", "d->re = sqrt(u2 / N) * c->n[0] / c->nu;"),
    "3D equilibrium basis row": (
        "case 10: return (3.0 * s - 5.0) * (3.0 * x * x - s);", "case 10: return (3.0 * s - 5.0) * (3.0 * y * y - s);"),
}

PINS = ["tests/test_oracle_lattice.py", "tests/test_oracle_collision.py", "tests/test_oracle_physics.py",
        "tests/test_oracle_diagnostics.py"]


def _run_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique or missing: {old}"
    d = os.path.join(tmp, str(abs(hash(name))))
    os.makedirs(d, exist_ok=True)
    shutil.copy(os.path.join(ROOT, "oracle", "lbmref.h"), d)
    c = os.path.join(d, "lbmref.c")
    open(c, "w").write(src.replace(old, new))
    so = os.path.join(d, "liblbmref.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                    "-fPIC", "-shared", "-w", "-o", so, c, "-lm"], check=True)
    env = dict(os.environ, LBMREF_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-k", "not onset"] + PINS, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    return name, r.returncode, r.stdout[-400:]


def test_pins_catch_every_planted_mistake(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda n: _run_mutant(n, str(tmp_path)), MUTANTS))
    survivors = [(n, out) for n, rc, out in results if rc == 0]
    for n, rc, out in results:
        print(f"{n}: {'caught' if rc != 0 else 'SURVIVED'}")
    assert not survivors, survivors


def test_unmutated_copy_passes(tmp_path):
    """The harness itself: a verbatim copy of the oracle passes the pins."""
    MUTANTS["(none)"] = ("#include <math.h>", "#include <math.h>")
    try:
        name, rc, out = _run_mutant("(none)", str(tmp_path))
    finally:
        del MUTANTS["(none)"]
    assert rc == 0, out
