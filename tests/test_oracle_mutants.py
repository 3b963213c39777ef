"""The oracle's pins reject plausible mistakes: each case below plants one
mistake (a flipped sign, a term moved or dropped, a wrong coefficient, axis
or field) into a temporary copy of the C oracle, builds it, and runs the
checks of tests/oracle_checks.py on it. Every check listed for a mistake must
fail on the mutant (and all of them pass on the real oracle, in
tests/test_oracle_energy_pins.py). Nothing here touches the real oracle's
sources or library.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

from oracle import oracle as O
from tests import oracle_checks as C

PHYS_VISC = dict(Re=50.0, Ma=0.3, Pr=0.71, gamma=1.4)

# name -> (text in nsf_oracle_body.inc, replacement, checks that must fail)
MUTANTS = {
    # energy equation, eq (3) with the skew split of eq (8)
    "pressure_work_sign": (
        "out[4] = -conv / (REAL)2 - pflux",
        "out[4] = -conv / (REAL)2 + pflux",
        ("continuum", "wave_iso", "wave_p")),
    "pressure_work_inside_skew_split": (
        "pflux += FN(d1prod)(c, p, vel[b], b, i, j, k);",
        "pflux += (FN(d1prod)(c, p, vel[b], b, i, j, k) + u[b] * FN(d1)(c, p, b, i, j, k)"
        " + p[idx] * G[b][b]) / (REAL)2;",
        ("wave_iso", "wave_p")),
    "pressure_work_product_rule": (
        "pflux += FN(d1prod)(c, p, vel[b], b, i, j, k);",
        "pflux += u[b] * FN(d1)(c, p, b, i, j, k) + p[idx] * G[b][b];",
        ("wave_iso", "wave_p")),
    "energy_skew_density_for_energy": (
        "+ rhoE[idx] * G[b][b];",
        "+ rho[idx] * G[b][b];",
        ("continuum", "wave_iso", "wave_p")),
    "energy_skew_without_half": (
        "out[4] = -conv / (REAL)2",
        "out[4] = -conv",
        ("continuum", "wave_iso", "wave_p")),
    "viscous_work_dropped": (
        "work += tau * G[a][b];",
        "work += (REAL)0 * tau;",
        ("continuum", "wave_iso", "wave_p")),
    "velocity_times_viscous_force_dropped": (
        "vwork += u[a] * V[a];",
        "vwork += (REAL)0;",
        ("continuum", "wave_iso", "wave_p")),
    "heat_flux_sign": (
        "+ kappa * heat",
        "- kappa * heat",
        ("continuum", "wave_p")),
    "conductivity_without_mach_square": (
        "((c->gamma - (REAL)1) * c->Ma * c->Ma * c->Pr * Re)",
        "((c->gamma - (REAL)1) * c->Ma * c->Pr * Re)",
        ("continuum", "wave_p")),
    # momentum equation, eqs (2) and (4)
    "viscous_third_as_two_thirds": (
        "V[a] = (lap + (FN(d2)(c, vel[a], a, i, j, k) + cross) / (REAL)3) / Re;",
        "V[a] = (lap + (REAL)2 * (FN(d2)(c, vel[a], a, i, j, k) + cross) / (REAL)3) / Re;",
        ("continuum", "wave_iso", "wave_p")),
    "stress_trace_coefficient": (
        "(a == b ? (REAL)2 * div / (REAL)3 : (REAL)0)",
        "(a == b ? div / (REAL)3 : (REAL)0)",
        ("continuum", "wave_iso", "wave_p")),
    "pressure_gradient_axis": (
        "out[1 + a] = -conv / (REAL)2 - FN(d1)(c, p, a, i, j, k) + V[a];",
        "out[1 + a] = -conv / (REAL)2 - FN(d1)(c, p, (a + 1) % 3, i, j, k) + V[a];",
        ("continuum", "wave_iso", "wave_p")),
    "momentum_skew_density_for_momentum": (
        "+ mom[a][idx] * G[b][b];",
        "+ rho[idx] * G[b][b];",
        ("continuum", "wave_iso", "wave_p")),
    # mass equation, eq (1)
    "mass_skew_term_dropped": (
        "s += FN(d1)(c, mom[b], b, i, j, k) + u[b] * FN(d1)(c, rho, b, i, j, k)\n"
        "             + rho[idx] * G[b][b];",
        "s += FN(d1)(c, mom[b], b, i, j, k) + u[b] * FN(d1)(c, rho, b, i, j, k);",
        ("continuum", "wave_iso")),
    # diagnostics (Section 3)
    "min_pressure_from_temperature": (
        "REAL pp = prim[3 * npts + idx];",
        "REAL pp = prim[4 * npts + idx];",
        ("extrema",)),
    "max_norm_signed": (
        "REAL a = val < 0 ? -val : val;",
        "REAL a = val;",
        ("norms",)),
    # single-precision stage model: the accumulator rounded instead
    "rounded_accumulator": (
        "for (size_t e = 0; e < n5; ++e) q[e] = (REAL)(float)q[e];",
        "for (size_t e = 0; e < n5; ++e) qacc[e] = (REAL)(float)qacc[e];",
        ("stage_model",)),
}


def _check(name):
    if name == "continuum":
        return C.continuum_ok(PHYS_VISC)[0]
    if name == "wave_iso":
        return C.wave_ok(16, PHYS_VISC, "isothermal", 0)[0] and \
            C.wave_ok(12, PHYS_VISC, "isothermal", 1)[0]
    if name == "wave_p":
        return C.wave_ok(16, PHYS_VISC, "pressure", 2)[0]
    if name == "extrema":
        return C.extrema_ok(16, PHYS_VISC)[0]
    if name == "norms":
        return C.diag_norm_errors(PHYS_VISC) == 0
    if name == "stage_model":
        return C.stage_model_mismatch(PHYS_VISC) == 0.0
    raise KeyError(name)


def _build(tmp, name):
    src_dir = os.path.dirname(O._SRC)
    d = os.path.join(tmp, name)
    os.makedirs(d)
    shutil.copy(O._SRC, d)
    body = open(os.path.join(src_dir, "nsf_oracle_body.inc")).read()
    old, new, _ = MUTANTS[name]
    assert body.count(old) == 1, (name, body.count(old))
    with open(os.path.join(d, "nsf_oracle_body.inc"), "w") as f:
        f.write(body.replace(old, new))
    lib = os.path.join(d, "liboracle_mutant.so")
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-std=gnu11", "-fPIC",
                           "-shared", os.path.join(d, "nsf_oracle.c"), "-o", lib, "-lm"])
    return lib


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("oracle_mutants"))
    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        libs = dict(zip(MUTANTS, ex.map(lambda n: _build(tmp, n), MUTANTS)))
    return libs


def test_real_oracle_passes_every_check():
    for name in ("continuum", "wave_iso", "wave_p", "extrema", "norms", "stage_model"):
        assert _check(name), name


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_mutant_is_caught(mutant, mutant_libs):
    with O.library(mutant_libs[mutant]):
        passed = {c: _check(c) for c in MUTANTS[mutant][2]}
    assert not any(passed.values()), (mutant, passed)
