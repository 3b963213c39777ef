"""Pins of the oracle's energy equation, diagnostics extrema and
single-precision stage model (Section 2, eqs (1)-(10); Section 3).

The continuum check (fourth-order convergence to the exact residual of the
divergence form) fixes every term's sign, coefficient and axis; the exact
discrete residual of one-dimensional compressive waves fixes the discrete
arrangement (skew split with phi = E, pressure work in divergence form
outside the split), which the continuum cannot see. tests/oracle_checks.py
states both constructions; tests/test_oracle_mutants.py shows each failing on
oracle copies with a planted mistake.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests import oracle_checks as C

PHYS = dict(Re=1600.0, Ma=0.1, Pr=0.71, gamma=1.4)  # Section 3
# viscous, heat and pressure terms of comparable size
PHYS_VISC = dict(Re=50.0, Ma=0.3, Pr=0.71, gamma=1.4)


@pytest.mark.parametrize("phys", [PHYS_VISC, dict(Re=400.0, Ma=0.5, Pr=1.0, gamma=1.6)],
                         ids=["Re50", "Re400"])
def test_continuum_residual_fourth_order(phys):
    # observed order 4 on N = 16, 32, 64: per-halving error ratios within
    # C.CONT_RATIO_BOUNDS (16 in the limit; the 16 -> 32 step still carries
    # the sixth-order term of the triple-product harmonics), and the finest
    # grid within 1e-4 (truncation, not a wrong term)
    ok, e = C.continuum_ok(phys)
    assert ok, (e[:-1] / e[1:], e)


@pytest.mark.parametrize("kind", ["isothermal", "pressure"])
@pytest.mark.parametrize("N", [12, 16])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_compressive_wave_exact_discrete_residual(kind, N, axis):
    ok, e = C.wave_ok(N, PHYS_VISC, kind, axis)
    assert ok, e


@pytest.mark.parametrize("kind", ["isothermal", "pressure"])
def test_compressive_wave_paper_parameters_double(kind):
    # the double instantiation at the Taylor-Green parameters (p0 = 71: the
    # pressure terms dominate, the floor is the round-off of the double run)
    e0, e1, e4, other = C.wave_closed_form_errors(16, PHYS, kind, 0, prec="d")
    assert e0 < 1e-13 and e1 < 1e-13 and e4 < 1e-13, (e0, e1, e4)


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("Ma", [0.1, 0.3])
def test_tgv_diagnostics_extrema(N, Ma):
    ok, e = C.extrema_ok(N, dict(PHYS, Ma=Ma))
    assert ok, e


def test_diagnostics_count_nonfinite_and_max_norms():
    # max |q_f| is the largest magnitude whatever the sign, min rho the
    # smallest density, and the non-finite count the NaN and Inf entries
    assert C.diag_norm_errors(PHYS) == 0


@pytest.mark.parametrize("prec", ["d", "ld"])
def test_single_precision_stage_model(prec):
    # rk_step_slab(stage_dtype=float32), the reference of the full-size check
    # of the single-precision form, against the full-grid C step with the
    # same model written separately (each substep's input rounded to float,
    # the accumulator not): bitwise equal on the slab's output planes
    shape = (12, 10, 20)
    tgv = {"pert_kind": 1, "pert_amp": 0.05, "seed": 23}
    q = O.init(shape, PHYS, tgv, prec=prec)
    dt = 0.01
    full = O.rk_step_rounded(q, PHYS, dt, 1, prec=prec)
    for k0, m in ((0, 2), (11, 3), (18, 2)):
        idx = [(k % 20) for k in range(k0 - 6, k0 + m + 6)]
        got = O.rk_step_slab(q[:, idx], 20, PHYS, dt, prec=prec, stage_dtype=np.float32)
        assert np.array_equal(got, full[:, idx[6:6 + m]])
    # and the rounding moves the result by single-precision amounts only
    plain = O.rk_step(q, PHYS, dt, 1, prec=prec)
    inc = (plain - q).astype(np.float64).reshape(5, -1)
    d32 = (full - plain).astype(np.float64).reshape(5, -1)
    rel = np.abs(d32).max(axis=1) / np.abs(inc).max(axis=1)
    assert np.all(rel > 1e-9) and np.all(rel < 1e-4), rel
