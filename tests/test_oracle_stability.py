"""Oracle: the time step's stability limit and the blow-up it reports.

The three-stage scheme is stable for lambda_max dt up to sqrt(3) (its
stability polynomial 1 + z + z^2/2 + z^3/6 on the imaginary axis); the
paper's dt (3.385e-3 at 64^3, halved per doubling of N) gives about 0.87 on
every grid. On a 16^3 Taylor-Green state with +-1e-3 pointwise noise (all
grid modes present), 200 steps at that dt stay physical, while three times
it (about 2.6: growth by 2.4 per step for the acoustic grid modes) must be
reported by the diagnostics: non-finite values, or a density or pressure
that is no longer positive.
"""
import numpy as np

from oracle import oracle as O
from paper_1610_09146_amd import workloads as W

PHYS = W.TGV_PHYS
MIN_RHO, MIN_P, NONFINITE = 12, 13, 14


def broken(d):
    return d[NONFINITE] > 0 or not (d[MIN_RHO] > 0) or not (d[MIN_P] > 0)


def run(factor, steps=200, chunk=25):
    n = 16
    q = O.init((n, n, n), PHYS, W.tgv_pointwise(3, 1e-3), prec="d")
    dt = factor * 3.385e-3 * 64 / n
    for done in range(chunk, steps + 1, chunk):
        with np.errstate(all="ignore"):
            q = O.rk_step(q, PHYS, dt, chunk, prec="d")
        d = O.diagnostics(q, PHYS)
        if broken(d):
            return done, d
    return None, O.diagnostics(q, PHYS)


def test_paper_step_stays_physical():
    at, d = run(1.0)
    assert at is None, d
    # kinetic energy decays, never grows, at a stable step
    assert d[0] < 0.125


def test_three_times_the_step_is_reported():
    at, d = run(3.0)
    assert at is not None and at <= 200, d
