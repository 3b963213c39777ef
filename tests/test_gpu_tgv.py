"""GPU: Taylor-Green evolution over many steps (paper Section 3).

The comparison curves the paper uses are not available, so these runs are
checked for self-consistency against what the discretisation fixes:
  * the kinetic-energy decay rate at t = 0, a closed form of the modified
    wavenumbers k'(1) and k''(1) (the same formula the oracle is pinned to),
    read here off the monitored kinetic energy of the time-stepped run;
  * fourth-order spatial convergence of the kinetic energy at fixed time
    on 32^3, 64^3 and 128^3 (the fourth-order central differences);
  * conservation of mass and momentum over the run (skew-symmetric
    convection and central differences on a periodic grid).
"""
import numpy as np
import pytest

from paper_1610_09146_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1610_09146_amd import tgv  # noqa: E402

PHYS = W.TGV_PHYS


def _kp(n):
    h = 2 * np.pi / n
    kp = (8 * np.sin(h) - np.sin(2 * h)) / (6 * h)
    kpp2 = (15 - 16 * np.cos(h) + np.cos(2 * h)) / (6 * h * h)
    return kp, kpp2


def test_ke_rate_at_start_matches_closed_form():
    # -dKE/dt(0) = (3 k''^2 + (k''^2 - k'^2)/3) / (4 Re) for V0 = 1. The
    # central difference of the per-step KE at t = dt differs from the t = 0
    # rate by about |d^2 KE/dt^2| dt (the rate drifts by ~1.5e-5 per unit time
    # early on, i.e. 1e-4 relative over one step): bar 5e-4.
    n = 64
    print(f"case tgv ke-rate n={n}", flush=True)
    rec = tgv.run(n, 4 * W.tgv_dt(n))
    kp, kpp2 = _kp(n)
    rate0 = (3 * kpp2 + (kpp2 - kp ** 2) / 3) / (4 * PHYS["Re"])
    got = rec["dissipation"][1]
    assert abs(got - rate0) <= 5e-4 * rate0, (got, rate0)
    # the enstrophy record starts at its closed form (density weighted)
    ens0 = kp ** 2 * (3 / 8 - 5 * PHYS["gamma"] * PHYS["Ma"] ** 2 / 128)
    assert abs(rec["enstrophy"][0] - ens0) <= 1e-13 * ens0


def test_ke_fourth_order_in_space():
    # KE(t = 1) on 32^3, 64^3, 128^3: the observed order
    # log2(|KE32 - KE64| / |KE64 - KE128|) of the fourth-order scheme lies in
    # [3.5, 4.5] (measured 3.8; a second-order slip would give about 2).
    # Time errors (RK3, dt <= 3.4e-3) are below 1e-10, far under the
    # 4e-9 difference between the two finest grids.
    t_end = 1.0
    ke = []
    for n in (32, 64, 128):
        print(f"case tgv convergence n={n}", flush=True)
        rec = tgv.run(n, t_end)
        ke.append(np.interp(t_end, rec["t"], rec["ke"]))
    order = np.log2(abs(ke[0] - ke[1]) / abs(ke[1] - ke[2]))
    assert 3.5 <= order <= 4.5, (ke, order)


def test_long_run_conserves_mass_and_momentum():
    n = 64
    print(f"case tgv conservation n={n}", flush=True)
    rec = tgv.run(n, 2.0, tgv=W.tgv_pointwise(7, 1e-3))
    s0, s1 = rec["sums_initial"], rec["sums_final"]
    assert abs(s1[0] - s0[0]) <= 1e-14 * abs(s0[0])
    # momentum means start at round-off level (perturbed Taylor-Green)
    assert np.all(np.abs(s1[1:4] - s0[1:4]) <= 1e-14)
    # kinetic energy decays (viscous, unforced) and stays finite
    assert np.all(np.isfinite(rec["ke"]))
    assert rec["ke"][-1] < rec["ke"][0]
