"""GPU: kinetic-energy / enstrophy monitor of the RK driver.

nsf_rk_step_monitored records, per step, the grid means of rho|u|^2/2 and
rho|curl u|^2/2 (Section 3 diagnostics) of the state at the start of the
step. The fused SN and RA forms take these sums inside their first stage
kernel, the other forms run the diagnostics pass. Checked against the oracle's
diagnostics of the oracle's own RK trajectory (extended precision) and
against nsf_diagnostics of the same GPU states, and the monitored run must
leave the same state as the unmonitored one.

Bars. Double precision: 1e-11 against the oracle (the state itself agrees
to ~1e-12 after these few steps and both integrals are smooth functionals of
it); 1e-13 against nsf_diagnostics (same state, summation order only).
Single precision: the fused kernel forms u and curl u in float. Each
derivative sums differences with weight about 18/(12 h), so with h = 2 pi/72
the vorticity carries about 17 float roundings (6e-8 each) relative to |u|,
and |omega|^2 twice that: 2e-6. With a factor 4 the single-precision bar is
1e-5 against nsf_diagnostics (which works in double from the same float
state) and 2e-5 against the oracle (which adds the float trajectory's own
drift, itself below 1e-6 after three steps).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1610_09146_amd import workloads as W
from tests.helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1610_09146_amd import nsf  # noqa: E402

PHYS = W.TGV_PHYS
# 72 x 40 x 36: ragged x tile (72 = 2 * 32 + 8), ragged y for 16-high tiles
SHAPE = (72, 40, 36)
NSTEPS = 3
TGV = W.tgv_pointwise(5, 1e-3)

CASES = [
    ("SN", "f64", {"fuse": 1}),
    ("SN", "f64", {"fuse": 1, "block_y": 8, "zchunk": 7}),
    ("SN", "f32", {"fuse": 1}),
    ("SN", "f32", {"fuse": 1, "block_y": 16, "zchunk": 5}),
    ("RA", "f64", {"fuse": 1}),
    ("RA", "f64", {"fuse": 1, "block_y": 8, "zchunk": 7}),
    ("RA", "f32", {"fuse": 1, "block_y": 16, "zchunk": 5}),
    ("RA", "f64", None),
    ("SN", "f64", None),
    ("SS", "f64", None),
    ("SS", "f64", {"fuse": 1}),
    ("RS", "f64", None),
    ("BL", "f64", None),
    ("SS", "f32", None),
    ("RS", "f32", None),
]


@pytest.fixture(scope="module")
def oracle_run():
    """(KE, enstrophy) of the oracle's states at the start of each step, and
    the oracle's state after the last step."""
    q = O.init(SHAPE, PHYS, TGV, prec="ld")
    dt = W.tgv_dt(max(SHAPE))
    out = []
    for _ in range(NSTEPS):
        d = O.diagnostics(q, PHYS, prec="ld")
        out.append((d[0], d[1]))
        q = O.rk_step(q, PHYS, dt, 1, prec="ld")
    return np.array(out), q


def _solver(variant, precision, tune):
    s = nsf.Solver(SHAPE, PHYS, variant, precision, tune=tune)
    s.init(TGV)
    return s


@pytest.mark.parametrize("variant,precision,tune", CASES)
def test_monitor(variant, precision, tune, oracle_run):
    oracle_monitor, oracle_final = oracle_run
    print(f"case monitor {variant} {precision} {tune} {SHAPE}", flush=True)
    dt = W.tgv_dt(max(SHAPE))
    mon_solver = _solver(variant, precision, tune)
    mon = torch.full((2 * NSTEPS,), float("nan"), dtype=torch.float64, device="cuda")
    mon_solver.step_monitored(dt, NSTEPS, mon)
    torch.cuda.synchronize()
    got = mon.cpu().numpy().reshape(NSTEPS, 2)
    assert np.all(np.isfinite(got))

    # the same states, one step at a time through nsf_diagnostics
    ref_solver = _solver(variant, precision, tune)
    gpu_diag = []
    for _ in range(NSTEPS):
        d = ref_solver.diagnostics()
        gpu_diag.append((d[0], d[1]))
        ref_solver.step(dt, 1)
    gpu_diag = np.array(gpu_diag)

    f64 = precision == "f64"
    bar_same, bar_oracle = (1e-13, 1e-11) if f64 else (1e-5, 2e-5)
    rel_same = np.abs(got - gpu_diag) / np.abs(gpu_diag)
    rel_oracle = np.abs(got - oracle_monitor) / np.abs(oracle_monitor)
    assert np.all(rel_same <= bar_same), rel_same
    assert np.all(rel_oracle <= bar_oracle), rel_oracle

    # monitoring does not change the trajectory. The monitored kernel is a
    # separate build; where it keeps the branching form (single precision,
    # the 8-row double-precision tile) the compiler may fuse multiply-adds
    # differently. The two runs must agree to 1e-14 in double precision, or
    # within 4x the unmonitored run's own error against the
    # extended-precision oracle, per field (rho w starts near zero, so its
    # relative rounding error is the largest).
    a = mon_solver.q.cpu().numpy().astype(np.float64)
    b = ref_solver.q.cpu().numpy().astype(np.float64)
    own = rel_err(b, oracle_final)
    if f64:
        assert np.all(rel_err(a, b) <= np.maximum(1e-14, 4 * own)), (rel_err(a, b), own)
        assert torch.equal(mon_solver.q_acc, mon_solver.q)
    else:
        assert np.all(rel_err(a, b) <= 4 * own), (rel_err(a, b), own)


def test_monitor_deterministic_and_zero_steps():
    dt = W.tgv_dt(max(SHAPE))
    runs = []
    for _ in range(2):
        s = _solver("SN", "f64", {"fuse": 1})
        mon = torch.zeros(2 * NSTEPS, dtype=torch.float64, device="cuda")
        s.step_monitored(dt, NSTEPS, mon)
        runs.append(mon.cpu())
    assert torch.equal(runs[0], runs[1])
    # nsteps = 0 writes nothing and leaves the state alone
    s = _solver("SN", "f64", {"fuse": 1})
    before = s.q.clone()
    mon = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    s.step_monitored(dt, 0, mon)
    torch.cuda.synchronize()
    assert torch.equal(mon.cpu(), torch.full((2,), 7.0, dtype=torch.float64))
    assert torch.equal(s.q, before)


def test_monitor_tgv_closed_forms():
    # unperturbed Taylor-Green at t = 0: KE = 1/8 and enstrophy =
    # k'(1)^2 (3/8 - 5 gamma Ma^2/128) (the closed forms the oracle is pinned to)
    n = 64
    # float: the initial state is rounded to float and the fused kernel forms
    # u and curl u in float (about 2e-6 relative, see the bars above)
    for variant, precision, tol in (("SN", "f64", 1e-13), ("SN", "f32", 1e-5), ("RA", "f64", 1e-13),
                                    ("RA", "f32", 1e-5)):
        s = nsf.Solver((n, n, n), PHYS, variant, precision, tune={"fuse": 1})
        s.init(W.tgv_unperturbed())
        mon = torch.zeros(2, dtype=torch.float64, device="cuda")
        s.step_monitored(W.tgv_dt(n), 1, mon)
        ke, ens = mon.cpu().numpy()
        h = 2 * np.pi / n
        kp = (8 * np.sin(h) - np.sin(2 * h)) / (6 * h)
        ens_ref = kp ** 2 * (3 / 8 - 5 * PHYS["gamma"] * PHYS["Ma"] ** 2 / 128)
        assert abs(ke - 0.125) <= tol * 0.125, (precision, ke)
        assert abs(ens - ens_ref) <= tol * ens_ref, (precision, ens, ens_ref)
