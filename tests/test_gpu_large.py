"""GPU: the largest single-GPU grid, 1024^3 (2^30 points; the strong-scaling
problem size of the paper's Section 4): the residual of SN and RA, the fused
SN step, and the stored-gradient SS form (whose separate update pass covers
5 * 2^30 elements, more than one dispatch can address).

Needs about 215 GB of device memory: q, q_acc and r (5 fields each) plus the
work area (one rotating state sharing the primitive region, and a second).
The residual is checked on sampled z-slabs against the oracle (planes at the
periodic seam and in the interior); one monitored RK step is checked against
the closed forms of the initial kinetic energy, enstrophy and kinetic-energy
decay rate of the Taylor-Green vortex.
"""
import numpy as np
import pytest

from paper_1610_09146_amd import workloads as W
from tests.helpers import rel_err, slab_rhs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1610_09146_amd import nsf  # noqa: E402

PHYS = W.TGV_PHYS
N = 1024
TUNE = {"fuse": 1}


def _room():
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    need = nsf.workspace_bytes((N, N, N), "SN", "f64", TUNE) + 3 * 5 * N ** 3 * 8
    if free < need + (2 << 30):
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")


@pytest.mark.parametrize("variant", ["SN", "RA"])
def test_1024_rhs_sampled_planes(variant):
    _room()
    print(f"case large rhs {variant} {N}", flush=True)
    s = nsf.Solver((N, N, N), PHYS, variant, "f64", tune=TUNE)
    s.init(W.tgv_pointwise(1610))
    s.rhs()
    torch.cuda.synchronize()
    for k0 in (0, N // 2 - 1, N - 2):
        k1 = k0 + 2
        qs = s.q[:, [(k % N) for k in range(k0 - 2, k1 + 2)]].cpu().numpy()
        ref = slab_rhs(qs, N, PHYS, "ld")
        floor = rel_err(slab_rhs(qs, N, PHYS, "d"), ref)
        got = s.r[:, [(k % N) for k in range(k0, k1)]].cpu().numpy()
        err = rel_err(got, ref)
        assert np.all(err <= np.maximum(1e-12, 4 * floor)), (k0, err, floor)
    del s
    torch.cuda.empty_cache()


def test_1024_monitored_step_closed_forms():
    _room()
    print(f"case large monitored step {N}", flush=True)
    s = nsf.Solver((N, N, N), PHYS, "SN", "f64", tune=TUNE)
    s.init(W.tgv_unperturbed())
    dt = W.tgv_dt(N)
    mon = torch.zeros(4, dtype=torch.float64, device="cuda")
    s.step_monitored(dt, 2, mon)
    ke0, ens0, ke1, _ = mon.cpu().numpy()
    h = 2 * np.pi / N
    kp = (8 * np.sin(h) - np.sin(2 * h)) / (6 * h)
    kpp2 = (15 - 16 * np.cos(h) + np.cos(2 * h)) / (6 * h * h)
    # initial integrals: exact up to the summation round-off of 2^30 terms
    assert abs(ke0 - 0.125) <= 1e-12
    ens_ref = kp ** 2 * (3 / 8 - 5 * PHYS["gamma"] * PHYS["Ma"] ** 2 / 128)
    assert abs(ens0 - ens_ref) <= 1e-12 * ens_ref
    # one step later KE has dropped by rate0 * dt: the forward difference
    # differs from the t = 0 rate by dt/2 times the rate's drift (~1.5e-5 per
    # unit time), 3e-6 relative; bar 1e-4
    rate0 = (3 * kpp2 + (kpp2 - kp ** 2) / 3) / (4 * PHYS["Re"])
    assert abs((ke0 - ke1) / dt - rate0) <= 1e-4 * rate0, ((ke0 - ke1) / dt, rate0)
    d = s.diagnostics()
    assert abs(d[2] - 1.0) <= 1e-12  # mean density unchanged
    del s
    torch.cuda.empty_cache()


def test_1024_ss_rhs_and_step():
    # the stored-gradient algorithm SS at 1024^3: the nine gradient arrays
    # make its footprint q, r and q_acc (15 fields) plus primitives and
    # gradients (14 fields), 29 x 8.6 GB = 249 GB. The residual on sampled
    # z-slabs against the oracle, then (when the accumulator fits too) one
    # monitored RK step against the closed forms of the initial integrals
    # and kinetic-energy decay rate.
    torch.cuda.empty_cache()
    shape = (N, N, N)
    work_b = nsf.workspace_bytes(shape, "SS", "f64")
    field5 = 5 * N ** 3 * 8
    free, _ = torch.cuda.mem_get_info()
    print(f"case large SS {N}: work {work_b / 1e9:.0f} GB, free {free / 1e9:.0f} GB", flush=True)
    if free < work_b + 2 * field5 + (2 << 30):
        pytest.skip(f"SS at {N}^3 needs {(work_b + 2 * field5) / 1e9:.0f} GB for its residual, "
                    f"{free / 1e9:.0f} GB free")
    q = torch.empty((5, N, N, N), dtype=torch.float64, device="cuda")
    r = torch.empty_like(q)
    work = torch.empty(work_b, dtype=torch.uint8, device="cuda")
    nsf.init_fields(shape, PHYS, W.tgv_pointwise(1610), "f64", q, None)
    nsf.rhs(shape, PHYS, "SS", "f64", q, r, work)
    torch.cuda.synchronize()
    for k0 in (0, N // 2 - 1, N - 2):
        k1 = k0 + 2
        qs = q[:, [(k % N) for k in range(k0 - 2, k1 + 2)]].cpu().numpy()
        ref = slab_rhs(qs, N, PHYS, "ld")
        floor = rel_err(slab_rhs(qs, N, PHYS, "d"), ref)
        got = r[:, [(k % N) for k in range(k0, k1)]].cpu().numpy()
        err = rel_err(got, ref)
        assert np.all(err <= np.maximum(1e-12, 4 * floor)), (k0, err, floor)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < field5 + (1 << 30):
        print(f"SS {N}^3 step skipped: {free / 1e9:.0f} GB free for the accumulator", flush=True)
        return
    q_acc = torch.empty_like(q)
    nsf.init_fields(shape, PHYS, W.tgv_unperturbed(), "f64", q, q_acc)
    dt = W.tgv_dt(N)
    mon = torch.zeros(4, dtype=torch.float64, device="cuda")
    nsf.rk_step_monitored(shape, PHYS, "SS", "f64", dt, 2, q, q_acc, r, work, mon)
    ke0, ens0, ke1, _ = mon.cpu().numpy()
    h = 2 * np.pi / N
    kp = (8 * np.sin(h) - np.sin(2 * h)) / (6 * h)
    kpp2 = (15 - 16 * np.cos(h) + np.cos(2 * h)) / (6 * h * h)
    assert abs(ke0 - 0.125) <= 1e-12
    ens_ref = kp ** 2 * (3 / 8 - 5 * PHYS["gamma"] * PHYS["Ma"] ** 2 / 128)
    assert abs(ens0 - ens_ref) <= 1e-12 * ens_ref
    rate0 = (3 * kpp2 + (kpp2 - kp ** 2) / 3) / (4 * PHYS["Re"])
    assert abs((ke0 - ke1) / dt - rate0) <= 1e-4 * rate0, ((ke0 - ke1) / dt, rate0)
    del q, r, work, q_acc
    torch.cuda.empty_cache()
