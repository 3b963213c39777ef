"""GPU: failure detection and checkpoint / resume of the time loop.

Blow-up: the three-stage scheme is stable for lambda_max dt up to sqrt(3)
(its stability polynomial 1 + z + z^2/2 + z^3/6 on the imaginary axis). The
paper's dt gives lambda_max dt of about 0.87 at 64^3 (the rule halves dt per
doubling of N, so the number is the same on every grid), and three times
that dt, about 2.6, amplifies the acoustic grid modes by |1 + z + z^2/2 +
z^3/6| = 2.4 per step at z = 2.6i. Seeded by round-off, they reach the size
of the flow within about 45 steps; within 600 steps nsf_diagnostics must
report the state broken: non-finite values (NSF_ENONFINITE), or a density or
pressure that is no longer positive. The same run at the paper's dt reports
neither.

Resume: at a step boundary q_acc equals the state, so saving q and q_acc to
host memory and loading them into a new solver resumes the run exactly: ten
steps equal five, a save and load, and five more, bitwise. Cases: the fused
SN stage in double precision (its third substep stores q_acc only in a
call's last step), the FP32 form (single-precision state, double
accumulator) and the fused SS stage (its state rotates through r).
"""
import numpy as np
import pytest

from paper_1610_09146_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1610_09146_amd import nsf  # noqa: E402

PHYS = W.TGV_PHYS
MIN_RHO, MIN_P, NONFINITE = 12, 13, 14


def broken(d):
    return d[NONFINITE] > 0 or not (d[MIN_RHO] > 0) or not (d[MIN_P] > 0)


@pytest.mark.parametrize("variant,tune", [("SN", {"fuse": 1}), ("SS", None)])
def test_unstable_step_is_reported(variant, tune):
    n = 64
    print(f"case blow-up {variant} {tune}", flush=True)
    found = {}
    for factor in (1.0, 3.0):
        s = nsf.Solver((n, n, n), PHYS, variant, "f64", tune=tune)
        s.init(W.tgv_unperturbed())
        dt = factor * W.tgv_dt(n)
        steps = 0
        found[factor] = None
        while steps < 600:
            s.step(dt, 50)
            steps += 50
            d = s.diagnostics(check=False)
            if broken(d):
                found[factor] = steps
                if d[NONFINITE] > 0:
                    with pytest.raises(nsf.NsfError) as ei:
                        s.diagnostics()
                    assert ei.value.code == nsf.ENONFINITE
                break
        print(f"  dt x {factor}: broken after {found[factor]} steps", flush=True)
    assert found[1.0] is None
    assert found[3.0] is not None and found[3.0] <= 600


@pytest.mark.parametrize("variant,precision,tune", [("SN", "f64", {"fuse": 1}),
                                                    ("SN", "f32", {"fuse": 1}),
                                                    ("SS", "f64", {"fuse": 1})])
def test_resume_from_saved_state_is_exact(variant, precision, tune):
    shape = (48, 40, 36)
    print(f"case resume {variant} {precision} {tune}", flush=True)
    tgv = W.tgv_pointwise(31, 1e-3)
    dt = W.tgv_dt(48)
    full = nsf.Solver(shape, PHYS, variant, precision, tune=tune)
    full.init(tgv)
    full.step(dt, 10)
    first = nsf.Solver(shape, PHYS, variant, precision, tune=tune)
    first.init(tgv)
    first.step(dt, 5)
    torch.cuda.synchronize()
    saved = (first.q.cpu().numpy().copy(), first.q_acc.cpu().numpy().copy())
    del first
    resumed = nsf.Solver(shape, PHYS, variant, precision, tune=tune)
    resumed.q.copy_(torch.from_numpy(saved[0]))
    resumed.q_acc.copy_(torch.from_numpy(saved[1]))
    resumed.step(dt, 5)
    torch.cuda.synchronize()
    assert torch.equal(resumed.q, full.q)
    assert torch.equal(resumed.q_acc, full.q_acc)
    assert np.array_equal(resumed.diagnostics(), full.diagnostics())
