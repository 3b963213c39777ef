"""Autotuner and the SN / RS algorithm entries on the GPU."""
import os

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


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_autotune_choice_is_parity_gated_and_used_by_auto(tmp_path, precision):
    shape = (48, 40, 36)
    cache = str(tmp_path / "tune.jsonl")
    best = nsf.autotune(shape, PHYS, precision, quick=False, steps=1, cache_path=cache)
    bar = 1e-10 if precision == "f64" else 1e-3
    assert best["pt_rhs_per_s"] > 0 and best["parity_rel_err"] <= bar
    assert nsf.tune_get(shape, precision)["variant"] == best["variant"]
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"gfx950"' in lines[0]
    assert nsf.tune_load(cache) == 1
    # AUTO runs exactly the recorded configuration
    tgv = W.tgv_pointwise(5, 1e-3)
    a = nsf.Solver(shape, PHYS, "AUTO", precision)
    b = nsf.Solver(shape, PHYS, best["variant"], precision, tune=best["tune"])
    for s in (a, b):
        s.init(tgv)
        s.step(2e-3, 2)
    assert torch.equal(a.q, b.q) and torch.equal(a.q_acc, b.q_acc)


@pytest.mark.parametrize("variant", ["SN", "RS"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (40, 36, 50)])
def test_sn_rs_parity(variant, shape):
    q = O.init(shape, PHYS, W.tgv_pointwise(3, 1e-3), prec="ld")
    ref = O.rhs(q, PHYS, prec="ld")
    s = nsf.Solver(shape, PHYS, variant, "f64")
    s.q.copy_(torch.from_numpy(q.astype(np.float64)))
    s.rhs()
    err = rel_err(s.r.cpu().numpy(), ref)
    floor = rel_err(O.rhs(q.astype(np.float64), PHYS, prec="d"), ref)
    assert np.all(err <= np.maximum(1e-12, 4 * floor)), err


@pytest.mark.parametrize("tune", [None, {"naive": 1}, {"zchunk": 7, "block_y": 8},
                                  {"block_y": 16, "zchunk": 5}])
@pytest.mark.parametrize("shape", [(16, 16, 16), (70, 11, 9), (40, 36, 50), (5, 6, 7)])
def test_ss_parity_tunings(tune, shape):
    q = O.init(shape, PHYS, W.tgv_pointwise(3, 1e-3), prec="ld")
    ref = O.rhs(q, PHYS, prec="ld")
    s = nsf.Solver(shape, PHYS, "SS", "f64", tune=tune)
    s.q.copy_(torch.from_numpy(q.astype(np.float64)))
    s.rhs()
    err = rel_err(s.r.cpu().numpy(), ref)
    floor = rel_err(O.rhs(q.astype(np.float64), PHYS, prec="d"), ref)
    assert np.all(err <= np.maximum(1e-12, 4 * floor)), err
