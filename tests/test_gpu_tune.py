"""Autotuner, and the RA / SN / RS algorithms as kernels of their own, on the GPU."""
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
    assert len(lines) == 1 and '"gfx950"' in lines[0] and '"gstore"' in lines[0]
    assert nsf.tune_load(cache) == 1
    # AUTO runs exactly the recorded configuration
    tgv = W.tgv_pointwise(5, 1e-3)
    a = nsf.Solver(shape, PHYS, "AUTO", precision)
    b = nsf.Solver(shape, PHYS, best["variant"], precision, tune=best["tune"])
    for s in (a, b):
        s.init(tgv)
        s.step(2e-3, 2)
    assert torch.equal(a.q, b.q) and torch.equal(a.q_acc, b.q_acc)


FAMILIES = ("ra_zsweep", "sn_zsweep", "ss_zsweep", "rs_zsweep", "ra_fused", "ra_fused_first",
            "ra_fused_last", "sn_fused", "sn_fused_first", "sn_fused_last", "ss_fused")


@pytest.mark.parametrize("variant,tune,family", [
    ("RA", None, "ra_zsweep"), ("SN", None, "sn_zsweep"), ("SS", None, "ss_zsweep"),
    ("RS", None, "rs_zsweep"), ("RA", {"fuse": 1}, "ra_fused"), ("SN", {"fuse": 1}, "sn_fused"),
    ("SS", {"fuse": 1}, "ss_fused")])
def test_each_algorithm_runs_its_own_kernel(variant, tune, family):
    # RA, SN, RS and SS are separate kernels: two RK steps of each launch six
    # kernels of its own family (the fused SN and RA stages: first substep,
    # middle, third without and with the q_acc store) and none of the others'
    shape = (40, 36, 50)
    s = nsf.Solver(shape, PHYS, variant, "f64", tune=tune)
    s.init(W.tgv_pointwise(3, 1e-3))
    counts = {}
    for fam in FAMILIES:
        nsf.timer_enable(fam)
        s.step(1e-3, 2)
        torch.cuda.synchronize()
        counts[fam], _ = nsf.timer_read()
        nsf.timer_enable(None)
    own = {f: c for f, c in counts.items() if f.startswith(family)}
    assert sum(own.values()) == 6, counts
    assert all(c == 0 for f, c in counts.items() if f not in own), counts
    if tune and variant != "SS":  # fused double precision: 2 first, 2 middle + 1 final third, 1 third
        assert (own[family + "_first"], own[family], own[family + "_last"]) == (2, 3, 1), own


@pytest.mark.parametrize("variant", ["SN", "RS", "RA"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (40, 36, 50), (70, 11, 9), (5, 6, 7)])
@pytest.mark.parametrize("tune", [None, {"block_y": 16, "zchunk": 5}, {"block_y": 8, "zchunk": 7}])
def test_sn_rs_ra_parity(variant, shape, tune):
    print(f"case parity {variant} {shape} {tune}", flush=True)
    q = O.init(shape, PHYS, W.tgv_pointwise(3, 1e-3), prec="ld")
    ref = O.rhs(q, PHYS, prec="ld")
    s = nsf.Solver(shape, PHYS, variant, "f64", tune=tune)
    s.q.copy_(torch.from_numpy(q.astype(np.float64)))
    s.rhs()
    err = rel_err(s.r.cpu().numpy(), ref)
    floor = rel_err(O.rhs(q.astype(np.float64), PHYS, prec="d"), ref)
    assert np.all(err <= np.maximum(1e-12, 4 * floor)), err


@pytest.mark.parametrize("variant", ["SS", "RS"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(16, 16, 16), (40, 36, 50), (70, 11, 9), (5, 6, 7)])
@pytest.mark.parametrize("tune", [{"gstore": 3}, {"gstore": 3, "block_y": 8, "zchunk": 7},
                                  {"gstore": 9, "block_y": 16, "zchunk": 5}])
def test_store_set_parity(variant, precision, shape, tune):
    # the stored-gradient algorithms with the diagonal store set (the other
    # six gradients formed in the kernel) and the full set
    print(f"case store set {variant} {precision} {shape} {tune}", flush=True)
    q = O.init(shape, PHYS, W.tgv_pointwise(3, 1e-3), prec="ld")
    qin = q.astype(np.float64 if precision == "f64" else np.float32)
    ref = O.rhs(qin.astype(np.longdouble), PHYS, prec="ld")
    s = nsf.Solver(shape, PHYS, variant, precision, tune=tune)
    s.q.copy_(torch.from_numpy(qin))
    s.rhs()
    err = rel_err(s.r.cpu().numpy().astype(np.float64), ref)
    if precision == "f64":
        bar = np.maximum(1e-12, 4 * rel_err(O.rhs(q.astype(np.float64), PHYS, prec="d"), ref))
    else:
        bar = 4 * rel_err(ref, O.rhs(q, PHYS, prec="ld"))
    assert np.all(err <= bar), (err, bar)


def test_recompute_and_thread_local_forms_round_differently():
    # RA and SN (and RS and SS) form the same derivatives in different
    # orders, so their residuals agree to round-off but not bit for bit
    shape = (40, 36, 50)
    q = O.init(shape, PHYS, W.tgv_pointwise(3, 1e-3), prec="d")
    out = {}
    for v in ("RA", "SN", "RS", "SS"):
        s = nsf.Solver(shape, PHYS, v, "f64")
        s.q.copy_(torch.from_numpy(q))
        s.rhs()
        out[v] = s.r.clone()
    assert not torch.equal(out["RA"], out["SN"])
    assert not torch.equal(out["RS"], out["SS"])
    ref = O.rhs(q.astype(np.longdouble), PHYS, prec="ld")
    bar = np.maximum(1e-12, 8 * rel_err(O.rhs(q, PHYS, prec="d"), ref))
    assert np.all(rel_err(out["RA"].cpu().numpy(), out["SN"].cpu().numpy()) <= bar)
    assert np.all(rel_err(out["RS"].cpu().numpy(), out["SS"].cpu().numpy()) <= bar)


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
