#!/usr/bin/env python3
"""Throughput benchmark of the Navier-Stokes RHS + low-storage RK3 hot path.

Workload (default): the paper's Taylor-Green vortex (Section 3) on a 512^3
periodic grid in double precision, Re=1600, Ma=0.1, Pr=0.71, dt=4.23125e-4,
with the kinetic-energy and enstrophy integrals reduced every step in FP64.
One timed step = one three-stage RK step (3 residual evaluations + stage
updates) + the diagnostics. The metric is grid-point RHS evaluations per
second: n^3 * 3 * steps / time, with all state resident in HBM.

Beside the main line it reports the roofline of the dominant kernel (HIP
events on its launch stream), the other algorithms and the FP32 form at the
same size, and the CPU oracle timed on a bounded slab of the same grid.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point RHS evals/s and % HBM roofline at 512^3 FP64; FP32/batched vs FP64"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

# Algorithmic HBM bytes per grid point per launch of each kernel family,
# as (bytes with FP64 fields, bytes with FP32 fields): every input field
# read once, every output field written once; stencil neighbours are
# on-chip reuse. The RK accumulator is FP64 in both precisions.
FAMILY_BYTES = {
    "prims": (80, 40),            # q -> u, v, w, p, T
    "update": (160, 120),         # r, q_acc -> q, q_acc
    "ra_naive": (120, 60),        # q, prims -> r (untiled, RA and SN)
    "ra_zsweep": (120, 60),       # RA: q, prims -> r
    "sn_zsweep": (120, 60),       # SN: q, prims -> r
    # fused stages. Double precision: the first substep reads the
    # accumulator from q (equal at a step boundary) and stores none: q ->
    # q_next; the second forms that accumulator from the step's initial state
    # and reads it in place of q_acc (160 B as before); a third substep other
    # than a call's last leaves q_acc unwritten: q, q_acc -> q_next
    "ra_fused": (160, 120),       # RA: q, q_acc -> q_next, q_acc
    "ra_fused_mon": (80, 120),    # RA first substep, plus per-tile KE / enstrophy sums
    "ra_fused_first": (80, 120),  # RA first substep, unmonitored
    "ra_fused_last": (120, 120),  # RA third substep without the q_acc store
    "sn_fused": (160, 120),       # SN: q, q_acc -> q_next, q_acc
    "sn_fused_mon": (80, 120),    # SN first substep, plus per-tile KE / enstrophy sums
    "sn_fused_first": (80, 120),  # SN first substep, unmonitored
    "sn_fused_last": (120, 120),  # SN third substep without the q_acc store
    "rs_zsweep": (192, 96),       # RS: q, prims, 9 gradients -> r
    "ss_grad_naive": (96, 48),    # u, v, w -> 9 gradients
    "ss_naive": (192, 96),        # q, prims, 9 gradients -> r
    "ss_prims_grad": (152, 76),   # q -> u, v, w, p, T and 9 gradients (one pass)
    "ss_zsweep": (192, 96),       # q, prims, 9 gradients -> r
    "ss_fused": (272, 176),       # fused SS: q, prims, 9 gradients, q_acc -> q_next, q_acc
    "bl_deriv": (16, 8),          # one field -> one derivative
    "bl_product": (24, 12),       # two fields -> one product
    "bl_assemble": (584, 292),    # 60 derivatives, q, u -> r
    "diag": (40, 20),             # q -> 16 scalars
}

# Counter-measured HBM traffic per launch lives in a committed summary under
# profiles/, stamped with a digest of the kernel sources it was taken with;
# it is reported only while those sources are unchanged.
TRAFFIC_SOURCES = ["paper_1610_09146_amd/csrc/nsf_zsweep.hip",
                   "paper_1610_09146_amd/csrc/nsf_device.h",
                   "paper_1610_09146_amd/csrc/nsf_internal.h"]


def source_digest(paths=TRAFFIC_SOURCES) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel_tag: str):
    """traffic_bytes_per_launch from profiles/*counters*.md for `kernel_tag`
    (e.g. 'ra_fused f64 32x16'), or None when absent or stale."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    digest = source_digest()
    for name in sorted(os.listdir(pdir)):
        if "counters" not in name:
            continue
        text = open(os.path.join(pdir, name)).read()
        for block in re.findall(r"```traffic\n(.*?)```", text, flags=re.S):
            kv = dict(re.findall(r"^(\w+):\s*(.+?)\s*$", block, flags=re.M))
            if kv.get("kernel") == kernel_tag and kv.get("source_sha256") == digest:
                return float(kv["traffic_bytes_per_launch"])
    return None


def families(variant, tune):
    if variant == "BL":
        return ["prims", "bl_product", "bl_deriv", "bl_assemble", "update", "diag"]
    if variant in ("RA", "SN"):
        k = variant.lower()
        if tune and tune.get("fuse"):
            return [f"{k}_fused", f"{k}_fused_mon", f"{k}_fused_last"]
        if tune and tune.get("naive"):
            return ["prims", "ra_naive", "update", "diag"]
        return ["prims", f"{k}_zsweep", "update", "diag"]
    if tune and tune.get("naive"):
        return ["prims", "ss_grad_naive", "ss_naive", "update", "diag"]
    if variant == "SS" and tune and tune.get("fuse"):
        return ["ss_prims_grad", "ss_fused", "diag"]
    return ["ss_prims_grad", "rs_zsweep" if variant == "RS" else "ss_zsweep", "update", "diag"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_variant(nsf, torch, W, n, variant, precision, steps, warmup, time_families=True,
                tune=None, tgv=None):
    """Time `steps` RK steps of one configuration, the kinetic energy and
    enstrophy reduced on the device every step (nsf_rk_step_monitored), with
    no host synchronisation inside the timed region."""
    shape = (n, n, n)
    phys = W.TGV_PHYS
    dt = W.tgv_dt(n)
    s = nsf.Solver(shape, phys, variant, precision, tune=tune)
    s.init(tgv or W.tgv_unperturbed())
    mon = torch.zeros(2 * max(steps, 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    # warmup; also find the family with the largest summed kernel time, in
    # untimed calls of the same form as the timed one (a few steps each)
    fam_ms, fam_n = {}, {}
    fams = families(variant, tune)
    for w in range(max(warmup, 1)):
        s.step_monitored(dt, 1, mon)
    s.diagnostics()  # raises on non-finite values
    if time_families:
        k = min(steps, 5)
        for fam in fams:
            nsf.timer_enable(fam)
            s.step_monitored(dt, k, mon)
            torch.cuda.synchronize()
            c, ms = nsf.timer_read()
            fam_ms[fam], fam_n[fam] = ms / k, c / k
        nsf.timer_enable(None)
    dominant = max(fam_ms, key=fam_ms.get) if fam_ms else None
    # per-launch time of the dominant family (roofline): HIP events around
    # each of its launches, in an untimed pass of the same number of steps
    kcount, kms = 0, 0.0
    if dominant:
        nsf.timer_enable(dominant)
        s.step_monitored(dt, steps, mon)
        torch.cuda.synchronize()
        kcount, kms = nsf.timer_read()
        nsf.timer_enable(None)
    # the timed region: no per-launch timer
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step_monitored(dt, steps, mon)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    monitor = mon.cpu().numpy().reshape(-1, 2)[:steps]
    diag = s.diagnostics()  # the final state, outside the timed region
    ms_per_step = (t1 - t0) * 1e3 / steps
    rate = n ** 3 * 3 * steps / (t1 - t0)
    out = {
        "variant": variant, "precision": precision, "n": n, "steps": steps, "tune": tune,
        "ms_per_step": ms_per_step, "pt_rhs_per_s": rate, "dominant": dominant,
        "dominant_launches": kcount, "dominant_ms_total": kms,
        "family_ms_one_step": fam_ms, "family_launches_one_step": fam_n,
        "ke": float(diag[0]),
        "enstrophy": float(diag[1]),
        "monitor_first": [float(x) for x in monitor[0]],
        "monitor_last": [float(x) for x in monitor[-1]],
    }
    del s
    torch.cuda.empty_cache()
    return out


def run_batch(nsf, torch, W, precision, steps, warmup=1):
    """64 uneven Taylor-Green instances, each step one graph replay (three
    persistent stage launches)."""
    insts = W.batch_instances()
    # the batched form's own autotuner: stage algorithm (SN / RA), tile
    # height and z-chunk, searched on the ensemble
    pick = nsf.batch_autotune(insts, precision, steps=3)
    b = nsf.Batch(insts, precision, variant=pick["variant"], tune=pick["tune"])
    pts = b.points()
    for _ in range(warmup):
        b.step(1)
    nsf.timer_enable("batch_step")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c, ms = nsf.timer_read()
    nsf.timer_enable(None)
    d = b.diagnostics()
    nitems, nblocks = b.info()
    # algorithmic bytes per point and step of the batched stages: in double
    # precision with 16-row tiles the first substep reads the accumulator
    # from q and stores none, and the third leaves it unwritten (but in a
    # call's last step)
    cfg = b.config()
    if precision == "f64" and cfg["tile_y"] == 16:
        per_pt = (FAMILY_BYTES["sn_fused_first"][0] + FAMILY_BYTES["sn_fused"][0]
                  + FAMILY_BYTES["sn_fused_last"][0])
    else:
        per_pt = FAMILY_BYTES["sn_fused"][0 if precision == "f64" else 1] * 3
    avg_s = ms / max(c, 1) / 1e3
    out = {
        "instances": len(insts), "points": pts, "precision": precision, "steps": steps,
        "ms_per_step": (t1 - t0) * 1e3 / steps,
        "pt_rhs_per_s": pts * 3 * steps / (t1 - t0),
        "work_items": nitems, "persistent_blocks": nblocks,
        "batch_autotune": pick, "batch_config": b.config(),
        "roofline": {"bound": "hbm", "kernel": "ra_batch (3 stage launches per graph replay)",
                     "achieved": round(per_pt * pts / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(per_pt * pts / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "avg_graph_ms": round(avg_s * 1e3, 4)},
        "ke_min_max": [float(d[:, 0].min()), float(d[:, 0].max())],
    }
    b.close()
    del b
    torch.cuda.empty_cache()
    # the same ensemble advanced by the plain single-grid FP64/FP32 path, one
    # instance after another (fused SN, one rk_step call per instance)
    solvers = []
    for inst in insts:
        sv = nsf.Solver(inst["shape"], inst["phys"], "SN", precision, tune={"fuse": 1})
        sv.init(inst["tgv"])
        sv.step(inst["dt"], 1)
        solvers.append(sv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for sv, inst in zip(solvers, insts):
            sv.step(inst["dt"], 1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out["sequential_single_pt_rhs_per_s"] = pts * 3 * steps / (t1 - t0)
    del solvers
    torch.cuda.empty_cache()
    return out


def precision_errors(nsf, torch, W, n, steps, tuned):
    """FP32 form against the parity-checked FP64 GPU run (proxy for the FP64
    oracle at this size) after `steps` steps: relative errors of KE,
    enstrophy, the KE change over the run, and per-field max-norms."""
    out = {}
    for prec in ("f64", "f32"):
        var = tuned[prec]["variant"] if tuned else "SN"
        tune = tuned[prec]["tune"] if tuned else {"fuse": 1}
        s = nsf.Solver((n, n, n), W.TGV_PHYS, var, prec, tune=tune)
        s.init(W.tgv_unperturbed())
        s.step(W.tgv_dt(n), steps)
        d = s.diagnostics()
        out[prec] = (d, s.q_acc.abs().amax(dim=(1, 2, 3)).cpu().numpy(),
                     s.q_acc.clone() if prec == "f64" else s.q_acc)
        if prec == "f32":
            diff = (s.q_acc - out["f64"][2]).abs().amax(dim=(1, 2, 3)).cpu().numpy()
        del s
    d64, d32 = out["f64"][0], out["f32"][0]
    del out
    torch.cuda.empty_cache()
    return {"n": n, "steps": steps, "reference": "FP64 GPU run (parity-checked path)",
            "ke_rel_err": abs(d32[0] - d64[0]) / abs(d64[0]),
            "enstrophy_rel_err": abs(d32[1] - d64[1]) / abs(d64[1]),
            "dke_rel_err": abs((d32[0] - 0.125) - (d64[0] - 0.125)) / abs(d64[0] - 0.125),
            "maxnorm_rel_err": [float(x) for x in diff / out_max(d64)],
            "ke_f64": float(d64[0]), "ke_f32": float(d32[0])}


def out_max(d):
    """Per-field max norms from a diagnostics vector."""
    import numpy as np
    return np.asarray(d[7:12])


def batch_precision_errors(nsf, torch, W, steps):
    """Batched FP32 form against the batched FP64 form, per instance, after
    `steps` steps: largest relative KE error over the 64 instances."""
    import numpy as np
    insts = W.batch_instances()
    ke = {}
    for prec in ("f64", "f32"):
        b = nsf.Batch(insts, prec)
        b.step(steps)
        ke[prec] = b.diagnostics()[:, 0]
        b.close()
        del b
        torch.cuda.empty_cache()
    rel = np.abs(ke["f32"] - ke["f64"]) / np.abs(ke["f64"])
    return {"steps": steps, "instances": len(insts), "ke_rel_err_max": float(rel.max()),
            "ke_rel_err_median": float(np.median(rel))}


# Bandwidth of the library's streaming copy on 4 GiB, measured at start-up
# (the achievable HBM rate next to the vendor peak).
COPY_PEAK = {}


def copy_peak(nsf, torch, gib=4, reps=5):
    """Read + write bytes / time of nsf_device_copy over `gib` GiB, best of
    `reps` launches, HIP events on the launch stream."""
    n = gib << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    nsf.device_copy(src, dst)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        nsf.device_copy(src, dst)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": round(2 * n * 8 / best / 1e6, 1), "ms": round(best, 4),
            "kernel": f"k_copy16 (nsf_device_copy), {gib} GiB read + {gib} GiB written, best of {reps}"}


def stage_roofline(res, precision):
    """Algorithmic bytes over kernel time of all the kernels of one step
    (every timed family), per step: the whole step's HBM roofline."""
    col = 0 if precision == "f64" else 1
    ms = sum(res["family_ms_one_step"].values())
    if not ms:
        return None
    byts = sum(FAMILY_BYTES[f][col] * res["family_launches_one_step"][f] * res["n"] ** 3
               for f in res["family_ms_one_step"])
    return {"algorithmic_bytes_per_step": byts, "kernel_ms_per_step": round(ms, 4),
            "achieved_GBps": round(byts / ms / 1e6, 1),
            "frac": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4)}


def roofline_of(res, precision):
    fam = res["dominant"]
    if not fam or res["dominant_launches"] == 0:
        return None
    per_pt = FAMILY_BYTES[fam][0 if precision == "f64" else 1]
    avg_s = res["dominant_ms_total"] / res["dominant_launches"] / 1e3
    alg_bytes = per_pt * res["n"] ** 3
    achieved = alg_bytes / avg_s / 1e9
    tune = res.get("tune") or {}
    tag = f"{fam} {precision} 32x{tune.get('block_y', 0)} zchunk{tune.get('zchunk', 0)} n{res['n']}"
    return {"bound": "hbm", "kernel": fam, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(tag), "traffic_key": tag,
            "algorithmic_bytes_per_launch": alg_bytes,
            "avg_launch_ms": round(avg_s * 1e3, 4),
            "copy_peak_GBps": COPY_PEAK.get("GBps"),
            "frac_of_copy": round(achieved / COPY_PEAK["GBps"], 4) if COPY_PEAK else None}


def cpu_sizes(W):
    """The oracle on whole small grids: one residual and one RK step at 64^3
    and 128^3 with one thread and with every host thread, and one residual
    at 256^3 with every host thread (pt-RHS/s)."""
    from oracle import oracle as O
    phys = W.TGV_PHYS
    all_threads = O.get_threads()
    rows = []
    for n, threads, what in ((64, 1, "rhs"), (64, 1, "rk_step"), (64, all_threads, "rhs"),
                             (64, all_threads, "rk_step"), (128, 1, "rhs"),
                             (128, 1, "rk_step"), (128, all_threads, "rhs"),
                             (128, all_threads, "rk_step"), (256, all_threads, "rhs")):
        q = O.init((n, n, n), phys, W.tgv_pointwise(1610, 1e-3))
        O.set_threads(threads)
        t0 = time.perf_counter()
        if what == "rhs":
            O.rhs(q, phys)
            evals = n ** 3
        else:
            O.rk_step(q, phys, W.tgv_dt(n), 1)
            evals = 3 * n ** 3
        dt_s = time.perf_counter() - t0
        rows.append({"n": n, "call": what, "threads": threads, "seconds": round(dt_s, 3),
                     "pt_rhs_per_s": evals / dt_s})
    O.set_threads(all_threads)
    return rows


def cpu_host():
    """Host CPU model name and logical core count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(W, budget_s=12.0, n=512, planes_per_call=8):
    """Oracle (plain C, FP64) residual on consecutive z-slabs of the same
    512^3 Taylor-Green grid until about budget_s seconds have elapsed."""
    from oracle import oracle as O
    phys, tgv = W.TGV_PHYS, W.tgv_unperturbed()
    threads = O.get_threads()
    done_pts, spent, k0 = 0, 0.0, 0
    while spent < budget_s and k0 < n:
        qs = O.init_slab((n, n, n), k0 - 2, planes_per_call + 4, phys, tgv)
        t0 = time.perf_counter()
        O.rhs_slab(qs, n, phys)
        spent += time.perf_counter() - t0
        done_pts += planes_per_call * n * n
        k0 += planes_per_call
    return {"value": done_pts / spent, "unit": "pt-RHS/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle residual of z-planes 0..{k0 - 1} of the {n}^3 Taylor-Green "
                      f"grid ({done_pts} point-RHS in {spent:.1f} s, {threads} threads)",
            "host": cpu_host(), "sizes": cpu_sizes(W)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--variant", default="AUTO",
                    help="AUTO = the autotuner's pick for this grid (default), or BL/RA/SS/SN/RS")
    ap.add_argument("--fuse", type=int, default=1, help="RA/SN/SS: fused stage kernel (1) or not (0)")
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"],
                    help="precision of the main line (the metric is quoted for f64)")
    ap.add_argument("--block-y", type=int, default=0, help="tile height 8/16 (explicit variant)")
    ap.add_argument("--zchunk", type=int, default=0, help="planes per tile (explicit variant)")
    ap.add_argument("--no-extras", action="store_true", help="skip BL/SS/FP32 side measurements")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy three times (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the domain-decomposed form is a design note only); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_1610_09146_amd import nsf, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    nsf.lib()  # fail loudly if the HIP library is missing
    COPY_PEAK.update(copy_peak(nsf, torch))
    log(f"copy peak: {COPY_PEAK['GBps']} GB/s")
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            nsf.device_copy(src, dst)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB")
        del src, dst
    n = args.n
    tuned = {}
    if args.variant == "AUTO":
        for prec in ("f64", "f32"):
            log(f"autotune {n}^3 {prec}")
            tuned[prec] = nsf.autotune((n, n, n), W.TGV_PHYS, prec, quick=True, steps=3)
            log(f"  -> {tuned[prec]}")
        main_variant, main_tune = tuned[args.precision]["variant"], tuned[args.precision]["tune"]
    else:
        main_variant = args.variant
        main_tune = {"fuse": args.fuse if args.variant in ("RA", "SN", "SS") else 0,
                     "block_y": args.block_y, "zchunk": args.zchunk}
    log(f"main: {main_variant} {main_tune} {args.precision} n={n} steps={args.steps}")
    main_res = run_variant(nsf, torch, W, n, main_variant, args.precision, args.steps, args.warmup,
                           tune=main_tune)
    log(f"main done: {main_res['pt_rhs_per_s']:.3e} pt-RHS/s")
    extras = {}
    if not args.no_extras:
        for name, v, prec, k, tune in (("BL_f64", "BL", "f64", 3, None),
                                       ("SS_f64", "SS", "f64", 5, None),
                                       ("SS_f64_fused", "SS", "f64", 5, {"fuse": 1}),
                                       ("RS_f64", "RS", "f64", 5, None),
                                       ("SN_f64_stored_prims", "SN", "f64", 5, None),
                                       ("RA_f64_stored_prims", "RA", "f64", 5, None),
                                       ("RA_f64_fused", "RA", "f64", 5, {"fuse": 1}),
                                       ("SN_f32_fused", "SN", "f32", 10, {"fuse": 1})) + (
                (("f32_autotuned", tuned["f32"]["variant"], "f32", 10, tuned["f32"]["tune"]),)
                if tuned else ()):
            log(f"extra: {name}")
            r = run_variant(nsf, torch, W, n, v, prec, k, 1, tune=tune)
            r["roofline"] = roofline_of(r, prec)
            extras[name] = r
        # the paper's Table 1 on one MI355X: the five algorithms in the
        # paper's form (stored primitives, separate update) and the fused SS, RA
        # and SN, FP64, at 64^3, 128^3 and 256^3, pointwise +-1e-3
        # perturbation (seed 1610), 100 steps
        table = []
        for nt in (64, 128, 256):
            for name, v, tune in (("BL", "BL", None), ("RA", "RA", None), ("RS", "RS", None),
                                  ("SN", "SN", None), ("SS", "SS", None),
                                  ("RA_fused", "RA", {"fuse": 1}), ("SN_fused", "SN", {"fuse": 1}),
                                  ("SS_fused", "SS", {"fuse": 1})):
                log(f"extra: {nt}^3 {name}")
                r = run_variant(nsf, torch, W, nt, v, "f64", 100, 1, tune=tune,
                                tgv=W.tgv_pointwise(1610, 1e-3))
                rl = roofline_of(r, "f64")
                sr = stage_roofline(r, "f64")
                table.append({"n": nt, "algorithm": name, "ms_per_step": round(r["ms_per_step"], 4),
                              "pt_rhs_per_s": r["pt_rhs_per_s"], "dominant": r["dominant"],
                              "dominant_frac_of_8TBs": rl["frac"] if rl else None,
                              "step_frac_of_8TBs": sr["frac"] if sr else None,
                              "family_ms_one_step": r["family_ms_one_step"]})
        extras["table1_f64"] = table
        # the largest single-GPU grid, 1024^3 (about 215 GB), when it fits
        torch.cuda.empty_cache()
        need = nsf.workspace_bytes((1024,) * 3, "SN", "f64", {"fuse": 1}) + 15 * 1024 ** 3 * 8
        if torch.cuda.mem_get_info()[0] > need + (2 << 30):
            log("extra: 1024^3 SN fused f64")
            r = run_variant(nsf, torch, W, 1024, "SN", "f64", 3, 1, tune={"fuse": 1})
            r["roofline"] = roofline_of(r, "f64")
            extras["n1024_SN_fused_f64"] = r
        for prec in ("f64", "f32"):
            log(f"extra: batch64 {prec}")
            extras[f"batch64_{prec}"] = run_batch(nsf, torch, W, prec, 10)
        log("extra: FP32-form errors after 100 steps (512^3 and batch)")
        extras["f32_errors_512_100steps"] = precision_errors(nsf, torch, W, n, 100, tuned)
        extras["f32_errors_batch64_100steps"] = batch_precision_errors(nsf, torch, W, 100)
    line = {
        "metric": METRIC,
        "value": main_res["pt_rhs_per_s"],
        "unit": "pt-RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"taylor-green {n}^3 {args.precision.upper()}, Re=1600 Ma=0.1 Pr=0.71, "
                               f"dt={W.tgv_dt(n)}, KE+enstrophy every step",
                   "variant": main_variant, "tune": main_tune, "selected_by": args.variant,
                   "n": n, "dt": W.tgv_dt(n), "diag_every": 1,
                   "diag": "KE and enstrophy reduced on the GPU every step, no host sync"},
        "autotune": tuned,
        "copy_peak": COPY_PEAK,
        "roofline": roofline_of(main_res, args.precision),
        "step_roofline": stage_roofline(main_res, args.precision),
        "main": main_res,
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(W)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
