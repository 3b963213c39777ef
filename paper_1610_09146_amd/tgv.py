"""Long Taylor-Green evolution (paper Section 3): kinetic energy and
enstrophy every step, recorded on the device by nsf_rk_step_monitored.

    python -m paper_1610_09146_amd.tgv --n 256 --t-end 20 --out tgv256.json

The time step is the paper's (3.385e-3 on 64^3, halved for every 2^3
increase in points). Besides the two integrals the record holds the
dissipation rate -dKE/dt (second-order central difference of the per-step
KE) and, for comparison, 2 * enstrophy / Re, which it approaches in the
incompressible limit (the enstrophy here is the density-weighted
<rho |omega|^2 / 2>). Every `chunk` steps the full diagnostics run once
(non-finite values stop the run).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import nsf, workloads as W


def run(n: int, t_end: float, precision: str = "f64", variant="SN", tune: dict | None = None,
        phys: dict | None = None, tgv: dict | None = None, chunk: int = 2000,
        log=None) -> dict:
    """Evolve the n^3 Taylor-Green vortex to t_end; returns the record
    (numpy arrays t, ke, enstrophy, dissipation; conservation sums)."""
    phys = phys or W.TGV_PHYS
    tune = tune if tune is not None else ({"fuse": 1} if variant in ("RA", "SN") else None)
    dt = W.tgv_dt(n)
    nsteps = int(math.ceil(t_end / dt - 1e-9))
    s = nsf.Solver((n, n, n), phys, variant, precision, tune=tune)
    s.init(tgv or W.tgv_unperturbed())
    d0 = s.diagnostics()
    mon = torch.empty(2 * min(chunk, max(nsteps, 1)), dtype=torch.float64, device=s.q.device)
    ke, ens, sums = [], [], []
    done = 0
    t0 = time.perf_counter()
    while done < nsteps:
        k = min(chunk, nsteps - done)
        s.step_monitored(dt, k, mon)
        m = mon[: 2 * k].cpu().numpy().reshape(k, 2)  # synchronises
        ke.append(m[:, 0])
        ens.append(m[:, 1])
        d = s.diagnostics()  # raises on non-finite values
        sums.append(d[2:7].copy())
        done += k
        if log:
            log(f"n={n} step {done}/{nsteps} t={done * dt:.3f} KE={d[0]:.6e} enstrophy={d[1]:.6e}")
    wall = time.perf_counter() - t0
    d_end = s.diagnostics()
    # the monitor holds the state at the start of each step; append the end
    ke = np.concatenate(ke + [[d_end[0]]])
    ens = np.concatenate(ens + [[d_end[1]]])
    t = dt * np.arange(nsteps + 1)
    diss = np.full_like(ke, np.nan)
    diss[1:-1] = -(ke[2:] - ke[:-2]) / (2 * dt)
    return {"n": n, "precision": precision, "variant": variant, "tune": tune, "phys": phys,
            "dt": dt, "steps": nsteps, "t": t, "ke": ke, "enstrophy": ens, "dissipation": diss,
            "two_enstrophy_over_Re": 2 * ens / phys["Re"],
            "sums_initial": d0[2:7], "sums_final": d_end[2:7], "wall_s": wall,
            "pt_rhs_per_s": n ** 3 * 3 * nsteps / wall}


def summary(rec: dict) -> dict:
    """Peak dissipation and peak enstrophy (value and time) of a record."""
    diss, ens, t = rec["dissipation"], rec["enstrophy"], rec["t"]
    i = int(np.nanargmax(diss))
    j = int(np.argmax(ens))
    return {"n": rec["n"], "t_end": float(t[-1]), "ke_end": float(rec["ke"][-1]),
            "peak_dissipation": float(diss[i]), "t_peak_dissipation": float(t[i]),
            "peak_enstrophy": float(ens[j]), "t_peak_enstrophy": float(t[j]),
            "mass_drift": float(abs(rec["sums_final"][0] - rec["sums_initial"][0])),
            "pt_rhs_per_s": rec["pt_rhs_per_s"]}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, nargs="+", default=[64])
    ap.add_argument("--t-end", type=float, default=20.0)
    ap.add_argument("--precision", default="f64", choices=["f64", "f32"])
    ap.add_argument("--variant", default="SN")
    ap.add_argument("--every", type=int, default=10, help="keep every k-th sample in the output")
    ap.add_argument("--out", default=None, help="JSON file for the records")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("tgv.py needs a GPU", file=sys.stderr)
        return 2
    out = {"runs": []}
    for n in args.n:
        rec = run(n, args.t_end, args.precision, args.variant,
                  log=lambda m: print(m, file=sys.stderr, flush=True))
        summ = summary(rec)
        print(json.dumps(summ), flush=True)
        sl = slice(None, None, max(1, args.every))
        out["runs"].append({"summary": summ, "t": rec["t"][sl].tolist(), "ke": rec["ke"][sl].tolist(),
                            "enstrophy": rec["enstrophy"][sl].tolist(),
                            "dissipation": [None if not np.isfinite(x) else float(x)
                                            for x in rec["dissipation"][sl]]})
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
