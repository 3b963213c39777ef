"""Seeded synthetic workloads: the Taylor-Green runs of the paper's
Section 3 and the batched ensemble, as plain parameter sets.

This module holds no arithmetic of the method (no stencil, residual or
time update); it only describes inputs, so both the GPU tests and the CPU
oracle can be driven from the same recipe. It imports neither the GPU
binding nor the oracle.
"""
from __future__ import annotations

import math

import numpy as np

# Section 3: Ma = 0.1, Pr = 0.71, Re = 1600; gamma = 1.4 (air)
TGV_PHYS = {"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4}

# Section 3: dt = 3.385e-3 on 64^3, halved for every 2^3 increase in points.
DT_64 = 3.385e-3


def tgv_dt(n: int) -> float:
    """Time step of the paper's Taylor-Green runs for an n^3 grid; the 32^3
    case keeps the 64^3 step (it is then half the 64^3 CFL number)."""
    return DT_64 if n <= 64 else DT_64 * 64.0 / n


def tgv_unperturbed() -> dict:
    return {"V0": 1.0, "pert_kind": 0, "pert_amp": 0.0, "seed": 0}


def tgv_pointwise(seed: int = 1610, amp: float = 1e-3) -> dict:
    """Pointwise multiplicative velocity noise, U[-amp, amp), SplitMix64."""
    return {"V0": 1.0, "pert_kind": 1, "pert_amp": amp, "seed": seed}


def tgv_random_phase(phase, amp: float = 1e-2) -> dict:
    """Divergence-free Taylor-Green-shaped mode with shifted phases."""
    return {"V0": 1.0, "pert_kind": 2, "pert_amp": amp, "phase": tuple(float(p) for p in phase)}


# The five measured configurations (grid, steps, algorithms, precision).
CONFIGS = [
    {"name": "tgv32_f64_bl", "n": 32, "steps": 10, "variants": ["BL"], "precision": "f64",
     "tgv": tgv_unperturbed()},
    {"name": "tgv256_f64", "n": 256, "steps": 100, "variants": ["BL", "RA", "SS"],
     "precision": "f64", "tgv": tgv_pointwise(1610)},
    {"name": "tgv512_f64", "n": 512, "steps": 50, "variants": ["best", "BL"], "precision": "f64",
     "tgv": tgv_unperturbed(), "diag_every": 1},
    {"name": "tgv512_f32", "n": 512, "steps": 100, "variants": ["best"], "precision": "f32",
     "tgv": tgv_unperturbed(), "diag_every": 1},
    {"name": "batch64", "count": 64, "seed": 9146, "precision": ["f64", "f32"]},
]


def batch_dt(n: int, Ma: float) -> float:
    """Batched-instance time step: the paper's acoustic CFL number at every
    (n, Ma): dt scales with h and with 1/(1 + sqrt(3)/Ma) relative to the
    Ma = 0.1, 64^3 run."""
    return DT_64 * (64.0 / n) * (1.0 + math.sqrt(3.0) / 0.1) / (1.0 + math.sqrt(3.0) / Ma)


def batch_instances(count: int = 64, seed: int = 9146, sizes=(32, 48, 64, 96, 128)) -> list[dict]:
    """Ensemble of independent Taylor-Green instances with uneven grids:
    n ~ U(sizes), Re ~ U[400, 3200], Ma ~ U[0.05, 0.2], phases ~ U[0, 2 pi)^3,
    random-phase velocity perturbation of amplitude 1e-2 (numpy PCG64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        Re = float(rng.uniform(400.0, 3200.0))
        Ma = float(rng.uniform(0.05, 0.2))
        phase = tuple(float(x) for x in rng.uniform(0.0, 2 * math.pi, size=3))
        out.append({
            "shape": (n, n, n),
            "phys": {"Re": Re, "Ma": Ma, "Pr": 0.71, "gamma": 1.4},
            "tgv": tgv_random_phase(phase, 1e-2),
            "dt": batch_dt(n, Ma),
        })
    return out
