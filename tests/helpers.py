"""Shared helpers of the test suite (comparison metrics, slab oracle)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def rel_err(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Per-field max-norm error of a against reference b, relative to the
    reference field's max norm: ||a_f - b_f||_inf / ||b_f||_inf."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, dtype=np.float64).reshape(b.shape[0], -1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return np.abs(a - b).max(axis=1) / den


def slab_rhs(q_slab: np.ndarray, nz_glob: int, phys, prec: str) -> np.ndarray:
    """Oracle residual on the interior planes of a z-slab.

    q_slab holds planes k0-2 .. k1+1 of a periodic nz_glob-plane state
    (full x and y extents); the residual of planes k0 .. k1-1 depends on
    those planes only, so it equals what the full-grid oracle gives.
    """
    return O.rhs_slab(q_slab, nz_glob, phys, prec=prec)


def take_planes(a: np.ndarray, k0: int, k1: int) -> np.ndarray:
    """Planes k0..k1-1 (wrapping periodically) of a [5, nz, ny, nx] array."""
    nz = a.shape[1]
    idx = [(k % nz) for k in range(k0, k1)]
    return a[:, idx]
