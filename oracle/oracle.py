"""ctypes front end of the CPU oracle (plain C, ``nsf_oracle.c``).

TEST INFRASTRUCTURE ONLY. The oracle is the slow, obviously-correct CPU
statement of the method of Jammy, Jacobs & Sandham (arXiv 1610.09146,
Sections 2-3) that the GPU library is checked against. Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this module. It imports nothing from the GPU package.

Arrays are numpy, field-major ``[5][nz][ny][nx]`` (x fastest). ``prec``
selects the C instantiation: ``"d"`` (float64) or ``"ld"`` (x87 extended,
``numpy.longdouble``), the latter giving the round-off floor.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NDIAG = 16
DIAG_NAMES = [
    "ke", "enstrophy", "mean_rho", "mean_rhou", "mean_rhov", "mean_rhow", "mean_rhoE",
    "max_rho", "max_rhou", "max_rhov", "max_rhow", "max_rhoE", "min_rho", "min_p",
    "nonfinite", "mean_p",
]

# Low-storage RK3 coefficients (reading of Section 2; the paper names none).
RK_A = (2.0 / 3.0, 5.0 / 12.0)
RK_B = (1.0 / 4.0, 3.0 / 20.0, 3.0 / 5.0)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-std=gnu11", "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def load(path: str):
    """Open a compiled oracle library and declare its entry points."""
    L = ctypes.CDLL(path)
    i, d, u64, vp = ctypes.c_int, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
    L.oracle_splitmix64.restype = u64
    L.oracle_splitmix64.argtypes = [u64, u64]
    L.oracle_splitmix_uniform.restype = d
    L.oracle_splitmix_uniform.argtypes = [u64, u64]
    L.oracle_set_threads.argtypes = [i]
    L.oracle_get_threads.restype = i
    for s in ("_d", "_ld"):
        getattr(L, "oracle_init" + s).argtypes = [i, i, i, d, d, d, i, d, u64, d, d, d, vp]
        getattr(L, "oracle_init_slab" + s).argtypes = [i, i, i, i, i, d, d, d, i, d, u64, d, d,
                                                      d, vp]
        getattr(L, "oracle_rhs_slab" + s).argtypes = [i, i, i, i, d, d, d, d, vp, vp]
        getattr(L, "oracle_prims" + s).argtypes = [i, i, i, d, d, d, d, vp, vp]
        getattr(L, "oracle_rhs" + s).argtypes = [i, i, i, d, d, d, d, vp, vp]
        getattr(L, "oracle_rhs_planes" + s).argtypes = [i, i, i, d, d, d, d, vp, vp, i, i]
        getattr(L, "oracle_rk_step" + s).argtypes = [i, i, i, d, d, d, d, d, i, vp]
        getattr(L, "oracle_diag" + s).argtypes = [i, i, i, d, d, d, d, vp, vp]
        getattr(L, "oracle_derivs" + s).argtypes = [i, i, i, d, d, d, d, vp, vp]
        getattr(L, "oracle_rk_step_rounded" + s).argtypes = [i, i, i, d, d, d, d, d, i, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = load(_LIB)
    return _lib


@contextlib.contextmanager
def library(path: str):
    """Route every call of this module to another build of the oracle (the
    tests use it to run the pins on copies with a planted mistake)."""
    global _lib
    saved = lib()
    _lib = load(path)
    try:
        yield _lib
    finally:
        _lib = saved


def _dtype(prec: str):
    return {"d": np.float64, "ld": np.longdouble}[prec]


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def _phys(phys):
    return (float(phys["Re"]), float(phys["Ma"]), float(phys["Pr"]), float(phys["gamma"]))


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def splitmix64(seed: int, counter: int) -> int:
    return int(lib().oracle_splitmix64(seed, counter))


def init(shape, phys, tgv, prec: str = "d") -> np.ndarray:
    """Taylor-Green state q[5][nz][ny][nx] (Section 3)."""
    nx, ny, nz = shape
    q = np.zeros((5, nz, ny, nx), dtype=_dtype(prec))
    ph = tgv.get("phase", (0.0, 0.0, 0.0))
    getattr(lib(), "oracle_init_" + prec)(
        nx, ny, nz, float(phys["gamma"]), float(phys["Ma"]), float(tgv.get("V0", 1.0)),
        int(tgv.get("pert_kind", 0)), float(tgv.get("pert_amp", 0.0)),
        int(tgv.get("seed", 0)), float(ph[0]), float(ph[1]), float(ph[2]), _ptr(q))
    return q


def init_slab(shape, k0: int, nk: int, phys, tgv, prec: str = "d") -> np.ndarray:
    """Planes k0 .. k0+nk-1 (periodic) of the Taylor-Green state of an
    nx x ny x nz grid, as a [5][nk][ny][nx] array."""
    nx, ny, nz = shape
    q = np.zeros((5, nk, ny, nx), dtype=_dtype(prec))
    ph = tgv.get("phase", (0.0, 0.0, 0.0))
    getattr(lib(), "oracle_init_slab_" + prec)(
        nx, ny, nz, int(k0), int(nk), float(phys["gamma"]), float(phys["Ma"]),
        float(tgv.get("V0", 1.0)), int(tgv.get("pert_kind", 0)), float(tgv.get("pert_amp", 0.0)),
        int(tgv.get("seed", 0)), float(ph[0]), float(ph[1]), float(ph[2]), _ptr(q))
    return q


def rhs_slab(q_slab: np.ndarray, nz_glob: int, phys, prec: str = "d") -> np.ndarray:
    """Residual on the interior planes 2 .. nzs-3 of a slab of nzs
    consecutive planes of an nz_glob-plane periodic grid; returns those
    nzs-4 planes."""
    q_slab = np.ascontiguousarray(q_slab, dtype=_dtype(prec))
    _, nzs, ny, nx = q_slab.shape
    if nzs < 5 or nzs > nz_glob + 4:
        raise ValueError("slab needs 5 <= nzs <= nz_glob + 4 planes")
    r = np.zeros_like(q_slab)
    getattr(lib(), "oracle_rhs_slab_" + prec)(nx, ny, int(nz_glob), nzs, *_phys(phys),
                                              _ptr(q_slab), _ptr(r))
    return r[:, 2:nzs - 2]


def _shape_of(q):
    _, nz, ny, nx = q.shape
    return nx, ny, nz


def prims(q: np.ndarray, phys, prec: str = "d") -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=_dtype(prec))
    nx, ny, nz = _shape_of(q)
    out = np.empty_like(q)
    getattr(lib(), "oracle_prims_" + prec)(nx, ny, nz, *_phys(phys), _ptr(q), _ptr(out))
    return out


def rhs(q: np.ndarray, phys, prec: str = "d") -> np.ndarray:
    """Residual R(q) (Section 2, eqs (1)-(5), (8))."""
    q = np.ascontiguousarray(q, dtype=_dtype(prec))
    nx, ny, nz = _shape_of(q)
    r = np.empty_like(q)
    getattr(lib(), "oracle_rhs_" + prec)(nx, ny, nz, *_phys(phys), _ptr(q), _ptr(r))
    return r


def rhs_planes(q: np.ndarray, phys, k0: int, k1: int, r: np.ndarray | None = None,
               prec: str = "d") -> np.ndarray:
    """Residual on z-planes [k0, k1) only (used to time a bounded sample)."""
    nx, ny, nz = _shape_of(q)
    if r is None:
        r = np.zeros_like(q)
    getattr(lib(), "oracle_rhs_planes_" + prec)(nx, ny, nz, *_phys(phys), _ptr(q), _ptr(r),
                                               int(k0), int(k1))
    return r


def rk_step(q: np.ndarray, phys, dt: float, nsteps: int = 1, prec: str = "d") -> np.ndarray:
    """Advance nsteps low-storage RK3 steps; returns a new array."""
    q = np.array(q, dtype=_dtype(prec), order="C", copy=True)
    nx, ny, nz = _shape_of(q)
    getattr(lib(), "oracle_rk_step_" + prec)(nx, ny, nz, *_phys(phys), float(dt), int(nsteps),
                                            _ptr(q))
    return q


def rk_step_rounded(q: np.ndarray, phys, dt: float, nsteps: int = 1,
                    prec: str = "d") -> np.ndarray:
    """rk_step with each substep's input state rounded to float32 (the
    single-precision state of the FP32 form; the accumulator keeps prec)."""
    q = np.array(q, dtype=_dtype(prec), order="C", copy=True)
    nx, ny, nz = _shape_of(q)
    getattr(lib(), "oracle_rk_step_rounded_" + prec)(nx, ny, nz, *_phys(phys), float(dt),
                                                    int(nsteps), _ptr(q))
    return q


def rk_step_slab(q_slab: np.ndarray, nz_glob: int, phys, dt: float, prec: str = "d",
                 stage_dtype=None) -> np.ndarray:
    """One step of the same low-storage RK3 (2R form, Section 2) on a z-slab.

    q_slab holds planes k0-6 .. k1+5 of a periodic nz_glob-plane state (full
    x and y extents). A stage's residual on a plane needs the two planes on
    either side, so each of the three stages gives up two planes at both
    ends; the result, planes k0 .. k1-1 after the step, equals what the
    full-grid step gives there. The update is the one of oracle_rk_step:
    q <- q_acc + a_s dt r (first two stages), then q_acc <- q_acc + b_s dt r,
    the step's result being q_acc.

    stage_dtype (e.g. numpy.float32) models the single-precision form: the
    state each stage's residual is evaluated on is first rounded through
    that type, while the accumulator stays in ``prec``.
    """
    t = _dtype(prec)
    q = np.ascontiguousarray(q_slab, dtype=t)
    if q.shape[1] < 13:
        raise ValueError("slab needs at least 13 planes (one output plane)")
    a = (t(2) / t(3), t(5) / t(12))
    b = (t(1) / t(4), t(3) / t(20), t(3) / t(5))
    tdt = t(dt)
    acc = q
    for s in range(3):
        if stage_dtype is not None:
            q = q.astype(stage_dtype).astype(t)
        r = rhs_slab(q, nz_glob, phys, prec=prec)  # interior planes of this slab
        acc = acc[:, 2:-2]
        if s < 2:
            q = np.ascontiguousarray(acc + a[s] * tdt * r)
        acc = acc + b[s] * tdt * r
    return acc


def diagnostics(q: np.ndarray, phys, prec: str = "d") -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=_dtype(prec))
    nx, ny, nz = _shape_of(q)
    out = np.zeros(NDIAG, dtype=np.float64)
    getattr(lib(), "oracle_diag_" + prec)(nx, ny, nz, *_phys(phys), _ptr(q), _ptr(out))
    return out


def derivs(q: np.ndarray, phys, prec: str = "d") -> np.ndarray:
    """The 60 derivative groups as fields [60][nz][ny][nx] (order documented
    with oracle_derivs in the C source)."""
    q = np.ascontiguousarray(q, dtype=_dtype(prec))
    nx, ny, nz = _shape_of(q)
    d = np.empty((60, nz, ny, nx), dtype=_dtype(prec))
    getattr(lib(), "oracle_derivs_" + prec)(nx, ny, nz, *_phys(phys), _ptr(q), _ptr(d))
    return d
