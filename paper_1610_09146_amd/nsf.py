"""Python binding of the C ABI in ``include/nsf.h`` (``libnsf.so``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library. PyTorch supplies device memory (tensors) and
streams; tensors are passed to the library as raw device pointers.

``torch`` is imported before the library is loaded so that ``libnsf.so``
binds to the same HIP runtime instance as torch (same ``libamdhip64.so.7``
soname), which lets torch's streams be passed straight through.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnsf.so")

OK, EINVAL, EWORKSPACE, EHIP, EUNSUPPORTED, ENONFINITE = 0, -1, -2, -3, -4, -5
BL, RA, SS, SN, RS, AUTO = 0, 1, 2, 3, 4, 5
F64, F32 = 0, 1
NDIAG = 16
TUNE_QUICK = 1
VARIANTS = {"BL": BL, "RA": RA, "SS": SS, "SN": SN, "RS": RS, "AUTO": AUTO}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}
PRECISIONS = {"f64": F64, "f32": F32}
DIAG_NAMES = [
    "ke", "enstrophy", "mean_rho", "mean_rhou", "mean_rhov", "mean_rhow", "mean_rhoE",
    "max_rho", "max_rhou", "max_rhov", "max_rhow", "max_rhoE", "min_rho", "min_p",
    "nonfinite", "mean_p",
]


class NsfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class Phys(ctypes.Structure):
    _fields_ = [("Re", ctypes.c_double), ("Ma", ctypes.c_double), ("Pr", ctypes.c_double),
                ("gamma", ctypes.c_double)]


class TGV(ctypes.Structure):
    _fields_ = [("V0", ctypes.c_double), ("pert_amp", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("pert_kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("phase", ctypes.c_double * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("zchunk", ctypes.c_int32), ("fuse", ctypes.c_int32), ("naive", ctypes.c_int32),
                ("gstore", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class TuneResult(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("tune", Tuning), ("pt_rhs_per_s", ctypes.c_double),
                ("parity_rel_err", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnsf.so; fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NsfError(EUNSUPPORTED, f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_size_t)
        G, P, Tg, Tu = (ctypes.POINTER(Grid), ctypes.POINTER(Phys), ctypes.POINTER(TGV),
                        ctypes.POINTER(Tuning))
        L.nsf_status_string.restype = ctypes.c_char_p
        L.nsf_status_string.argtypes = [ctypes.c_int]
        L.nsf_last_error.restype = ctypes.c_char_p
        L.nsf_version.restype = ctypes.c_int
        L.nsf_workspace_bytes.argtypes = [G, ctypes.c_int, ctypes.c_int, Tu, ctypes.POINTER(sz)]
        L.nsf_init_fields.argtypes = [G, P, Tg, ctypes.c_int, vp, vp, vp]
        L.nsf_rhs.argtypes = [G, P, ctypes.c_int, ctypes.c_int, Tu, vp, vp, vp, sz, vp]
        L.nsf_rk_step.argtypes = [G, P, ctypes.c_int, ctypes.c_int, Tu, d, i32, vp, vp, vp, vp, sz, vp]
        L.nsf_rk_step_monitored.argtypes = [G, P, ctypes.c_int, ctypes.c_int, Tu, d, i32, vp, vp,
                                            vp, vp, sz, vp, vp]
        L.nsf_diagnostics.argtypes = [G, P, ctypes.c_int, vp, vp, sz, ctypes.POINTER(d), vp]
        L.nsf_diagnostics_noalloc.argtypes = [G, P, ctypes.c_int, vp, ctypes.POINTER(d), vp]
        L.nsf_device_copy.argtypes = [vp, vp, sz, vp]
        L.nsf_timer_enable.argtypes = [ctypes.c_char_p]
        L.nsf_timer_read.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(d)]
        L.nsf_timer_names.restype = ctypes.c_char_p
        L.nsf_batch_workspace_bytes.argtypes = [i32, G, ctypes.c_int, ctypes.POINTER(sz)]
        L.nsf_batch_create.argtypes = [i32, G, P, ctypes.POINTER(d), ctypes.c_int,
                                       ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp,
                                       ctypes.POINTER(vp)]
        L.nsf_batch_step.argtypes = [vp, i32, vp]
        L.nsf_batch_step_eager.argtypes = [vp, i32, vp]
        L.nsf_batch_diagnostics.argtypes = [vp, ctypes.POINTER(d), vp]
        L.nsf_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.nsf_batch_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
        L.nsf_batch_create_variant.argtypes = [i32, G, P, ctypes.POINTER(d), ctypes.c_int,
                                               ctypes.c_int, Tu, ctypes.POINTER(vp),
                                               ctypes.POINTER(vp), vp, sz, vp, ctypes.POINTER(vp)]
        L.nsf_batch_autotune_workspace_bytes.argtypes = [i32, G, ctypes.c_int, ctypes.POINTER(sz)]
        L.nsf_batch_autotune.argtypes = [i32, G, P, ctypes.POINTER(d), ctypes.c_int, i32, vp, sz,
                                         ctypes.POINTER(i32), Tu, ctypes.POINTER(d), vp]
        L.nsf_batch_destroy.argtypes = [vp]
        L.nsf_batch_create_tuned.argtypes = [i32, G, P, ctypes.POINTER(d), ctypes.c_int, Tu,
                                             ctypes.POINTER(vp), ctypes.POINTER(vp), vp, sz, vp,
                                             ctypes.POINTER(vp)]
        TR = ctypes.POINTER(TuneResult)
        L.nsf_autotune_workspace_bytes.argtypes = [G, ctypes.c_int, ctypes.c_int,
                                                   ctypes.POINTER(sz)]
        L.nsf_autotune.argtypes = [G, P, ctypes.c_int, ctypes.c_int, i32, ctypes.c_char_p, vp, sz,
                                   TR, vp]
        L.nsf_tune_load.argtypes = [ctypes.c_char_p]
        L.nsf_tune_get.argtypes = [G, ctypes.c_int, TR]
        _lib = L
    return _lib


def _check(rc: int, what: str) -> int:
    if rc != OK:
        L = lib()
        raise NsfError(rc, f"{what}: {L.nsf_status_string(rc).decode()}: "
                           f"{L.nsf_last_error().decode()}")
    return rc


def _grid(shape) -> Grid:
    nx, ny, nz = (int(v) for v in shape)
    return Grid(nx, ny, nz)


def _phys(phys: dict) -> Phys:
    return Phys(float(phys["Re"]), float(phys["Ma"]), float(phys["Pr"]), float(phys["gamma"]))


def _tgv(tgv: dict | None) -> TGV:
    tgv = tgv or {}
    ph = tgv.get("phase", (0.0, 0.0, 0.0))
    t = TGV(float(tgv.get("V0", 1.0)), float(tgv.get("pert_amp", 0.0)),
            int(tgv.get("seed", 0)) & (2**64 - 1), int(tgv.get("pert_kind", 0)), 0)
    for a in range(3):
        t.phase[a] = float(ph[a])
    return t


def _tuning(tune: dict | None):
    if not tune:
        return None
    t = Tuning(int(tune.get("block_x", 0)), int(tune.get("block_y", 0)), int(tune.get("zchunk", 0)),
               int(tune.get("fuse", 0)), int(tune.get("naive", 0)), int(tune.get("gstore", 0)))
    return ctypes.byref(t)


def _variant(v) -> int:
    return VARIANTS[v] if isinstance(v, str) else int(v)


def _precision(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise NsfError(EINVAL, "tensor must be on the GPU")
    if not t.is_contiguous():
        raise NsfError(EINVAL, "tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def field_dtype(precision) -> torch.dtype:
    return torch.float32 if _precision(precision) == F32 else torch.float64


def version() -> int:
    return int(lib().nsf_version())


def _fields(shape, precision, **tensors) -> None:
    """Check that every given state tensor holds 5 fields of the grid in the
    right dtype (q, r: the precision's dtype; q_acc: float64): the library
    takes plain pointers and cannot see the allocation sizes."""
    nx, ny, nz = (int(v) for v in shape)
    need = 5 * nx * ny * nz
    for name, t in tensors.items():
        if t is None:
            continue
        dt = torch.float64 if name == "q_acc" else field_dtype(precision)
        if t.dtype != dt:
            raise NsfError(EINVAL, f"{name} must be {dt}, got {t.dtype}")
        if t.numel() != need:
            raise NsfError(EINVAL, f"{name} must hold 5 x {nx}x{ny}x{nz} values, got {t.numel()}")


def workspace_bytes(shape, variant, precision, tune: dict | None = None) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().nsf_workspace_bytes(ctypes.byref(_grid(shape)), _variant(variant),
                                     _precision(precision), _tuning(tune), ctypes.byref(out)),
           "nsf_workspace_bytes")
    return int(out.value)


def init_fields(shape, phys, tgv, precision, q: torch.Tensor, q_acc: torch.Tensor | None,
                stream=None) -> None:
    _fields(shape, precision, q=q, q_acc=q_acc)
    _check(lib().nsf_init_fields(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                                 ctypes.byref(_tgv(tgv)), _precision(precision), _ptr(q),
                                 _ptr(q_acc), _stream(stream)), "nsf_init_fields")


def rhs(shape, phys, variant, precision, q, r, work, tune: dict | None = None, stream=None) -> None:
    _fields(shape, precision, q=q, r=r)
    _check(lib().nsf_rhs(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)), _variant(variant),
                         _precision(precision), _tuning(tune), _ptr(q), _ptr(r), _ptr(work),
                         work.numel() * work.element_size(), _stream(stream)), "nsf_rhs")


def rk_step(shape, phys, variant, precision, dt, nsteps, q, q_acc, r, work,
            tune: dict | None = None, stream=None) -> None:
    _fields(shape, precision, q=q, q_acc=q_acc, r=r)
    _check(lib().nsf_rk_step(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                             _variant(variant), _precision(precision), _tuning(tune), float(dt),
                             int(nsteps), _ptr(q), _ptr(q_acc), _ptr(r), _ptr(work),
                             work.numel() * work.element_size(), _stream(stream)), "nsf_rk_step")


def rk_step_monitored(shape, phys, variant, precision, dt, nsteps, q, q_acc, r, work,
                      monitor: torch.Tensor, tune: dict | None = None, stream=None) -> None:
    """rk_step that writes (KE, enstrophy) of the state at the start of every
    step into ``monitor``, a float64 device tensor of at least 2 * nsteps."""
    if monitor.dtype != torch.float64 or not monitor.is_contiguous() or monitor.numel() < 2 * nsteps:
        raise ValueError("monitor must be a contiguous float64 tensor of >= 2 * nsteps elements")
    _fields(shape, precision, q=q, q_acc=q_acc, r=r)
    _check(lib().nsf_rk_step_monitored(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                                       _variant(variant), _precision(precision), _tuning(tune),
                                       float(dt), int(nsteps), _ptr(q), _ptr(q_acc), _ptr(r),
                                       _ptr(work), work.numel() * work.element_size(),
                                       _ptr(monitor), _stream(stream)), "nsf_rk_step_monitored")


def diagnostics(shape, phys, precision, q, work, stream=None, check: bool = True) -> np.ndarray:
    _fields(shape, precision, q=q)
    out = (ctypes.c_double * NDIAG)()
    rc = lib().nsf_diagnostics(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                               _precision(precision), _ptr(q), _ptr(work),
                               work.numel() * work.element_size(), out, _stream(stream))
    if check or rc != ENONFINITE:
        _check(rc, "nsf_diagnostics")
    return np.array(out[:], dtype=np.float64)


def diagnostics_noalloc(shape, phys, precision, q, stream=None, check: bool = True) -> np.ndarray:
    """nsf_diagnostics_noalloc: the diagnostics of q with no work buffer
    (the library's fixed per-GPU scratch holds the partial sums)."""
    _fields(shape, precision, q=q)
    out = (ctypes.c_double * NDIAG)()
    rc = lib().nsf_diagnostics_noalloc(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                                       _precision(precision), _ptr(q), out, _stream(stream))
    if check or rc != ENONFINITE:
        _check(rc, "nsf_diagnostics_noalloc")
    return np.array(out[:], dtype=np.float64)


def batch_autotune(instances, precision, steps: int = 3, stream=None) -> dict:
    """nsf_batch_autotune on an ensemble (list of instance dicts): the
    fastest parity-checked (stage algorithm, tile height, z-chunk)."""
    n = len(instances)
    grids = (Grid * n)(*[_grid(i["shape"]) for i in instances])
    phys = (Phys * n)(*[_phys(i["phys"]) for i in instances])
    dts = (ctypes.c_double * n)(*[float(i["dt"]) for i in instances])
    v, t, rate = ctypes.c_int32(0), Tuning(), ctypes.c_double(0)
    nb = ctypes.c_size_t(0)
    _check(lib().nsf_batch_autotune_workspace_bytes(n, grids, _precision(precision),
                                                    ctypes.byref(nb)),
           "nsf_batch_autotune_workspace_bytes")
    work = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device="cuda")
    _check(lib().nsf_batch_autotune(n, grids, phys, dts, _precision(precision), int(steps),
                                    _ptr(work), int(nb.value), ctypes.byref(v), ctypes.byref(t),
                                    ctypes.byref(rate), _stream(stream)), "nsf_batch_autotune")
    del work
    return {"variant": VARIANT_NAMES.get(int(v.value)),
            "tune": {"block_y": t.block_y, "zchunk": t.zchunk}, "pt_rhs_per_s": float(rate.value)}


def _tune_dict(r: TuneResult) -> dict:
    t = r.tune
    return {"variant": VARIANT_NAMES.get(int(r.variant), int(r.variant)),
            "tune": {"block_x": t.block_x, "block_y": t.block_y, "zchunk": t.zchunk,
                     "fuse": t.fuse, "naive": t.naive, "gstore": t.gstore},
            "pt_rhs_per_s": float(r.pt_rhs_per_s), "parity_rel_err": float(r.parity_rel_err)}


def autotune(shape, phys, precision, quick: bool = True, steps: int = 2,
             cache_path: str | None = None, stream=None) -> dict:
    """Run the autotuner for one grid and precision (synchronous); the choice
    is recorded for variant "AUTO" in this process."""
    r = TuneResult()
    flags = TUNE_QUICK if quick else 0
    nb = ctypes.c_size_t(0)
    _check(lib().nsf_autotune_workspace_bytes(ctypes.byref(_grid(shape)), _precision(precision),
                                              flags, ctypes.byref(nb)),
           "nsf_autotune_workspace_bytes")
    work = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device="cuda")
    _check(lib().nsf_autotune(ctypes.byref(_grid(shape)), ctypes.byref(_phys(phys)),
                              _precision(precision), flags, int(steps),
                              cache_path.encode() if cache_path else None, _ptr(work),
                              int(nb.value), ctypes.byref(r), _stream(stream)), "nsf_autotune")
    del work
    return _tune_dict(r)


def tune_load(cache_path: str) -> int:
    rc = lib().nsf_tune_load(cache_path.encode())
    if rc < 0:
        _check(rc, "nsf_tune_load")
    return int(rc)


def tune_get(shape, precision) -> dict | None:
    r = TuneResult()
    rc = lib().nsf_tune_get(ctypes.byref(_grid(shape)), _precision(precision), ctypes.byref(r))
    return _tune_dict(r) if rc == OK else None


def device_copy(src: torch.Tensor, dst: torch.Tensor, nbytes: int | None = None, stream=None) -> None:
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    _check(lib().nsf_device_copy(_ptr(src), _ptr(dst), n, _stream(stream)), "nsf_device_copy")


def timer_enable(name: str | None) -> None:
    _check(lib().nsf_timer_enable(name.encode() if name else None), "nsf_timer_enable")


def timer_read() -> tuple[int, float]:
    c, ms = ctypes.c_int64(0), ctypes.c_double(0.0)
    _check(lib().nsf_timer_read(ctypes.byref(c), ctypes.byref(ms)), "nsf_timer_read")
    return int(c.value), float(ms.value)


def timer_names() -> list[str]:
    return lib().nsf_timer_names().decode().split(",")


@dataclass
class Solver:
    """Device buffers of one Taylor-Green run, allocated with torch.

    q (precision dtype), q_acc (float64), r (precision dtype) are
    ``[5, nz, ny, nx]`` tensors; work is a byte tensor of
    ``workspace_bytes`` bytes.
    """
    shape: tuple
    phys: dict
    variant: int | str = RA
    precision: int | str = F64
    tune: dict | None = None
    device: str = "cuda"
    q: torch.Tensor = field(init=False)
    q_acc: torch.Tensor = field(init=False)
    r: torch.Tensor = field(init=False)
    work: torch.Tensor = field(init=False)

    def __post_init__(self):
        nx, ny, nz = self.shape
        dt = field_dtype(self.precision)
        self.q = torch.empty((5, nz, ny, nx), dtype=dt, device=self.device)
        self.q_acc = torch.empty((5, nz, ny, nx), dtype=torch.float64, device=self.device)
        self.r = torch.empty((5, nz, ny, nx), dtype=dt, device=self.device)
        nb = workspace_bytes(self.shape, self.variant, self.precision, self.tune)
        self.work = torch.empty(nb, dtype=torch.uint8, device=self.device)

    def init(self, tgv: dict | None = None) -> None:
        init_fields(self.shape, self.phys, tgv, self.precision, self.q, self.q_acc)

    def rhs(self, q: torch.Tensor | None = None, r: torch.Tensor | None = None) -> torch.Tensor:
        q = self.q if q is None else q
        r = self.r if r is None else r
        rhs(self.shape, self.phys, self.variant, self.precision, q, r, self.work, self.tune)
        return r

    def step(self, dt: float, nsteps: int = 1) -> None:
        rk_step(self.shape, self.phys, self.variant, self.precision, dt, nsteps, self.q,
                self.q_acc, self.r, self.work, self.tune)

    def step_monitored(self, dt: float, nsteps: int, monitor: torch.Tensor) -> None:
        rk_step_monitored(self.shape, self.phys, self.variant, self.precision, dt, nsteps, self.q,
                          self.q_acc, self.r, self.work, monitor, self.tune)

    def diagnostics(self, check: bool = True) -> np.ndarray:
        return diagnostics(self.shape, self.phys, self.precision, self.q, self.work, check=check)


class Batch:
    """Batched form: independent Taylor-Green instances of uneven grids and
    parameters advanced together (one persistent launch per RK stage, the
    step captured in a hipGraph). ``instances`` is a list of dicts with
    ``shape``, ``phys``, ``tgv`` and ``dt`` (see workloads.batch_instances).
    Per-instance q / q_acc tensors and the shared work buffer are allocated
    with torch and kept alive by this object."""

    def __init__(self, instances, precision="f64", device="cuda", stream=None, tune=None,
                 variant="SN"):
        self.instances = list(instances)
        self.precision = _precision(precision)
        self.count = len(self.instances)
        dt = field_dtype(precision)
        self.q, self.q_acc = [], []
        for inst in self.instances:
            nx, ny, nz = inst["shape"]
            q = torch.empty((5, nz, ny, nx), dtype=dt, device=device)
            qa = torch.empty((5, nz, ny, nx), dtype=torch.float64, device=device)
            init_fields(inst["shape"], inst["phys"], inst["tgv"], precision, q, qa, stream)
            self.q.append(q)
            self.q_acc.append(qa)
        grids = (Grid * self.count)(*[_grid(i["shape"]) for i in self.instances])
        phys = (Phys * self.count)(*[_phys(i["phys"]) for i in self.instances])
        dts = (ctypes.c_double * self.count)(*[float(i["dt"]) for i in self.instances])
        qp = (ctypes.c_void_p * self.count)(*[t.data_ptr() for t in self.q])
        ap = (ctypes.c_void_p * self.count)(*[t.data_ptr() for t in self.q_acc])
        nb = ctypes.c_size_t(0)
        L = lib()
        _check(L.nsf_batch_workspace_bytes(self.count, grids, self.precision, ctypes.byref(nb)),
               "nsf_batch_workspace_bytes")
        self.work = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        handle = ctypes.c_void_p(0)
        torch.cuda.synchronize()
        if tune or variant != "SN":
            _check(L.nsf_batch_create_variant(self.count, grids, phys, dts, self.precision,
                                              _variant(variant), _tuning(tune), qp, ap,
                                              _ptr(self.work), int(nb.value), _stream(stream),
                                              ctypes.byref(handle)), "nsf_batch_create_variant")
        else:
            _check(L.nsf_batch_create(self.count, grids, phys, dts, self.precision, qp, ap,
                                      _ptr(self.work), int(nb.value), _stream(stream),
                                      ctypes.byref(handle)), "nsf_batch_create")
        self.handle = handle

    def step(self, nsteps: int = 1, graph: bool = True, stream=None) -> None:
        fn = lib().nsf_batch_step if graph else lib().nsf_batch_step_eager
        _check(fn(self.handle, int(nsteps), _stream(stream)), "nsf_batch_step")

    def diagnostics(self, stream=None) -> np.ndarray:
        out = (ctypes.c_double * (self.count * NDIAG))()
        _check(lib().nsf_batch_diagnostics(self.handle, out, _stream(stream)),
               "nsf_batch_diagnostics")
        return np.array(out[:], dtype=np.float64).reshape(self.count, NDIAG)

    def info(self) -> tuple[int, int]:
        a, b = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().nsf_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b)), "nsf_batch_info")
        return int(a.value), int(b.value)

    def config(self) -> dict:
        """Stage algorithm, tile height and per-instance z-chunks (nsf_batch_config)."""
        v, ty = ctypes.c_int32(0), ctypes.c_int32(0)
        zc = (ctypes.c_int32 * self.count)()
        _check(lib().nsf_batch_config(self.handle, ctypes.byref(v), ctypes.byref(ty), zc),
               "nsf_batch_config")
        return {"variant": VARIANT_NAMES.get(int(v.value)), "tile_y": int(ty.value),
                "zchunk": [int(x) for x in zc]}

    def points(self) -> int:
        return sum(int(np.prod(i["shape"])) for i in self.instances)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().nsf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
