"""CPU checks of the C ABI: the built library loads, exports every function
declared in include/nsf.h, and rejects bad arguments before touching the
GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def nsf():
    from paper_1610_09146_amd import nsf as N
    if not os.path.exists(N.LIB_PATH):
        from paper_1610_09146_amd import build
        build.build()
    return N


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("nsf_init_fields", "nsf_rhs", "nsf_rk_step", "nsf_diagnostics",
                 "nsf_workspace_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol(nsf):
    L = nsf.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_no_undeclared_nsf_exports(nsf):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", nsf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = sorted({l.split()[-1] for l in out.splitlines() if " T nsf_" in l})
    assert exported == declared_functions()


def test_status_strings(nsf):
    L = nsf.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.nsf_status_string(code).decode().startswith("NSF_")
    assert nsf.version() >= 100


def test_workspace_sizes(nsf):
    n = 32
    npts = n ** 3
    sizes = {v: nsf.workspace_bytes((n, n, n), v, "f64") for v in ("BL", "RA", "SS")}
    assert sizes["RA"] >= 5 * npts * 8
    assert sizes["SS"] - sizes["RA"] >= 9 * npts * 8
    # (RA and SS also hold their monitor's per-tile partial sums: two doubles
    # per tile, a few KB)
    assert sizes["BL"] - sizes["RA"] >= 61 * npts * 8 - 64 * 1024
    s32 = nsf.workspace_bytes((n, n, n), "RA", "f32")
    assert s32 >= 5 * npts * 4 and s32 < sizes["RA"]
    # the fused form adds one rotating state (the other shares the primitives)
    fused = nsf.workspace_bytes((n, n, n), "RA", "f64", {"fuse": 1})
    assert 5 * npts * 8 <= fused - sizes["RA"] < 6 * npts * 8
    # so does the fused SS form (the other is the caller's r)
    ss_fused = nsf.workspace_bytes((n, n, n), "SS", "f64", {"fuse": 1})
    assert 5 * npts * 8 <= ss_fused - sizes["SS"] < 6 * npts * 8


@pytest.mark.parametrize("shape", [(4, 8, 8), (8, 0, 8), (8, 8, -3), (2048, 2048, 1024),
                                   (8, 8, 2), (8, 8, 4), (1, 8, 8), (8, 1, 8),
                                   (16384, 16384, 1), (1 << 20, 256, 5)])
def test_bad_grid_rejected(nsf, shape):
    with pytest.raises(nsf.NsfError) as ei:
        nsf.workspace_bytes(shape, "RA", "f64")
    assert ei.value.code == nsf.EINVAL


def test_plane_limit(nsf):
    # a z-plane below 2^28 points is accepted (2D, 16383 x 16384), one at
    # 2^28 is not (the fused stage uses 32-bit byte offsets within a plane)
    assert nsf.workspace_bytes((16383, 16384, 1), "RA", "f64") > 0
    with pytest.raises(nsf.NsfError):
        nsf.workspace_bytes((16384, 16384, 1), "RA", "f64")


def test_bad_variant_and_precision_rejected(nsf):
    with pytest.raises(nsf.NsfError) as ei:
        nsf.workspace_bytes((8, 8, 8), 9, "f64")
    assert ei.value.code == nsf.EINVAL
    with pytest.raises(nsf.NsfError) as ei:
        nsf.workspace_bytes((8, 8, 8), "RA", 7)
    assert ei.value.code == nsf.EINVAL


def _call_rhs(nsf, shape, phys, q, r, work, nbytes, variant=1):
    L = nsf.lib()
    return L.nsf_rhs(ctypes.byref(nsf._grid(shape)), ctypes.byref(nsf._phys(phys)), variant, 0,
                     None, q, r, work, nbytes, None)


def test_rhs_validation_before_launch(nsf):
    # fake, never-dereferenced addresses: validation must fail first
    phys = {"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4}
    shape = (8, 8, 8)
    need = nsf.workspace_bytes(shape, "RA", "f64")
    q, r, w = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x20000000), ctypes.c_void_p(0x30000000)
    assert _call_rhs(nsf, shape, phys, q, r, w, need - 1) == nsf.EWORKSPACE
    assert _call_rhs(nsf, shape, phys, None, r, w, need) == nsf.EINVAL
    assert _call_rhs(nsf, shape, dict(phys, gamma=1.0), q, r, w, need) == nsf.EINVAL
    assert _call_rhs(nsf, shape, dict(phys, Re=-1.0), q, r, w, need) == nsf.EINVAL
    # r overlapping q
    assert _call_rhs(nsf, shape, phys, q, ctypes.c_void_p(0x10000008), w, need) == nsf.EINVAL
    assert "overlap" in nsf.lib().nsf_last_error().decode()


def test_rk_step_validation_before_launch(nsf):
    phys = {"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4}
    shape = (8, 8, 8)
    need = nsf.workspace_bytes(shape, "SS", "f64")
    L = nsf.lib()
    args = lambda dt, n, wb: (ctypes.byref(nsf._grid(shape)), ctypes.byref(nsf._phys(phys)), 2, 0,
                              None, dt, n, ctypes.c_void_p(0x1000000), ctypes.c_void_p(0x2000000),
                              ctypes.c_void_p(0x3000000), ctypes.c_void_p(0x4000000), wb, None)
    assert L.nsf_rk_step(*args(float("nan"), 1, need)) == nsf.EINVAL
    assert L.nsf_rk_step(*args(0.01, -1, need)) == nsf.EINVAL
    assert L.nsf_rk_step(*args(0.01, 1, need // 2)) == nsf.EWORKSPACE


def test_rk_step_monitored_validation_before_launch(nsf):
    # fake, never-dereferenced addresses: the monitor checks fail first
    phys = {"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4}
    shape = (8, 8, 8)
    need = nsf.workspace_bytes(shape, "RA", "f64", {"fuse": 1})
    L = nsf.lib()
    tune = nsf._tuning({"fuse": 1})

    def call(monitor, nsteps=4):
        return L.nsf_rk_step_monitored(
            ctypes.byref(nsf._grid(shape)), ctypes.byref(nsf._phys(phys)), 1, 0, tune, 0.01,
            nsteps, ctypes.c_void_p(0x1000000), ctypes.c_void_p(0x2000000),
            ctypes.c_void_p(0x3000000), ctypes.c_void_p(0x4000000), need, monitor, None)

    assert call(None) == nsf.EINVAL
    assert call(ctypes.c_void_p(0x5000004)) == nsf.EINVAL
    assert "aligned" in L.nsf_last_error().decode()
    # monitor inside q
    assert call(ctypes.c_void_p(0x1000008)) == nsf.EINVAL
    assert "overlap" in L.nsf_last_error().decode()
    assert call(ctypes.c_void_p(0x5000000), nsteps=-1) == nsf.EINVAL


def test_timer_names(nsf):
    names = nsf.timer_names()
    assert "update" in names and "diag" in names


def test_two_dimensional_grid_accepted(nsf):
    # nz = 1 is the z-independent (two-dimensional) problem
    n = nsf.workspace_bytes((16, 12, 1), "RA", "f64")
    assert n >= 5 * 16 * 12 * 8



def test_binding_checks_state_sizes_and_dtypes(nsf):
    # the library takes plain pointers; the binding rejects tensors that do
    # not hold five fields of the grid in the right dtype before any call
    import torch
    shape = (8, 8, 8)
    good = torch.zeros(5 * 8 ** 3, dtype=torch.float64)
    nsf._fields(shape, "f64", q=good, q_acc=good, r=good)
    with pytest.raises(nsf.NsfError):
        nsf._fields(shape, "f64", q=good[:-1])
    with pytest.raises(nsf.NsfError):
        nsf._fields(shape, "f32", q=good)
    with pytest.raises(nsf.NsfError):
        nsf._fields(shape, "f32", q=good.float(), q_acc=good.float())


def test_noalloc_rejects_before_any_work(nsf):
    """nsf_diagnostics_noalloc refuses, before any HIP call, a grid with more
    diagnostics tiles than its fixed scratch holds (ceil(nx/32) ceil(ny/8)
    ceil(nz/64) > 65536) and NULL pointers."""
    import ctypes
    L = nsf.lib()
    out = (ctypes.c_double * nsf.NDIAG)()
    phys = {"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4}
    dummy = ctypes.c_void_p(256)
    big = nsf._grid((1024, 1024, 1088))  # 32 x 128 x 17 tiles
    rc = L.nsf_diagnostics_noalloc(ctypes.byref(big), ctypes.byref(nsf._phys(phys)), 0, dummy,
                                   out, None)
    assert rc == nsf.EINVAL
    assert "65536" in L.nsf_last_error().decode()
    small = nsf._grid((16, 16, 16))
    rc = L.nsf_diagnostics_noalloc(ctypes.byref(small), ctypes.byref(nsf._phys(phys)), 0, None,
                                   out, None)
    assert rc == nsf.EINVAL
    rc = L.nsf_diagnostics_noalloc(ctypes.byref(small), ctypes.byref(nsf._phys(phys)), 0, dummy,
                                   None, None)
    assert rc == nsf.EINVAL


def test_store_set_workspace_and_validation(nsf):
    """The store set of SS / RS (nsf_tuning.gstore) sizes the gradient
    arrays: nine by default in 3D, three for the diagonal set, four in-plane
    ones on a single-plane grid; other values, other algorithms and the
    in-plane set on a 3D grid are rejected."""
    n = 32
    npts = n ** 3
    ra = nsf.workspace_bytes((n, n, n), "RA", "f64")
    for v in ("SS", "RS"):
        assert nsf.workspace_bytes((n, n, n), v, "f64") - ra >= 9 * npts * 8
        d3 = nsf.workspace_bytes((n, n, n), v, "f64", {"gstore": 3}) - ra
        assert 3 * npts * 8 <= d3 < 4 * npts * 8
        assert nsf.workspace_bytes((n, n, n), v, "f64", {"gstore": 9}) - ra >= 9 * npts * 8
    p2 = 40 * 36
    ra2 = nsf.workspace_bytes((40, 36, 1), "RA", "f64")
    ss2 = nsf.workspace_bytes((40, 36, 1), "SS", "f64") - ra2
    assert 4 * p2 * 8 <= ss2 < 5 * p2 * 8
    assert nsf.workspace_bytes((40, 36, 1), "SS", "f64", {"gstore": 9}) - ra2 >= 9 * p2 * 8
    for shape, v, tune in (((n, n, n), "SS", {"gstore": 4}), ((n, n, n), "SS", {"gstore": 5}),
                           ((n, n, n), "SN", {"gstore": 3}), ((n, n, n), "BL", {"gstore": 9})):
        with pytest.raises(nsf.NsfError) as ei:
            nsf.workspace_bytes(shape, v, "f64", tune)
        assert ei.value.code == nsf.EINVAL


def test_tune_cache_load_skips_invalid_lines(nsf, tmp_path):
    """nsf_tune_load keeps only lines that name a configuration the library
    runs on their grid."""
    base = ('{"arch": "gfx950", "nx": 48, "ny": 40, "nz": 36, "precision": 0, "variant": %d, '
            '"block_x": 32, "block_y": %d, "zchunk": %d, "fuse": %d, "naive": 0, "gstore": %d, '
            '"pt_rhs_per_s": 1e9, "parity_rel_err": 1e-14}')
    lines = [base % (3, 16, 32, 1, 0),   # SN fused: valid
             base % (7, 16, 32, 0, 0),   # no such algorithm
             base % (3, 12, 32, 1, 0),   # tile height 12
             base % (3, 16, 99, 1, 0),   # z-chunk beyond the grid
             base % (4, 16, 32, 1, 0),   # RS has no fused form
             base % (2, 16, 32, 0, 4),   # in-plane store set on a 3D grid
             base % (2, 16, 32, 0, 3)]   # SS, diagonal store set: valid
    path = tmp_path / "cache.jsonl"
    path.write_text("\n".join(lines) + "\n")
    assert nsf.tune_load(str(path)) == 2
    got = nsf.tune_get((48, 40, 36), "f64")
    assert got["variant"] == "SS" and got["tune"]["gstore"] == 3


def test_autotune_workspace_queries(nsf):
    """The autotuners take their device buffers from the caller: the size
    queries cover seven states (nine in single precision) and the largest
    candidate's work, or five ensemble states and the batch work area."""
    L = nsf.lib()
    n = 24
    npts = n ** 3
    g = nsf._grid((n, n, n))
    got = {}
    for prec in ("f64", "f32"):
        b = ctypes.c_size_t(0)
        assert L.nsf_autotune_workspace_bytes(ctypes.byref(g), nsf._precision(prec), 0,
                                              ctypes.byref(b)) == 0
        got[prec] = b.value
    bl = nsf.workspace_bytes((n, n, n), "BL", "f64")
    assert got["f64"] >= 3 * 5 * npts * 8 + 4 * 5 * npts * 8 + bl
    assert got["f32"] >= 3 * 5 * npts * 4 + 6 * 5 * npts * 8
    quick = ctypes.c_size_t(0)
    assert L.nsf_autotune_workspace_bytes(ctypes.byref(g), 0, nsf.TUNE_QUICK,
                                          ctypes.byref(quick)) == 0
    assert quick.value < got["f64"]  # no BL candidate: a smaller work area
    assert L.nsf_autotune_workspace_bytes(None, 0, 0, ctypes.byref(quick)) == nsf.EINVAL
    assert L.nsf_autotune_workspace_bytes(ctypes.byref(g), 7, 0, ctypes.byref(quick)) == nsf.EINVAL
    insts = [(16, 16, 16), (24, 24, 24)]
    grids = (nsf.Grid * 2)(*[nsf._grid(s) for s in insts])
    bb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert L.nsf_batch_autotune_workspace_bytes(2, grids, 0, ctypes.byref(bb)) == 0
    assert L.nsf_batch_workspace_bytes(2, grids, 0, ctypes.byref(wb)) == 0
    pts = sum(s[0] ** 3 for s in insts)
    assert bb.value >= 5 * 5 * pts * 8 + wb.value
    assert L.nsf_batch_autotune_workspace_bytes(0, grids, 0, ctypes.byref(bb)) == nsf.EINVAL


def test_autotune_rejects_a_small_workspace(nsf):
    """Checked before any device work: a workspace below the query's size
    is NSF_EWORKSPACE."""
    L = nsf.lib()
    g = nsf._grid((16, 16, 16))
    phys = nsf._phys({"Re": 1600.0, "Ma": 0.1, "Pr": 0.71, "gamma": 1.4})
    need = ctypes.c_size_t(0)
    assert L.nsf_autotune_workspace_bytes(ctypes.byref(g), 0, 0, ctypes.byref(need)) == 0
    r = nsf.TuneResult()
    rc = L.nsf_autotune(ctypes.byref(g), ctypes.byref(phys), 0, 0, 1, None,
                        ctypes.c_void_p(256), need.value - 1, ctypes.byref(r), None)
    assert rc == nsf.EWORKSPACE
