"""The allocation-free diagnostics entry point (nsf_diagnostics_noalloc),
called through the C ABI, against nsf_diagnostics on the same states: the
same kernels and the same fixed-order reduction, so the sixteen outputs must
agree bitwise. Two calls in a row, the second on a smaller grid, so stale
partials of the first call in the shared scratch would show."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _state(nsf, W, shape, precision, seed):
    s = nsf.Solver(shape, W.TGV_PHYS, "RA", precision)
    s.init(W.tgv_pointwise(seed, 1e-3))
    s.step(0.01, 1)  # a state with no symmetry left
    torch.cuda.synchronize()
    return s


def _call_noalloc(nsf, shape, phys, precision, q):
    L = nsf.lib()
    out = (ctypes.c_double * nsf.NDIAG)()
    rc = L.nsf_diagnostics_noalloc(ctypes.byref(nsf._grid(shape)), ctypes.byref(nsf._phys(phys)),
                                   nsf._precision(precision), ctypes.c_void_p(q.data_ptr()), out,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, nsf.lib().nsf_last_error().decode()
    return np.array(out[:])


def _call_work(nsf, shape, phys, precision, q, work):
    L = nsf.lib()
    out = (ctypes.c_double * nsf.NDIAG)()
    rc = L.nsf_diagnostics(ctypes.byref(nsf._grid(shape)), ctypes.byref(nsf._phys(phys)),
                           nsf._precision(precision), ctypes.c_void_p(q.data_ptr()),
                           ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(),
                           out, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, nsf.lib().nsf_last_error().decode()
    return np.array(out[:])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_noalloc_matches_diagnostics_two_calls(precision):
    from paper_1610_09146_amd import nsf, workloads as W
    phys = W.TGV_PHYS
    # second grid smaller than the first, with ragged tiles in x, y and z
    for shape, seed in (((72, 44, 130), 11), ((40, 20, 13), 12)):
        print(f"noalloc {precision} {shape}", flush=True)
        s = _state(nsf, W, shape, precision, seed)
        got = _call_noalloc(nsf, shape, phys, precision, s.q)
        ref = _call_work(nsf, shape, phys, precision, s.q, s.work)
        assert np.array_equal(got, ref), (shape, got - ref)
        assert got[14] == 0 and abs(got[2] - ref[2]) == 0
        del s
        torch.cuda.empty_cache()


def test_noalloc_binding_and_repeat():
    from paper_1610_09146_amd import nsf, workloads as W
    shape = (33, 17, 9)
    s = _state(nsf, W, shape, "f64", 5)
    a = nsf.diagnostics_noalloc(shape, W.TGV_PHYS, "f64", s.q)
    b = nsf.diagnostics_noalloc(shape, W.TGV_PHYS, "f64", s.q)
    c = s.diagnostics()
    assert np.array_equal(a, b) and np.array_equal(a, c)
