"""The allocation-free reduction entry point (lbpf_reduce_fields_noalloc)
against the context reduction of lbpf_read, through the C ABI: two calls in
a row, the second on a smaller domain, each equal bit for bit to the record
lbpf_read computes for the same fields (same kernels, same grid)."""
import ctypes
import math

import numpy as np
import pytest

from paper_1602_07483_amd import lbpf
from paper_1602_07483_amd.inputs import Problem, NOFLUX, SYMMETRY

pytestmark = pytest.mark.gpu

KEYS = ("solid_fraction", "solute_mass", "enthalpy")


def _hip():
    h = ctypes.CDLL("libamdhip64.so.7")
    h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    h.hipFree.argtypes = [ctypes.c_void_p]
    h.hipDeviceSynchronize.argtypes = []
    return h


def _problem(nx, ny, nz, seed):
    walls = (SYMMETRY, NOFLUX, NOFLUX, SYMMETRY, SYMMETRY, NOFLUX)
    return Problem("noalloc-%d" % nx, nx, ny, nz, 19, walls, dt=0.15, eps=0.05,
                   centres=[(-0.5, ny - 0.5, -0.5), (nx * 0.6, ny * 0.4, nz * 0.5)], radius=5.0,
                   U0=-0.5, theta0=-0.5, noise_amp=1e-3, noise_seed=seed)


def _equal(a, b):
    return (math.isnan(a) and math.isnan(b)) or a == b


@pytest.mark.parametrize("storage,dtype", [("f32", 0), ("f64", 1)])
def test_noalloc_reduction_matches_context_reduction(storage, dtype):
    hip = _hip()
    esize = 4 if dtype == 0 else 8
    for nx, ny, nz, seed in ((48, 40, 36, 11), (20, 17, 9, 12)):   # second call: a smaller input
        pb = _problem(nx, ny, nz, seed)
        s = lbpf.solver_for(pb, storage=storage)
        s.set_fields(*pb.initial_fields())
        s.step(30)
        ref = s.read()[3]                       # lbpf_read: the context's own reduction
        n = nx * ny * nz
        bufs = []
        for _ in range(3):
            p = ctypes.c_void_p()
            assert hip.hipMalloc(ctypes.byref(p), n * esize) == 0
            bufs.append(p)
        rec = ctypes.c_void_p()
        assert hip.hipMalloc(ctypes.byref(rec), 12 * 8) == 0
        try:
            s.read_fields_device(*(b.value for b in bufs), dtype="f32" if dtype == 0 else "f64")
            s.sync()
            st = lbpf.lbpf_reduce_fields_noalloc(bufs[0].value, bufs[1].value, bufs[2].value, dtype,
                                                 nx, ny, nz, pb.k, pb.dx, pb.centre(), rec.value, 0)
            assert st == lbpf.LBPF_OK, lbpf.lib().lbpf_last_error(None)
            assert hip.hipDeviceSynchronize() == 0
            out = np.zeros(12)
            assert hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), rec, 12 * 8, 2) == 0
        finally:
            for b in bufs + [rec]:
                hip.hipFree(b)
            s.close()
        print("%dx%dx%d %s: solid %.17g mass %.17g tip %s" % (nx, ny, nz, storage, out[1], out[2], out[4:7]))
        assert out[0] == 0.0
        for i, key in enumerate(KEYS):
            assert out[1 + i] == ref[key], key
        for a in range(3):
            assert _equal(out[4 + a], ref["tip"][a]), ("tip", a)
        assert out[7] == ref["phi_min"] and out[8] == ref["phi_max"]
        assert out[9] == ref["nonfinite"] == 0.0
        assert out[10] == ref["sum_U"] and out[11] == ref["sum_phi"]
