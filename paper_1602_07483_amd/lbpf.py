"""ctypes binding of the C ABI declared in include/lbpf.h.

Argument marshalling only: every step of the time step runs in the HIP
kernels of liblbpf.so.  There is no CPU fallback; importing this module
raises if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbpf.so")

LBPF_OK, LBPF_EINVAL, LBPF_ENOMEM, LBPF_EDEVICE, LBPF_EUNSTABLE, LBPF_ESTATE, LBPF_EIO = 0, -1, -2, -3, -4, -5, -6
LBPF_D3Q7, LBPF_D3Q15, LBPF_D3Q19 = 7, 15, 19
LBPF_WALL_NOFLUX, LBPF_WALL_SYMMETRY = 0, 1
LBPF_F32, LBPF_F16_DEV, LBPF_BF16_DEV, LBPF_F64 = 0, 1, 2, 3
LBPF_ANISO_CUBIC, LBPF_ANISO_K41K61 = 0, 1

STORAGE = {"f32": LBPF_F32, "f16": LBPF_F16_DEV, "bf16": LBPF_BF16_DEV, "f64": LBPF_F64}
_POP_DTYPE = {LBPF_F32: np.uint32, LBPF_F16_DEV: np.uint16, LBPF_BF16_DEV: np.uint16,
              LBPF_F64: np.uint64}


class lbpf_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lattice", ctypes.c_int32), ("wall", ctypes.c_int32 * 6),
                ("storage", ctypes.c_int32), ("lattice_ut", ctypes.c_int32)]


class lbpf_params(ctypes.Structure):
    _fields_ = [("dx", ctypes.c_double), ("dt", ctypes.c_double),
                ("W0", ctypes.c_double), ("tau0", ctypes.c_double),
                ("lam", ctypes.c_double), ("Mcinf", ctypes.c_double),
                ("k", ctypes.c_double), ("D", ctypes.c_double), ("kappa", ctypes.c_double),
                ("aniso", ctypes.c_int32), ("eps", ctypes.c_double), ("delta", ctypes.c_double),
                ("reduce_every", ctypes.c_int32), ("centre", ctypes.c_double * 3),
                ("vel", ctypes.c_double * 3), ("skip_U", ctypes.c_int32),
                ("skip_theta", ctypes.c_int32)]


class lbpf_reductions(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("solid_fraction", ctypes.c_double),
                ("solute_mass", ctypes.c_double), ("enthalpy", ctypes.c_double),
                ("tip", ctypes.c_double * 3), ("phi_min", ctypes.c_double),
                ("phi_max", ctypes.c_double), ("nonfinite", ctypes.c_double),
                ("sum_U", ctypes.c_double), ("sum_phi", ctypes.c_double),
                ("tip_vel", ctypes.c_double * 3)]

    def as_dict(self):
        return {"step": self.step, "solid_fraction": self.solid_fraction,
                "solute_mass": self.solute_mass, "enthalpy": self.enthalpy,
                "tip": tuple(self.tip), "phi_min": self.phi_min, "phi_max": self.phi_max,
                "nonfinite": self.nonfinite, "sum_U": self.sum_U, "sum_phi": self.sum_phi,
                "tip_vel": tuple(self.tip_vel)}


# Exported symbols, in header order (a CPU test checks each one is exported).
FIELD_TYPE = {"f32": 0, "f64": 1}

SYMBOLS = ["lbpf_create", "lbpf_destroy", "lbpf_set_fields", "lbpf_step", "lbpf_sync",
           "lbpf_read", "lbpf_history", "lbpf_read_populations", "lbpf_write_populations",
           "lbpf_read_populations_f64",
           "lbpf_debug_stream_only", "lbpf_set_velocity_field", "lbpf_set_timing",
           "lbpf_kernel_times",
           "lbpf_set_launch", "lbpf_get_launch", "lbpf_set_kernel_launch",
           "lbpf_get_kernel_launch", "lbpf_autotune", "lbpf_autotune_cached",
           "lbpf_storage_bytes", "lbpf_bench_copy", "lbpf_bench_bandwidth", "lbpf_reduce_fields_noalloc",
           "lbpf_last_error", "lbpf_set_graph",
           "lbpf_batch_create", "lbpf_batch_domain", "lbpf_batch_set_graph", "lbpf_batch_step",
           "lbpf_batch_set_launch", "lbpf_batch_get_launch", "lbpf_batch_autotune",
           "lbpf_batch_sync", "lbpf_batch_destroy", "lbpf_batch_last_error",
           "lbpf_set_fields_device", "lbpf_read_fields_device"]


class LbpfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lbpf status %d: %s" % (status, msg))
        self.status = status


def load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbpf.so is not built (run python -m paper_1602_07483_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, dp = ctypes.c_void_p, P(ctypes.c_double)
    sig = {
        "lbpf_create": ([P(lbpf_grid), P(lbpf_params), vp, P(vp)], ctypes.c_int),
        "lbpf_destroy": ([vp], ctypes.c_int),
        "lbpf_set_fields": ([vp, dp, dp, dp], ctypes.c_int),
        "lbpf_set_fields_device": ([vp, vp, vp, vp, ctypes.c_int32], ctypes.c_int),
        "lbpf_read_fields_device": ([vp, vp, vp, vp, ctypes.c_int32], ctypes.c_int),
        "lbpf_step": ([vp, ctypes.c_int64], ctypes.c_int),
        "lbpf_sync": ([vp], ctypes.c_int),
        "lbpf_read": ([vp, dp, dp, dp, P(lbpf_reductions)], ctypes.c_int),
        "lbpf_history": ([vp, P(lbpf_reductions), ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "lbpf_read_populations": ([vp, ctypes.c_int32, vp], ctypes.c_int),
        "lbpf_write_populations": ([vp, ctypes.c_int32, vp], ctypes.c_int),
        "lbpf_read_populations_f64": ([vp, ctypes.c_int32, dp], ctypes.c_int),
        "lbpf_debug_stream_only": ([vp, ctypes.c_int64], ctypes.c_int),
        "lbpf_set_velocity_field": ([vp, dp, dp, dp], ctypes.c_int),
        "lbpf_set_timing": ([vp, ctypes.c_int32], ctypes.c_int),
        "lbpf_kernel_times": ([vp, dp, P(ctypes.c_int64)], ctypes.c_int),
        "lbpf_set_launch": ([vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                            ctypes.c_int),
        "lbpf_get_launch": ([vp, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32),
                             P(ctypes.c_int32)], ctypes.c_int),
        "lbpf_set_kernel_launch": ([vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32], ctypes.c_int),
        "lbpf_get_kernel_launch": ([vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32),
                                    P(ctypes.c_int32), P(ctypes.c_int32)], ctypes.c_int),
        "lbpf_autotune": ([vp, ctypes.c_int32, dp], ctypes.c_int),
        "lbpf_autotune_cached": ([vp, ctypes.c_int32, ctypes.c_char_p, P(ctypes.c_int32), dp], ctypes.c_int),
        "lbpf_storage_bytes": ([ctypes.c_int32], ctypes.c_int32),
        "lbpf_bench_copy": ([vp, vp, ctypes.c_int64, vp], ctypes.c_int),
        "lbpf_reduce_fields_noalloc": ([vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        P(ctypes.c_double), vp, vp], ctypes.c_int),
        "lbpf_bench_bandwidth": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp,
                                  ctypes.c_int64, vp], ctypes.c_int),
        "lbpf_last_error": ([vp], ctypes.c_char_p),
        "lbpf_set_graph": ([vp, ctypes.c_int32], ctypes.c_int),
        "lbpf_batch_create": ([ctypes.c_int32, P(lbpf_grid), P(lbpf_params), vp, P(vp)], ctypes.c_int),
        "lbpf_batch_domain": ([vp, ctypes.c_int32], vp),
        "lbpf_batch_set_graph": ([vp, ctypes.c_int32], ctypes.c_int),
        "lbpf_batch_step": ([vp, ctypes.c_int64], ctypes.c_int),
        "lbpf_batch_set_launch": ([vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                                  ctypes.c_int),
        "lbpf_batch_get_launch": ([vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)],
                                  ctypes.c_int),
        "lbpf_batch_autotune": ([vp, ctypes.c_int32, dp], ctypes.c_int),
        "lbpf_batch_sync": ([vp], ctypes.c_int),
        "lbpf_batch_destroy": ([vp], ctypes.c_int),
        "lbpf_batch_last_error": ([vp], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def lbpf_storage_bytes(storage):
    return lib().lbpf_storage_bytes(int(storage))


def lbpf_bench_copy(dst_ptr, src_ptr, nbytes, stream_ptr=0):
    return lib().lbpf_bench_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr),
                                 int(nbytes), ctypes.c_void_p(stream_ptr))


def lbpf_bench_bandwidth(mode, width, nontemporal, blocks, dst_ptr, src_ptr, nbytes, stream_ptr=0):
    return lib().lbpf_bench_bandwidth(int(mode), int(width), int(nontemporal), int(blocks),
                                      ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr or 0),
                                      int(nbytes), ctypes.c_void_p(stream_ptr))


def lbpf_reduce_fields_noalloc(phi_ptr, U_ptr, theta_ptr, dtype, nx, ny, nz, k, dx, centre, rec_ptr,
                               stream_ptr=0):
    """Reduction record of device fields into 12 device doubles at rec_ptr,
    with no allocation (see include/lbpf.h)."""
    c = (ctypes.c_double * 3)(*[float(v) for v in centre])
    return lib().lbpf_reduce_fields_noalloc(ctypes.c_void_p(phi_ptr), ctypes.c_void_p(U_ptr),
                                            ctypes.c_void_p(theta_ptr), int(dtype), int(nx), int(ny), int(nz),
                                            float(k), float(dx), c, ctypes.c_void_p(rec_ptr),
                                            ctypes.c_void_p(stream_ptr))


def make_structs(nx, ny, nz, lattice=19, walls=(0,) * 6, storage="f32", dx=1.0, dt=1.0,
                 W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15, D=2.0, kappa=20.0, aniso=0,
                 eps=0.05, delta=0.0, reduce_every=0, centre=(0.0, 0.0, 0.0),
                 vel=(0.0, 0.0, 0.0), skip_U=0, skip_theta=0, lattice_ut=0):
    """(lbpf_grid, lbpf_params) filled from keyword arguments."""
    g = lbpf_grid()
    g.nx, g.ny, g.nz, g.lattice = int(nx), int(ny), int(nz), int(lattice)
    for i, w in enumerate(walls):
        g.wall[i] = int(w)
    g.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    g.lattice_ut = int(lattice_ut)
    p = lbpf_params()
    p.dx, p.dt, p.W0, p.tau0 = dx, dt, W0, tau0
    p.lam, p.Mcinf, p.k, p.D, p.kappa = lam, Mcinf, k, D, kappa
    p.aniso, p.eps, p.delta = int(aniso), eps, delta
    p.reduce_every = int(reduce_every)
    for i in range(3):
        p.centre[i] = float(centre[i])
        p.vel[i] = float(vel[i])
    p.skip_U = int(skip_U)
    p.skip_theta = int(skip_theta)
    return g, p


class Solver:
    """One lbpf context.  Methods mirror the C entry points
    (lbpf_create/set_fields/step/read/...); arrays are numpy (nz, ny, nx)."""

    @classmethod
    def _wrap(cls, handle, grid, params, owner):
        self = cls.__new__(cls)
        self._lib = lib()
        self.grid, self.params = grid, params
        self.shape = (grid.nz, grid.ny, grid.nx)
        self.q = grid.lattice
        self.q_ut = grid.lattice_ut or grid.lattice
        self.storage = grid.storage
        self._h = ctypes.c_void_p(handle)
        self._owner = owner          # the batch keeps the memory; never destroyed here
        return self

    def __init__(self, nx, ny, nz, lattice=19, walls=(0,) * 6, storage="f32", dx=1.0, dt=1.0,
                 W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15, D=2.0, kappa=20.0, aniso=0,
                 eps=0.05, delta=0.0, reduce_every=0, centre=(0.0, 0.0, 0.0),
                 vel=(0.0, 0.0, 0.0), skip_U=0, skip_theta=0, lattice_ut=0, stream=0):
        self._lib = lib()
        self._owner = None
        g, p = make_structs(nx, ny, nz, lattice, walls, storage, dx, dt, W0, tau0, lam, Mcinf, k,
                            D, kappa, aniso, eps, delta, reduce_every, centre, vel, skip_U,
                            skip_theta, lattice_ut)
        self.grid, self.params = g, p
        self.shape = (int(nz), int(ny), int(nx))
        self.q = int(lattice)
        self.q_ut = int(lattice_ut) or int(lattice)
        self.storage = g.storage
        h = ctypes.c_void_p()
        st = self._lib.lbpf_create(ctypes.byref(g), ctypes.byref(p), ctypes.c_void_p(stream),
                                   ctypes.byref(h))
        if st != LBPF_OK:
            raise LbpfError(st, self._lib.lbpf_last_error(None).decode())
        self._h = h

    # -- helpers
    def _check(self, st):
        if st != LBPF_OK:
            raise LbpfError(st, self._lib.lbpf_last_error(self._h).decode())
        return st

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owner", None) is None:
            self._lib.lbpf_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C entry points
    def set_fields(self, phi, U, theta):
        a = [np.ascontiguousarray(v, dtype=np.float64).reshape(self.shape) for v in (phi, U, theta)]
        self._check(self._lib.lbpf_set_fields(self._h, _dptr(a[0]), _dptr(a[1]), _dptr(a[2])))

    def step(self, n=1):
        self._check(self._lib.lbpf_step(self._h, int(n)))

    def sync(self, check=True):
        st = self._lib.lbpf_sync(self._h)
        return self._check(st) if check else st

    def read(self, reductions=True, check=True):
        """(phi, U, theta, reductions-dict or None); raises on EUNSTABLE if check."""
        out = [np.empty(self.shape) for _ in range(3)]
        red = lbpf_reductions() if reductions else None
        st = self._lib.lbpf_read(self._h, _dptr(out[0]), _dptr(out[1]), _dptr(out[2]),
                                 ctypes.byref(red) if red is not None else None)
        if check:
            self._check(st)
        return out[0], out[1], out[2], (red.as_dict() if red is not None else None)

    def set_fields_device(self, phi_ptr, U_ptr, theta_ptr, dtype="f32"):
        """Fields from device arrays (integer device addresses, [nz][ny][nx],
        element type dtype 'f32' or 'f64')."""
        self._check(self._lib.lbpf_set_fields_device(
            self._h, ctypes.c_void_p(phi_ptr), ctypes.c_void_p(U_ptr), ctypes.c_void_p(theta_ptr),
            FIELD_TYPE[dtype]))

    def read_fields_device(self, phi_ptr, U_ptr, theta_ptr, dtype="f32"):
        """Copy the fields into device arrays (0 skips one); asynchronous on
        the solver's stream."""
        self._check(self._lib.lbpf_read_fields_device(
            self._h, ctypes.c_void_p(phi_ptr or None), ctypes.c_void_p(U_ptr or None),
            ctypes.c_void_p(theta_ptr or None), FIELD_TYPE[dtype]))

    def read_status(self):
        red = lbpf_reductions()
        st = self._lib.lbpf_read(self._h, None, None, None, ctypes.byref(red))
        return st, red.as_dict()

    def history(self, max_records=8192):
        buf = (lbpf_reductions * max_records)()
        cnt = ctypes.c_int32()
        self._check(self._lib.lbpf_history(self._h, buf, int(max_records), ctypes.byref(cnt)))
        return [buf[i].as_dict() for i in range(cnt.value)]

    def lattice_of(self, field):
        """Directions of field's populations (0: phi; 1, 2: U, theta)."""
        return self.q if int(field) == 0 else self.q_ut

    def read_populations(self, field):
        out = np.empty((self.lattice_of(field),) + self.shape, dtype=_POP_DTYPE[self.storage])
        self._check(self._lib.lbpf_read_populations(self._h, int(field),
                                                    out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def read_populations_f64(self, field):
        out = np.empty((self.lattice_of(field),) + self.shape)
        self._check(self._lib.lbpf_read_populations_f64(self._h, int(field), _dptr(out)))
        return out

    def write_populations(self, field, arr):
        a = np.ascontiguousarray(arr).view(_POP_DTYPE[self.storage]).reshape((self.lattice_of(field),) + self.shape)
        self._check(self._lib.lbpf_write_populations(self._h, int(field),
                                                     a.ctypes.data_as(ctypes.c_void_p)))

    def debug_stream_only(self, n=1):
        self._check(self._lib.lbpf_debug_stream_only(self._h, int(n)))

    def set_velocity_field(self, vx, vy, vz):
        """Per-node advective velocity of theta, arrays of shape (nz, ny, nx);
        None for all three removes it."""
        if vx is None and vy is None and vz is None:
            self._check(self._lib.lbpf_set_velocity_field(self._h, None, None, None))
            return
        arr = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(self.shape))
               for v in (vx, vy, vz)]
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.lbpf_set_velocity_field(self._h, *[a.ctypes.data_as(dp) for a in arr]))

    def set_timing(self, enable=True):
        self._check(self._lib.lbpf_set_timing(self._h, 1 if enable else 0))

    def set_graph(self, steps_per_graph):
        self._check(self._lib.lbpf_set_graph(self._h, int(steps_per_graph)))

    def set_launch(self, tile_x, tile_y, zslab, xcd_remap=1):
        self._check(self._lib.lbpf_set_launch(self._h, int(tile_x), int(tile_y), int(zslab),
                                              int(xcd_remap)))

    def get_launch(self):
        """(tile_x, tile_y, zslab, xcd_remap) of k_ut."""
        a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.lbpf_get_launch(self._h, ctypes.byref(a), ctypes.byref(b),
                                              ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def set_kernel_launch(self, kernel, tile_x, tile_y, zslab, xcd_remap=1):
        """kernel 0: k_phi, 1: k_ut."""
        self._check(self._lib.lbpf_set_kernel_launch(self._h, int(kernel), int(tile_x), int(tile_y),
                                                     int(zslab), int(xcd_remap)))

    def get_kernel_launch(self, kernel):
        a, b, c, d = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.lbpf_get_kernel_launch(self._h, int(kernel), ctypes.byref(a),
                                                     ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return a.value, b.value, c.value, d.value

    def launches(self):
        """{"k_phi": (tx, ty, zslab, remap), "k_ut": (...)}."""
        return {"k_phi": self.get_kernel_launch(0), "k_ut": self.get_kernel_launch(1)}

    def autotune(self, steps_per_candidate=10):
        """Returns ({"k_phi": launch, "k_ut": launch}, best ms per step)."""
        best = ctypes.c_double()
        self._check(self._lib.lbpf_autotune(self._h, int(steps_per_candidate), ctypes.byref(best)))
        return self.launches(), best.value

    def autotune_cached(self, cache_path, steps_per_candidate=10):
        """lbpf_autotune_cached: returns (launches, best ms per step, hit)."""
        best, hit = ctypes.c_double(), ctypes.c_int32()
        self._check(self._lib.lbpf_autotune_cached(self._h, int(steps_per_candidate),
                                                   os.fsencode(cache_path), ctypes.byref(hit),
                                                   ctypes.byref(best)))
        return self.launches(), best.value, bool(hit.value)

    def kernel_times(self):
        ms = (ctypes.c_double * 3)()
        n = (ctypes.c_int64 * 3)()
        self._check(self._lib.lbpf_kernel_times(self._h, ms, n))
        return list(ms), list(n)


class Batch:
    """An ensemble of independent domains (lbpf_batch_*).  domains[i] is a
    Solver view of domain i for set_fields/read."""

    def __init__(self, specs, storage="f32", stream=0):
        self._lib = lib()
        n = len(specs)
        grids = (lbpf_grid * n)()
        params = (lbpf_params * n)()
        for i, kw in enumerate(specs):
            g, p = make_structs(storage=storage, **kw)
            grids[i], params[i] = g, p
        h = ctypes.c_void_p()
        st = self._lib.lbpf_batch_create(n, grids, params, ctypes.c_void_p(stream), ctypes.byref(h))
        if st != LBPF_OK:
            raise LbpfError(st, self._lib.lbpf_batch_last_error(None).decode())
        self._h = h
        self.domains = [Solver._wrap(self._lib.lbpf_batch_domain(h, i), grids[i], params[i], self)
                        for i in range(n)]

    def _check(self, st):
        if st != LBPF_OK:
            raise LbpfError(st, self._lib.lbpf_batch_last_error(self._h).decode())

    def step(self, n=1):
        self._check(self._lib.lbpf_batch_step(self._h, int(n)))

    def sync(self):
        self._check(self._lib.lbpf_batch_sync(self._h))

    def set_graph(self, steps_per_graph):
        self._check(self._lib.lbpf_batch_set_graph(self._h, int(steps_per_graph)))

    def set_launch(self, kernel, tile_x, tile_y, zslab):
        """kernel 0: k_phi, 1: k_ut (all domains)."""
        self._check(self._lib.lbpf_batch_set_launch(self._h, int(kernel), int(tile_x), int(tile_y), int(zslab)))

    def get_launch(self, kernel):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.lbpf_batch_get_launch(self._h, int(kernel), ctypes.byref(a), ctypes.byref(b),
                                                    ctypes.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, steps_per_candidate=4):
        """Returns ({"k_phi": (tx, ty, zslab), "k_ut": ...}, best ms per batch step)."""
        best = ctypes.c_double()
        self._check(self._lib.lbpf_batch_autotune(self._h, int(steps_per_candidate), ctypes.byref(best)))
        return {"k_phi": self.get_launch(0), "k_ut": self.get_launch(1)}, best.value

    def close(self):
        if getattr(self, "_h", None):
            for d in self.domains:
                d._h = None
            self._lib.lbpf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def problem_kwargs(problem):
    kw = problem.model_kwargs()
    kw.update(nx=problem.nx, ny=problem.ny, nz=problem.nz, reduce_every=problem.reduce_every,
              centre=problem.centre())
    return kw


def solver_for(problem, storage="f32", stream=0, **over):
    """Solver configured from an inputs.Problem (keyword overrides allowed)."""
    kw = problem.model_kwargs()
    kw.update(reduce_every=problem.reduce_every, centre=problem.centre())
    kw.update(over)
    return Solver(problem.nx, problem.ny, problem.nz, storage=storage, stream=stream, **kw)
