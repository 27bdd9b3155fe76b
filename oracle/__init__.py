"""Plain FP64 CPU oracle for the lattice-Boltzmann phase-field scheme of
Cartalade, Younsi & Plapp (arXiv:1602.07483).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and
by the CPU-baseline leg of the benchmark.  The product library never imports
it.  The arithmetic lives in ``lbpf_oracle.c``; this module only marshals
numpy arrays through ctypes.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbpf_oracle.so")

WALL_NOFLUX = 0
WALL_SYMMETRY = 1
ANISO_CUBIC = 0
ANISO_K41K61 = 1

R_SOLID, R_MASS, R_ENTHALPY, R_TIPX, R_TIPY, R_TIPZ, R_PHIMIN, R_PHIMAX, \
    R_NONFINITE, R_SUMU, R_SUMPHI, R_COUNT = range(12)


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lattice", ctypes.c_int32), ("wall", ctypes.c_int32 * 6),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("W0", ctypes.c_double), ("tau0", ctypes.c_double),
        ("lam", ctypes.c_double), ("Mcinf", ctypes.c_double),
        ("k", ctypes.c_double), ("D", ctypes.c_double), ("kappa", ctypes.c_double),
        ("aniso", ctypes.c_int32), ("eps", ctypes.c_double), ("delta", ctypes.c_double),
        ("vel", ctypes.c_double * 3),
        ("skip_theta", ctypes.c_int32),
        ("lattice_ut", ctypes.c_int32),
        ("skip_U", ctypes.c_int32),
        ("grad_stencil", ctypes.c_int32),
    ]


class OrcParamsF32(ctypes.Structure):
    """orc_params of the single-precision build (every double is a float)."""
    _fields_ = [(n, ctypes.c_float if t is ctypes.c_double else
                 (ctypes.c_float * 3 if n == "vel" else t)) for n, t in OrcParams._fields_]


class FdoParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double), ("W0", ctypes.c_double), ("tau0", ctypes.c_double),
        ("lam", ctypes.c_double), ("Mcinf", ctypes.c_double), ("k", ctypes.c_double),
        ("D", ctypes.c_double), ("kappa", ctypes.c_double),
        ("aniso", ctypes.c_int32), ("eps", ctypes.c_double), ("delta", ctypes.c_double),
        ("skip_theta", ctypes.c_int32), ("stencil", ctypes.c_int32),
        ("skip_U", ctypes.c_int32),
    ]


_lib = None
_lib_f32 = None


def _load_f32():
    """The single-precision build of the LB oracle (liblbpf_oracle_f32.so)."""
    global _lib_f32
    if _lib_f32 is not None:
        return _lib_f32
    path = os.path.join(_HERE, "liblbpf_oracle_f32.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    fp = P(ctypes.c_float)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [P(OrcParamsF32)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_init.argtypes = [ctypes.c_void_p, fp, fp, fp]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.orc_fields.argtypes = [ctypes.c_void_p, fp, fp, fp]
    _lib_f32 = lib
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [P(OrcParams)]
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_init.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.orc_set_velocity_field.restype = ctypes.c_int
    lib.orc_set_velocity_field.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.orc_stream_only.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    lib.orc_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.orc_get_pops.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    lib.orc_set_pops.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
    lib.orc_reduce.argtypes = [ctypes.c_void_p, dp, dp]
    lib.orc_step_count.restype = ctypes.c_int64
    lib.orc_step_count.argtypes = [ctypes.c_void_p]
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_num_threads.argtypes = []
    lib.orc_lattice.argtypes = [ctypes.c_int, P(ctypes.c_int32), dp, dp, dp, dp]
    lib.orc_anisotropy.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   dp, dp, dp]
    lib.orc_geq.argtypes = [ctypes.c_int, ctypes.c_double, dp, ctypes.c_double, dp]
    lib.orc_heq.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                            ctypes.c_double, dp]
    lib.fdo_create.restype = ctypes.c_void_p
    lib.fdo_create.argtypes = [P(FdoParams)]
    lib.fdo_destroy.argtypes = [ctypes.c_void_p]
    lib.fdo_set.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.fdo_get.argtypes = [ctypes.c_void_p, dp, dp, dp]
    lib.fdo_step.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int64]
    _lib = lib
    return lib


def num_threads():
    """OpenMP threads used by the oracle's loops."""
    return int(_load().orc_num_threads())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice(q):
    """(e [q,3] int, w, A, B, e2) as typed in the oracle."""
    lib = _load()
    e = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q); A = np.zeros(q); B = np.zeros(q); e2 = ctypes.c_double()
    rc = lib.orc_lattice(q, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         _dptr(w), _dptr(A), _dptr(B), ctypes.byref(e2))
    if rc:
        raise ValueError("unsupported lattice %r" % q)
    return e, w, A, B, e2.value


def anisotropy(p, aniso=ANISO_CUBIC, eps=0.05, delta=0.0):
    """a_s and the vector N for the gradient p (3 doubles)."""
    lib = _load()
    p = _f64(p)
    a = ctypes.c_double()
    N = np.zeros(3)
    lib.orc_anisotropy(aniso, eps, delta, _dptr(p), ctypes.byref(a), _dptr(N))
    return a.value, N


def geq(q, phi, N, cphi):
    lib = _load()
    out = np.zeros(q)
    lib.orc_geq(q, float(phi), _dptr(_f64(N)), float(cphi), _dptr(out))
    return out


def heq(q, U, r, J, dt_over_dx):
    lib = _load()
    out = np.zeros(q)
    lib.orc_heq(q, float(U), float(r), _dptr(_f64(J)), float(dt_over_dx), _dptr(out))
    return out


class Oracle:
    """One domain advanced by the FP64 oracle.  Fields are numpy arrays of
    shape (nz, ny, nx); populations (Q, nz, ny, nx)."""

    def __init__(self, nx, ny, nz, lattice=19, walls=(0,) * 6, dx=1.0, dt=1.0,
                 W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15, D=2.0, kappa=20.0,
                 aniso=ANISO_CUBIC, eps=0.05, delta=0.0, vel=(0.0, 0.0, 0.0), skip_theta=0,
                 lattice_ut=0, skip_U=0, grad_stencil=0):
        lib = _load()
        p = OrcParams()
        p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
        p.lattice = int(lattice)
        for i, wv in enumerate(walls):
            p.wall[i] = int(wv)
        p.dx, p.dt, p.W0, p.tau0 = dx, dt, W0, tau0
        p.lam, p.Mcinf, p.k, p.D, p.kappa = lam, Mcinf, k, D, kappa
        p.aniso, p.eps, p.delta = int(aniso), eps, delta
        for a in range(3):
            p.vel[a] = float(vel[a])
        p.skip_theta = int(skip_theta)
        p.lattice_ut = int(lattice_ut)
        p.skip_U = int(skip_U)
        p.grad_stencil = int(grad_stencil)
        self.params = p
        self.shape = (int(nz), int(ny), int(nx))
        self.q = int(lattice)
        self.q_ut = int(lattice_ut) or self.q
        self._h = lib.orc_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, phi, U, theta):
        a = [_f64(v).reshape(self.shape) for v in (phi, U, theta)]
        self._lib.orc_init(self._h, _dptr(a[0]), _dptr(a[1]), _dptr(a[2]))

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    def set_velocity_field(self, vx, vy, vz):
        """Per-node advective velocity of the heat equation, arrays of shape
        (nz, ny, nx); None for all three clears it (the uniform vel applies)."""
        if vx is None and vy is None and vz is None:
            rc = self._lib.orc_set_velocity_field(self._h, None, None, None)
        else:
            self._vf = [_f64(v).reshape(self.shape) for v in (vx, vy, vz)]
            rc = self._lib.orc_set_velocity_field(self._h, *[_dptr(a) for a in self._vf])
        if rc != 0:
            raise ValueError("orc_set_velocity_field failed")

    def stream_only(self, n=1):
        self._lib.orc_stream_only(self._h, int(n))

    @property
    def steps(self):
        return self._lib.orc_step_count(self._h)

    def fields(self):
        out = [np.zeros(self.shape) for _ in range(3)]
        self._lib.orc_fields(self._h, _dptr(out[0]), _dptr(out[1]), _dptr(out[2]))
        return out

    def pops(self, field):
        out = np.zeros((self.q if field == 0 else self.q_ut,) + self.shape)
        self._lib.orc_get_pops(self._h, int(field), _dptr(out))
        return out

    def set_pops(self, field, arr):
        a = _f64(arr).reshape((self.q if field == 0 else self.q_ut,) + self.shape)
        self._lib.orc_set_pops(self._h, int(field), _dptr(a))

    def reduce(self, centre=(0.0, 0.0, 0.0)):
        out = np.zeros(R_COUNT)
        self._lib.orc_reduce(self._h, _dptr(_f64(centre)), _dptr(out))
        return out


class FDOracle:
    """The independent finite-difference discretisation (fd_oracle.c) of the
    same PDEs, explicit Euler with time step dt.  All walls carry zero flux
    (mirror and no-flux walls coincide for this discretisation).  stencil 6
    or 18: the paper's FD6 and FD18 Laplacians of the phase-field equation
    (18: isotropic interface only, eps = 0).  skip_U: pure substance, U held.
    It has no advection: a nonzero vel is an error."""

    def __init__(self, nx, ny, nz, dx=1.0, W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15,
                 D=2.0, kappa=20.0, aniso=ANISO_CUBIC, eps=0.05, delta=0.0, skip_theta=0,
                 stencil=6, skip_U=0, vel=(0.0, 0.0, 0.0), **_ignored):
        if any(float(v) != 0.0 for v in vel):
            raise ValueError("the finite-difference oracle has no advection (vel must be 0)")
        lib = _load()
        p = FdoParams()
        p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
        p.dx, p.W0, p.tau0, p.lam, p.Mcinf, p.k = dx, W0, tau0, lam, Mcinf, k
        p.D, p.kappa, p.aniso, p.eps, p.delta = D, kappa, int(aniso), eps, delta
        p.skip_theta = int(skip_theta)
        p.stencil = int(stencil)
        p.skip_U = int(skip_U)
        self.shape = (int(nz), int(ny), int(nx))
        self._h = lib.fdo_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("finite-difference oracle rejected the parameters")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.fdo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, phi, U, theta):
        a = [_f64(v).reshape(self.shape) for v in (phi, U, theta)]
        self._lib.fdo_set(self._h, _dptr(a[0]), _dptr(a[1]), _dptr(a[2]))

    def step(self, dt, n=1):
        self._lib.fdo_step(self._h, float(dt), int(n))

    def fields(self):
        out = [np.zeros(self.shape) for _ in range(3)]
        self._lib.fdo_get(self._h, _dptr(out[0]), _dptr(out[1]), _dptr(out[2]))
        return out


class OracleF32:
    """The LB oracle's algorithm with every double replaced by float (the
    single-precision build of the same source): test evidence of the error
    that FP32 state and arithmetic alone give the method after n steps, used
    to bound FP32 parity where the growing interface amplifies rounding.  It
    is compared with the FP64 oracle, never used as a reference."""

    def __init__(self, nx, ny, nz, lattice=19, walls=(0,) * 6, dx=1.0, dt=1.0,
                 W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15, D=2.0, kappa=20.0,
                 aniso=ANISO_CUBIC, eps=0.05, delta=0.0, vel=(0.0, 0.0, 0.0), skip_theta=0,
                 lattice_ut=0, skip_U=0, grad_stencil=0):
        lib = _load_f32()
        p = OrcParamsF32()
        p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
        p.lattice = int(lattice)
        for i, wv in enumerate(walls):
            p.wall[i] = int(wv)
        p.dx, p.dt, p.W0, p.tau0 = dx, dt, W0, tau0
        p.lam, p.Mcinf, p.k, p.D, p.kappa = lam, Mcinf, k, D, kappa
        p.aniso, p.eps, p.delta = int(aniso), eps, delta
        for a in range(3):
            p.vel[a] = float(vel[a])
        p.skip_theta, p.lattice_ut = int(skip_theta), int(lattice_ut)
        p.skip_U, p.grad_stencil = int(skip_U), int(grad_stencil)
        self.shape = (int(nz), int(ny), int(nx))
        self._h = lib.orc_create(ctypes.byref(p))
        if not self._h:
            raise ValueError("oracle rejected the parameters")
        self._lib = lib

    def close(self):
        if self._h:
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, phi, U, theta):
        a = [np.ascontiguousarray(v, dtype=np.float32).reshape(self.shape) for v in (phi, U, theta)]
        fp = ctypes.POINTER(ctypes.c_float)
        self._lib.orc_init(self._h, *[x.ctypes.data_as(fp) for x in a])

    def step(self, n=1):
        self._lib.orc_step(self._h, int(n))

    def fields(self):
        out = [np.zeros(self.shape, dtype=np.float32) for _ in range(3)]
        fp = ctypes.POINTER(ctypes.c_float)
        self._lib.orc_fields(self._h, *[x.ctypes.data_as(fp) for x in out])
        return [x.astype(np.float64) for x in out]
