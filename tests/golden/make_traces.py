"""Write the FP64 oracle's reduction traces used as stored expected values.

Calls only the oracle and the seeded input generators.  Each trace holds the
oracle's reductions (tip position, solid fraction, solute mass, enthalpy,
phi range) every ``reduce_every`` steps of one workload.

    python tests/golden/make_traces.py [thermal2d] [octant128] [centred256]

thermal2d  -- the 2D thermal dendrite of Sec. 4.1 (37 500 steps, T = 300)
octant128  -- 128^3 octant dendrite, Delta = 0.55, 5000 steps
centred256 -- 256^3 centred seed through its octant (128^3), 10 000 steps
fd2d, fd3d -- the LB oracle and the finite-difference discretisation of the
              same PDEs side by side (dx/W0 = 0.4, dt/tau0 = 0.02 for LB and
              0.01 for FD): a 200^2 quadrant slab over 4000 steps and a 64^3
              octant over 1500 steps; tip positions every 200 / 100 steps
fd3d_iso   -- the same 64^3 octant as the paper's isothermal alloy benchmark
              (theta = 0 and held in both), 1500 steps, tips every 50
thermal2d_isograd -- thermal2d with the isotropic lattice gradient of phi
              (oracle grad_stencil = 1) instead of axis central differences
thermal2d_dx<h>_T150 -- thermal2d refined under diffusive scaling
              (dt = 0.008 (h/0.4)^2, seed radius 4 W0) in a 100 W0 quadrant
              up to T = 150, h = 0.4, 0.3, 0.2; records every T = 4
The thermal cases hold U (oracle skip_U: M c_inf = 0, U acts on nothing),
which leaves phi and theta bit for bit unchanged.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1602_07483_amd import inputs  # noqa: E402

KEYS = (("solid_fraction", oracle.R_SOLID), ("solute_mass", oracle.R_MASS),
        ("enthalpy", oracle.R_ENTHALPY), ("phi_min", oracle.R_PHIMIN),
        ("phi_max", oracle.R_PHIMAX), ("nonfinite", oracle.R_NONFINITE))

def fd_problem(n, nz, iso=False):
    """Alloy + heat dendrite at the resolution of the paper's alloy benchmark
    (Sec. 4.2: dx/W0 = 0.4, dt/tau0 = 0.02, D = 2, k = 0.15, eps = 0.03,
    lambda = 3.2, U0 = -0.55), with theta0 = -0.55 and kappa = D; seed of
    radius 10 dx at the mirror corner.  iso: the benchmark itself, isothermal
    (theta = 0 and held, skip_theta in both discretisations)."""
    walls = (inputs.SYMMETRY, inputs.NOFLUX, inputs.SYMMETRY, inputs.NOFLUX,
             inputs.SYMMETRY, inputs.SYMMETRY if nz == 1 else inputs.NOFLUX)
    cz = 0.0 if nz == 1 else -0.5
    return inputs.Problem("fd-%dx%d%s" % (n, nz, "-iso" if iso else ""), n, n, nz, 19, walls, dx=0.4,
                          dt=0.02, W0=1.0, tau0=1.0, lam=3.2, Mcinf=1.0, k=0.15, D=2.0, kappa=2.0,
                          eps=0.03, centres=[(-0.5, -0.5, cz)], radius=10.0, U0=-0.55,
                          theta0=0.0 if iso else -0.55)


def tip_along_x(phi, cx):
    """Largest phi = 0 crossing along +x (linear interpolation), minus cx."""
    a, b = phi[..., :-1], phi[..., 1:]
    m = (a > 0) & (b <= 0)
    if not m.any():
        return float("nan")
    x = np.arange(phi.shape[-1] - 1, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        xs = np.where(m, x + a / np.where(m, a - b, 1.0), -np.inf)
    return float(xs.max()) - cx


def fd_trace(pb, steps, every, log=print, skip_theta=0):
    """Tip positions of the LB oracle and of the FD discretisation (two FD
    steps of dt/2 per LB step) from the same initial fields."""
    f0 = pb.initial_fields()
    o = oracle.Oracle(pb.nx, pb.ny, pb.nz, skip_theta=skip_theta, **pb.model_kwargs())
    o.init(*f0)
    fd = oracle.FDOracle(pb.nx, pb.ny, pb.nz, skip_theta=skip_theta, **pb.model_kwargs())
    fd.set(*f0)
    out = []
    t0 = time.time()
    done = 0
    while done < steps:
        o.step(every)
        fd.step(pb.dt / 2.0, 2 * every)
        done += every
        lp, fp = o.fields()[0], fd.fields()[0]
        rec = {"step": done, "lb_tip": tip_along_x(lp, pb.centres[0][0]),
               "fd_tip": tip_along_x(fp, pb.centres[0][0]),
               "lb_solid": float(np.mean(0.5 * (1 + lp))), "fd_solid": float(np.mean(0.5 * (1 + fp)))}
        out.append(rec)
        log("%s step %d LB tip %.3f FD tip %.3f %.1fs" % (pb.name, done, rec["lb_tip"], rec["fd_tip"],
                                                         time.time() - t0))
        sys.stdout.flush()
    o.close()
    fd.close()
    return out


FD_CASES = {"fd2d": (lambda: fd_problem(200, 1), 4000, 200, 0),
            "fd3d": (lambda: fd_problem(64, 64), 1500, 100, 0),
            "fd3d_iso": (lambda: fd_problem(64, 64, iso=True), 1500, 50, 1)}

def thermal2d_refined(dx, box=100.0, T=150.0, T_every=4.0):
    pb = inputs.workload_thermal2d(n=int(round(box / dx)), dx=dx)
    pb.steps = int(round(T / pb.dt))
    pb.reduce_every = int(round(T_every / pb.dt))
    return pb


# extra oracle options per workload
EXTRA = {"thermal2d_isograd": {"skip_U": 1, "grad_stencil": 1}}
for _h in (0.4, 0.3, 0.2):
    EXTRA["thermal2d_dx%g_T150" % _h] = {"skip_U": 1}

WORKLOADS = {
    "thermal2d": lambda: inputs.workload_thermal2d(),
    "thermal2d_isograd": lambda: inputs.workload_thermal2d(),
    "thermal2d_dx0.4_T150": lambda: thermal2d_refined(0.4),
    "thermal2d_dx0.3_T150": lambda: thermal2d_refined(0.3),
    "thermal2d_dx0.2_T150": lambda: thermal2d_refined(0.2),
    "octant128": lambda: inputs.workload_octant(128, 5000),
    "centred256": lambda: inputs.workload_centred_octant(256, 10000),
}


def trace(pb, log=print, extra=None):
    o = oracle.Oracle(pb.nx, pb.ny, pb.nz, **pb.model_kwargs(), **(extra or {}))
    o.init(*pb.initial_fields())
    out = []
    t0 = time.time()
    done = 0
    while done < pb.steps:
        n = min(pb.reduce_every, pb.steps - done)
        o.step(n)
        done += n
        r = o.reduce(pb.centre())
        rec = {"step": done, "tip": [r[oracle.R_TIPX], r[oracle.R_TIPY], r[oracle.R_TIPZ]]}
        for name, idx in KEYS:
            rec[name] = float(r[idx])
        out.append(rec)
        log("%s step %d tip %.4f %.1fs" % (pb.name, done, rec["tip"][0], time.time() - t0))
        sys.stdout.flush()
    o.close()
    return out


def main(names):
    for name in names or ["thermal2d", "octant128", "centred256"] + list(FD_CASES):
        if name in FD_CASES:
            factory, steps, every, skip_theta = FD_CASES[name]
            pb = factory()
            rec = {"workload": pb.name, "problem": {k: v for k, v in pb.__dict__.items()},
                   "lb_dt": pb.dt, "fd_dt": pb.dt / 2.0, "every": every, "skip_theta": skip_theta,
                   "oracle_threads": oracle.num_threads(),
                   "trace": fd_trace(pb, steps, every, skip_theta=skip_theta)}
            path = os.path.join(HERE, "trace_%s.json" % name)
            with open(path, "w") as fh:
                json.dump(rec, fh, indent=0)
            print("wrote", path)
            continue
        pb = WORKLOADS[name]()
        extra = EXTRA.get(name, {})
        rec = {"workload": pb.name, "problem": {k: v for k, v in pb.__dict__.items()},
               "oracle_options": extra, "oracle_threads": oracle.num_threads(),
               "trace": trace(pb, extra=extra)}
        path = os.path.join(HERE, "trace_%s.json" % name)
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=0)
        print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1:])
