"""Write the grid anisotropy of the finite-difference discretisation with the
face stencil (FD6) and the face + edge stencil (FD18), the two FD codes the
paper sets beside its LB lattices in the isotropic-growth study of Sec. 4.1.

Calls only the oracle and the seeded input generators.

    python tests/golden/make_fd_anisotropy.py [6] [18] [--n N]

The setup is the lattice-unit form of that study: eps = 0, dx = W0, dt = 0.15
tau0, kappa dt/dx^2 = 0.105, lambda = 10, pure substance (M c_inf = 0), a
sphere of radius 8 at the mirror corner of a 150^3 octant (the 300^3 domain
about its centre), to t = 1500 tau0; the undercooling is not printed in
the paper and Delta = 0.2 is taken.  FD18 runs at the LB time step, dt =
0.15 tau0 (10^4 steps).  FD6 cannot: with explicit Euler its checkerboard
mode is amplified by 1 - (12 W0^2/dx^2 + 2) dt/tau0 per step (the 7-point
Laplacian's largest eigenvalue 12/dx^2 plus the linearised double well at
phi = -1), -1.1 at dt = 0.15 tau0, so it diverges; it runs at dt = 0.1 tau0
(15 000 steps).  Each stencil writes fd_anisotropy_<stencil>.json:
the radii of the phi = 0 surface along [100] and [110] from the mirror
point, A_g = |R100 - R110| / (R100 + R110), and the sums of phi and theta
after the first 100 steps (for a short reproduction test).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1602_07483_amd.inputs import Problem, NOFLUX, SYMMETRY  # noqa: E402

N, T_END, CHECK_STEPS = 150, 1500.0, 100
DT = {6: 0.1, 18: 0.15}     # time step per stencil, in units of tau0


def problem(n=N, dt=0.15):
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, NOFLUX)
    return Problem("isotropic", n, n, n, 19, walls, dx=1.0, dt=dt, W0=1.0, tau0=1.0, lam=10.0,
                   Mcinf=0.0, k=0.15, D=0.7, kappa=0.7, eps=0.0,
                   centres=[(-0.5, -0.5, -0.5)], radius=8.0, U0=0.0, theta0=-0.2,
                   steps=int(round(T_END / dt)))


def first_crossing(prof):
    """Position of the first phi > 0 -> phi <= 0 crossing (linear interpolation)."""
    i = np.nonzero((prof[:-1] > 0) & (prof[1:] <= 0))[0][0]
    return float(i + prof[i] / (prof[i] - prof[i + 1]))


def fd_solver(stencil, pb):
    # pure substance: U does not act on phi or theta and is not solved
    fd = oracle.FDOracle(pb.nx, pb.ny, pb.nz, stencil=stencil, skip_U=1, **pb.model_kwargs())
    fd.set(*pb.initial_fields())
    return fd


def check_sums(stencil, n=N):
    pb = problem(n, dt=DT[stencil])
    fd = fd_solver(stencil, pb)
    fd.step(pb.dt, CHECK_STEPS)
    phi, _, th = fd.fields()
    return float(phi.sum()), float(th.sum())


def out_name(stencil, n=N):
    return "fd_anisotropy_%d.json" % stencil if n == N else "fd_anisotropy_%d_n%d.json" % (stencil, n)


def run(stencil, n=N):
    pb = problem(n, dt=DT[stencil])
    sums = check_sums(stencil, n)
    fd = fd_solver(stencil, pb)
    t0 = time.time()
    done = 0
    while done < pb.steps:
        fd.step(pb.dt, 1000)
        done += 1000
        print("FD%d step %d (%.0f s)" % (stencil, done, time.time() - t0), flush=True)
    phi = fd.fields()[0]
    n = pb.nx
    r100 = first_crossing(phi[0, 0, :]) + 0.5
    r110 = (first_crossing(np.array([phi[0, i, i] for i in range(n)])) + 0.5) * np.sqrt(2.0)
    out = {"stencil": stencil, "n": n, "steps": pb.steps, "dt": pb.dt, "R100": r100, "R110": r110,
           "A_g_percent": abs(r100 - r110) / (r100 + r110) * 100.0,
           "check_steps": CHECK_STEPS, "check_sum_phi": sums[0], "check_sum_theta": sums[1]}
    with open(os.path.join(HERE, out_name(stencil, n)), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    n = N
    if "--n" in args:
        i = args.index("--n")
        n = int(args[i + 1])
        del args[i:i + 2]
    for s in args or ["6", "18"]:
        run(int(s), n)
