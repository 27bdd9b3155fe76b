"""Paper-scale growth-direction runs of Sec. 4.3 (non-standard dendrites).

The paper's parameters: dx = 0.01, dt = 1.5e-5, W0 = 0.0125,
tau0 = 1.5625e-4, lambda = 10, kappa = 1, Delta = 0.25, a seed of radius 8
nodes at the corner of three mirror planes, pure substance, 351^3 nodes.
The cubic anisotropy (eps = 0.05) is shown after 3e4 steps and grows along
[100]; the K41/K61 one (eps = 0, delta = -0.02) after 1.4e5 steps and grows
along [110].

Usage (one GPU):
    python -m paper_1602_07483_amd.showcase --case cubic
    python -m paper_1602_07483_amd.showcase --case k41k61
    python -m paper_1602_07483_amd.showcase --case cubic --lattice-ut 7   # theta on D3Q7

Prints one progress line per record and a final JSON line with the radii of
the phi = 0 surface along [100], [110] and [111] (lattice units from the
mirror point), the solid fraction and the throughput.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbpf
from .inputs import Problem, NOFLUX, SYMMETRY

CASES = {
    "cubic": dict(aniso=lbpf.LBPF_ANISO_CUBIC, eps=0.05, delta=0.0, steps=30000),
    "k41k61": dict(aniso=lbpf.LBPF_ANISO_K41K61, eps=0.0, delta=-0.02, steps=140000),
}


def problem(case, n=351):
    c = CASES[case]
    walls = (SYMMETRY, NOFLUX, SYMMETRY, NOFLUX, SYMMETRY, NOFLUX)
    return Problem("sec4.3-" + case, n, n, n, 19, walls, dx=0.01, dt=1.5e-5, W0=0.0125,
                   tau0=1.5625e-4, lam=10.0, Mcinf=0.0, k=0.15, D=1.0, kappa=1.0,
                   aniso=c["aniso"], eps=c["eps"], delta=c["delta"],
                   centres=[(-0.5, -0.5, -0.5)], radius=8.0, U0=0.0, theta0=-0.25,
                   steps=c["steps"])


def outer_crossing(prof):
    """Position of the outermost phi > 0 -> phi <= 0 crossing (linear
    interpolation), NaN if the profile never crosses."""
    i = np.nonzero((prof[:-1] > 0) & (prof[1:] <= 0))[0]
    if len(i) == 0:
        return float("nan")
    i = i[-1]
    return float(i + prof[i] / (prof[i] - prof[i + 1]))


def radii(phi):
    n = phi.shape[0]
    d = np.arange(n)
    r100 = outer_crossing(phi[0, 0, :]) + 0.5
    r110 = (outer_crossing(phi[0, d, d]) + 0.5) * np.sqrt(2.0)
    r111 = (outer_crossing(phi[d, d, d]) + 0.5) * np.sqrt(3.0)
    return r100, r110, r111


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), required=True)
    ap.add_argument("--n", type=int, default=351)
    ap.add_argument("--steps", type=int, default=0, help="default: the paper's figure time")
    ap.add_argument("--records", type=int, default=10)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--lattice-ut", type=int, default=0, choices=(0, 7, 15, 19),
                    help="lattice of theta (0: D3Q19, as phi); Sec. 4.1 pairs D2Q9 phi with D2Q5 theta")
    args = ap.parse_args(argv)
    pb = problem(args.case, args.n)
    steps = args.steps or pb.steps
    s = lbpf.solver_for(pb, storage=args.storage, skip_U=1,   # pure substance: theta only
                        lattice_ut=args.lattice_ut)
    s.set_fields(*pb.initial_fields())
    chunk = max(1, steps // args.records)
    done, stepping = 0, 0.0
    while done < steps:
        k = min(chunk, steps - done)
        t0 = time.perf_counter()
        s.step(k)
        s.sync()
        stepping += time.perf_counter() - t0
        done += k
        phi, _, _, red = s.read(check=False)
        r = radii(phi)
        print("%s step %7d: R100 %.2f R110 %.2f R111 %.2f solid %.4f phi [%.4f, %.4f] nonfinite %d"
              % (args.case, done, r[0], r[1], r[2], red["solid_fraction"], red["phi_min"],
                 red["phi_max"], red["nonfinite"]), flush=True)
    s.close()
    out = {"case": args.case, "n": args.n, "steps": steps, "storage": args.storage,
           "lattice_ut": args.lattice_ut or 19,
           "R100": r[0], "R110": r[1], "R111": r[2], "solid_fraction": red["solid_fraction"],
           "nonfinite": red["nonfinite"], "mlups": float(args.n) ** 3 * steps / stepping / 1e6}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
