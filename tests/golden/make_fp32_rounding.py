"""Write the error that single-precision rounding alone gives the method:
the LB oracle's algorithm built in float (oracle.OracleF32) against the FP64
oracle, from the same initial fields, on the cases whose FP32 parity the GPU
tests bound.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_fp32_rounding.py

Cases: the 136 x 40 x 24 interior-tile problem and the 32^3 corner workload
(200 steps), and the four sampled domains of the 64-domain ensemble (the
smallest and largest of each lattice, 200 steps).  For each, the max-abs
differences of phi, U and theta after 50 and 200 steps go to
fp32_rounding.json.  A growing interface amplifies the per-step rounding of
the FP32 state, so where this error exceeds 1e-5 no FP32 implementation of
the step can be held to 1e-5, and the GPU tests take this error as the bound.
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

CHECK, STEPS = 50, 200


def ensemble_picks():
    probs = inputs.workload_ensemble()
    half = len(probs) // 2
    picks = []
    for part in (probs[:half], probs[half:]):
        order = sorted(part, key=lambda p: p.nodes)
        picks += [order[0], order[-1]]
    return picks


def cases():
    return [inputs.workload_interior(), inputs.workload_small(steps=STEPS)] + ensemble_picks()


def rounding_error(pb, steps):
    f0 = pb.initial_fields()
    a = oracle.Oracle(pb.nx, pb.ny, pb.nz, **pb.model_kwargs())
    b = oracle.OracleF32(pb.nx, pb.ny, pb.nz, **pb.model_kwargs())
    a.init(*f0)
    b.init(*f0)
    out = {}
    done = 0
    for s in steps:
        a.step(s - done)
        b.step(s - done)
        done = s
        fa, fb = a.fields(), b.fields()
        out[str(s)] = [float(np.max(np.abs(x - y))) for x, y in zip(fa, fb)]
    a.close()
    b.close()
    return out


def main():
    res = {}
    for pb in cases():
        t0 = time.time()
        res[pb.name] = {"nx": pb.nx, "ny": pb.ny, "nz": pb.nz, "lattice": pb.lattice,
                        "max_abs_phi_U_theta": rounding_error(pb, (CHECK, STEPS))}
        print(pb.name, res[pb.name], "%.0f s" % (time.time() - t0), flush=True)
    with open(os.path.join(HERE, "fp32_rounding.json"), "w") as fh:
        json.dump({"check_steps": CHECK, "steps": STEPS, "cases": res}, fh, indent=1)


if __name__ == "__main__":
    main()
