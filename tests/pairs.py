"""Run one problem on the GPU library and on the FP64 oracle from the same
seeded initial fields (test helper)."""
import numpy as np

from oracle import Oracle
from paper_1602_07483_amd import lbpf


def make_oracle(pb):
    o = Oracle(pb.nx, pb.ny, pb.nz, **pb.model_kwargs())
    o.init(*pb.initial_fields())
    return o


def make_gpu(pb, storage="f32", **over):
    s = lbpf.solver_for(pb, storage=storage, **over)
    s.set_fields(*pb.initial_fields())
    return s


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
