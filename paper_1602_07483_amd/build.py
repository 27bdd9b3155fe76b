"""Build the gfx950 shared library liblbpf.so in-tree with hipcc.

The step kernels are instantiated per lattice and storage type: step.hip is
compiled once for each of the 12 pairs (LBPF_STEP_Q, LBPF_STEP_STORAGE), in
parallel with lbpf.hip (C ABI, initialisation, reductions, batches), and the
objects are linked into one library.

Usage: python -m paper_1602_07483_amd.build
"""
import concurrent.futures
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbpf.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("LBPF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=" + ARCH,
    # no packed-FP32 instructions in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]

LATTICES = (7, 15, 19)
STORAGES = (0, 1, 2, 3)      # lbpf_storage: F32, F16_DEV, BF16_DEV, F64


def kernel_build_id() -> str:
    """Digest of the kernel sources (every file under csrc/), 16 hex digits:
    persisted autotuner results are keyed by it."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hpp", ".hip")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def units():
    """(object name, source, extra flags) of every translation unit."""
    out = [("lbpf.o", os.path.join(CSRC, "lbpf.hip"), ['-DLBPF_KERNEL_BUILD="%s"' % kernel_build_id()])]
    for q in LATTICES:
        for st in STORAGES:
            out.append(("step_q%d_s%d.o" % (q, st), os.path.join(CSRC, "step.hip"),
                        ["-DLBPF_STEP_Q=%d" % q, "-DLBPF_STEP_STORAGE=%d" % st]))
    return out


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 1)

    def compile_one(u):
        name, src, extra = u
        obj = os.path.join(OBJ_DIR, name)
        cmd = [hipcc] + HIPCC_FLAGS + extra + ["-c", "-o", obj + ".tmp", src]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (name, r.stderr[-4000:]))
        os.replace(obj + ".tmp", obj)
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, units()))
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    cmd = ([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", LIB + ".tmp"] + objs +
           ["-L" + rocm_lib, "-Wl,-rpath," + rocm_lib, "-lrocprofiler-sdk-roctx"])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
