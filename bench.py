#!/usr/bin/env python3
"""Benchmark of the lattice-Boltzmann phase-field time step on one MI355X.

Workload: 256^3 nodes, D3Q19 for phi, U and theta, one centred seed of radius
10 in an undercooled melt (Delta = 0.6, eps = 0.05, k = 0.15), all walls
no-flux; FP32 populations (headline) and FP16/BF16 deviation storage.  A step
is one full time step of all three fields (one phase-field kernel + one
supersaturation/heat kernel).  Inputs are resident in HBM before the timed
region; the timed region is exactly --steps steps between two device
synchronisations.

Prints one JSON line.  The roofline entry is for the dominant kernel: its
algorithmic bytes per launch divided by its mean launch time, measured with
HIP events on the library's stream during the timed region.  The CPU baseline
is the FP64 oracle on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (all 3 fields) and HBM GB/s vs roofline; FP32 vs mixed storage, 1 GPU"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update and kernel, D3Q19, b bytes per stored
# population, 4-byte fields: k_phi reads/writes 19 g (2*19*b) + reads phi, U,
# theta and writes phi (16 B); k_ut reads/writes 19 h and 19 f (4*19*b) +
# reads phi^n, phi^{n+1}, U, theta and writes U, theta (24 B).
def bytes_per_lup(q, b):
    return {"k_phi": 2 * q * b + 16, "k_ut": 4 * q * b + 24}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "lattice.hpp", "runtime.hpp", "step.hip", "lbpf.hip"):
        with open(os.path.join(ROOT, "paper_1602_07483_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, storage):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_256cube_%s.md" % (kernel, storage))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_hash = re.search(r"kernel source hash:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def run_gpu(storage, steps, warmup, n, launch=None):
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_centred

    pb = workload_centred(n=n)
    pb.reduce_every = 100        # FP64 reductions (solute mass, tip) every 100 steps, timed
    stream = torch.cuda.current_stream().cuda_stream
    s = lbpf.solver_for(pb, storage=storage, stream=stream)
    fields0 = pb.initial_fields()
    t_in = time.perf_counter()
    s.set_fields(*fields0)          # host -> device copy and initial populations
    t_in = time.perf_counter() - t_in
    if launch == "auto":
        # launch of each kernel picked by the library's autotuner (state restored after)
        s.autotune(6)
    elif launch is not None:
        s.set_launch(*launch)
    launches = s.launches()
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, cnt = s.kernel_times()
    s.set_timing(False)
    t_out = time.perf_counter()
    _, _, _, red = s.read()          # device -> host copy of the fields and the reductions
    t_out = time.perf_counter() - t_out
    s.close()
    lups = float(n) ** 3 * steps
    b = lbpf.lbpf_storage_bytes(lbpf.STORAGE[storage])
    bpl = bytes_per_lup(19, b)
    kern = {}
    for i, name in enumerate(("k_phi", "k_ut")):
        avg_ms = ms[i] / max(cnt[i], 1)
        per_launch = bpl[name] * float(n) ** 3
        kern[name] = {"avg_ms": avg_ms, "launches": cnt[i], "bytes_per_launch": per_launch,
                      "GBps": per_launch / (avg_ms * 1e-3) / 1e9}
    return {"mlups": lups / wall / 1e6, "ms_per_step": wall / steps * 1e3,
            "launch": {k: {"tile": [v[0], v[1]], "zslab": v[2], "xcd_remap": v[3]}
                       for k, v in launches.items()},
            "algorithmic_GBps": lups * (bpl["k_phi"] + bpl["k_ut"]) / wall / 1e9,
            "kernels": kern, "solid_fraction": red["solid_fraction"],
            "phi_range": [red["phi_min"], red["phi_max"]],
            # the same steps with the host hand-over at both ends (fields in
            # and out through lbpf_set_fields / lbpf_read); not the headline
            "host_io": {"set_fields_ms": t_in * 1e3, "read_ms": t_out * 1e3,
                        "mlups_with_host_io": lups / (wall + t_in + t_out) / 1e6}}


def run_single_field(steps, warmup, n, storage="f32"):
    """The same 256^3 seed with one transport field: a pure substance
    (M c_inf = 0, skip_U: theta alone) and an isothermal alloy (theta held,
    skip_theta: U alone), as in the paper's thermal and alloy benchmarks."""
    import dataclasses
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_centred

    out = {"storage": storage, "steps": steps}
    base = workload_centred(n=n)
    base.reduce_every = 0
    stream = torch.cuda.current_stream().cuda_stream
    for name, pb, kw in (("skip_U (pure substance, Mcinf = 0)", dataclasses.replace(base, Mcinf=0.0),
                          {"skip_U": 1}),
                         ("skip_theta (isothermal, theta = 0)", dataclasses.replace(base, theta0=0.0),
                          {"skip_theta": 1})):
        s = lbpf.solver_for(pb, storage=storage, stream=stream, **kw)
        s.set_fields(*pb.initial_fields())
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        out[name] = {"mlups": float(n) ** 3 * steps / wall / 1e6}
    return out


def run_separate_lattices(steps, warmup, n):
    """The same 256^3 seed with phi on D3Q19 and U, theta on D3Q7 (each
    scheme on its own lattice, as Sec. 4.1 runs phi on D2Q9 and theta on
    D2Q5), at dt/tau0 = 0.11, inside the D3Q7 U scheme's stable window."""
    import dataclasses
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_centred

    pb = dataclasses.replace(workload_centred(n=n), dt=0.11, reduce_every=0)
    out = {"lattices": "phi D3Q19, U and theta D3Q7", "dt_over_tau0": 0.11, "steps": steps}
    stream = torch.cuda.current_stream().cuda_stream
    for storage in ("f32", "f16"):
        s = lbpf.solver_for(pb, storage=storage, stream=stream, lattice_ut=7)
        s.set_fields(*pb.initial_fields())
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        s.close()
        out[storage] = {"mlups": float(n) ** 3 * steps / wall / 1e6}
    return out


def run_ensemble(steps, seq_steps, storage="f16", graph_steps=50):
    """Batched ensemble of 64 uneven domains (mixed D3Q15/D3Q19, per-domain
    eps, Delta and noise seed) replayed from a HIP graph, against the same
    domains stepped one after another with their own launches."""
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_ensemble

    probs = workload_ensemble()
    nodes = float(sum(p.nodes for p in probs))
    stream = torch.cuda.current_stream().cuda_stream
    b = lbpf.Batch([lbpf.problem_kwargs(p) for p in probs], storage=storage, stream=stream)
    for d, p in zip(b.domains, probs):
        d.set_fields(*p.initial_fields())
    b.set_graph(graph_steps)
    b.step(graph_steps)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    reds = [d.read_status()[1] for d in b.domains]
    nonfinite = [p.name for p, r in zip(probs, reds) if r["nonfinite"]]
    peak = max(max(-r["phi_min"], r["phi_max"]) for p, r in zip(probs, reds) if p.eps <= 1.0 / 15.0)
    b.close()

    solvers = []
    for p in probs:
        s = lbpf.solver_for(p, storage=storage, stream=stream)
        s.set_fields(*p.initial_fields())
        s.step(2)
        solvers.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in solvers:
        s.step(seq_steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    for s in solvers:
        s.close()
    batch = nodes * steps / t_batch / 1e6
    seq = nodes * seq_steps / t_seq / 1e6
    return {"workload": "64 cubic domains, L in U{32..96} (%.1f M nodes), D3Q15 x32 + D3Q19 x32, "
                        "eps in U[0.02,0.07], Delta in U[0.45,0.65], centred seed R=8, no-flux, "
                        "dt/tau0 = 0.11 (D3Q15) / 0.15 (D3Q19)"
                        % (nodes / 1e6),
            "storage": storage, "steps": steps, "graph_steps": graph_steps,
            "batched_graph_mlups": batch, "sequential_mlups": seq, "sequential_steps": seq_steps,
            "speedup": batch / seq, "nonfinite_domains": nonfinite,
            "max_abs_phi_eps_le_1_15": peak}


def run_multiseed(steps, storage="f16"):
    """512^3 eight-nucleus domains in mixed storage (64-bit-addressed kernels,
    every field's populations exceed 4 GiB), cubic and K41/K61 anisotropy:
    throughput and FP64 solute-mass drift over the timed steps."""
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_multiseed

    out = {}
    stream = torch.cuda.current_stream().cuda_stream
    for aniso, label in ((0, "cubic eps=0.05"), (1, "K41/K61 eps=0 delta=-0.02")):
        pb = workload_multiseed(512, aniso=aniso)
        pb.reduce_every = 0
        s = lbpf.solver_for(pb, storage=storage, stream=stream)
        s.set_fields(*pb.initial_fields())
        s.step(10)
        _, r0 = s.read_status()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st, r1 = s.read_status()
        s.close()
        out[label] = {"mlups": float(pb.nodes) * steps / dt / 1e6, "steps": steps,
                      "mass_drift": (r1["solute_mass"] - r0["solute_mass"]) / abs(r0["solute_mass"]),
                      "solid_fraction": r1["solid_fraction"], "status": st}
    return {"workload": "512^3 D3Q19, 8 nuclei R=6 (separation >= 64), Delta=0.55, k=0.15, no-flux",
            "storage": storage, "runs": out}


def oracle_errors(storages, steps_small=200, n_big=256, steps_big=10000):
    """Error of each storage form against the FP64 oracle:
    * fields: max-abs of phi, U, theta after steps_small steps of the 32^3
      corner workload (seeded input), against a live oracle run;
    * tip velocity and solute-mass drift: a steps_big run of the 256^3
      centred workload with FP64 reductions every 100 steps, against the
      oracle's stored trace of the same run (tests/golden/trace_centred256.json,
      computed on the equivalent octant): the largest relative tip-velocity
      error over the intervals of free growth, and the solute-mass drift of
      both over the whole run."""
    import numpy as np
    import oracle
    import torch
    from paper_1602_07483_amd import lbpf
    from paper_1602_07483_amd.inputs import workload_small, workload_centred

    small = workload_small(steps=steps_small)
    f0 = small.initial_fields()
    o = oracle.Oracle(small.nx, small.ny, small.nz, **small.model_kwargs())
    o.init(*f0)
    o.step(steps_small)
    ref = o.fields()
    o.close()
    with open(os.path.join(ROOT, "tests", "golden", "trace_centred256.json")) as fh:
        tr = json.load(fh)["trace"]
    vo = np.diff([r["tip"][0] for r in tr])
    stream = torch.cuda.current_stream().cuda_stream
    out = {}
    for storage in storages:
        s = lbpf.solver_for(small, storage=storage, stream=stream)
        s.set_fields(*f0)
        s.step(steps_small)
        g = s.read(reductions=False)[:3]
        s.close()
        pb = workload_centred(n=n_big, steps=steps_big)
        s = lbpf.solver_for(pb, storage=storage, stream=stream)
        s.set_fields(*pb.initial_fields())
        s.step(steps_big)
        hist = s.history()
        s.close()
        vg = np.diff([h["tip"][0] for h in hist])
        tips_o = np.array([r["tip"][0] for r in tr])
        inside = tips_o < 0.9 * (n_big // 2)
        ok = inside[:-1] & inside[1:] & (np.abs(vo) > 1e-3)
        m0 = 8.0 * tr[0]["solute_mass"]
        out[storage] = {
            "fields_max_abs_after_%d_steps_32cube" % steps_small:
                {name: float(np.max(np.abs(a - b))) for name, a, b in zip(("phi", "U", "theta"), g, ref)},
            "tip_velocity_max_rel_error": float(np.max(np.abs(vg[ok] - vo[ok]) / np.abs(vo[ok]))),
            "tip_velocity_intervals": int(ok.sum()),
            "mass_drift": {"gpu": (hist[-1]["solute_mass"] - hist[0]["solute_mass"]) / abs(hist[0]["solute_mass"]),
                           "oracle": (8.0 * tr[-1]["solute_mass"] - m0) / abs(m0)},
            "steps": steps_big}
    return out


def copy_bandwidth(nbytes=2 << 30, reps=20):
    import torch
    from paper_1602_07483_amd import lbpf
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    lbpf.lbpf_bench_copy(b.data_ptr(), a.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lbpf.lbpf_bench_copy(b.data_ptr(), a.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return 2.0 * nbytes / dt / 1e9


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(pb, budget_s, max_steps):
    import oracle
    o = oracle.Oracle(pb.nx, pb.ny, pb.nz, **pb.model_kwargs())
    o.init(*pb.initial_fields())
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        o.step(1)
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    o.close()
    return float(pb.nodes) * steps / dt / 1e6, steps


def cpu_baseline(n=256):
    """The FP64 oracle, as it stands (initialisation excluded), on bounded
    samples: the benchmark's 256^3 workload on all host threads (the line's
    value), the 128^3 octant dendrite on all threads, and the same octant on
    one thread."""
    import ctypes
    import oracle
    from paper_1602_07483_amd.inputs import workload_centred, workload_octant
    threads = oracle.num_threads()
    v, steps = _oracle_rate(workload_centred(n=n), 12.0, 12)
    v128, s128 = _oracle_rate(workload_octant(128), 12.0, 100)   # the 128^3 run of 100 steps
    one = None
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        one, s1 = _oracle_rate(workload_octant(128), 8.0, 10)
        gomp.omp_set_num_threads(threads)
    except OSError:
        s1 = 0
    return {"value": v, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d^3 D3Q19 centred-seed workload, %d FP64 steps on %d host threads" % (n, steps, threads),
            "cpu_model": _cpu_model(),
            "octant128_all_threads": {"mlups": v128, "steps": s128},
            "octant128_one_thread": {"mlups": one, "steps": s1}}



def note(msg):
    """Progress of the legs, on stderr (the result line is the only stdout)."""
    print("bench: " + msg, file=sys.stderr, flush=True)

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-variants", action="store_true", help="FP32 only")
    ap.add_argument("--launch", default=None,
                    help="tile_x,tile_y,zslab,xcd_remap instead of the library default")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-multiseed", action="store_true", help="skip the 512^3 multi-seed leg")
    ap.add_argument("--multiseed-steps", type=int, default=200)
    ap.add_argument("--ensemble-steps", type=int, default=2000)
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the error of each storage form against the FP64 oracle")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner pick the launch before timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported "
              "(the design notes describe how the step would shard)" % args.gpus, file=sys.stderr)
        return 2
    rank = int(os.environ.get("RANK", "0"))

    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    if args.autotune:
        launch = "auto"
    res = run_gpu("f32", args.steps, args.warmup, args.n, launch)
    note("f32 %.0f MLUPS" % res["mlups"])
    variants = {}
    if not args.no_variants:
        for st in ("f16", "bf16"):
            r = run_gpu(st, args.steps, args.warmup, args.n, launch)
            variants[st] = {"mlups": r["mlups"], "ms_per_step": r["ms_per_step"], "launch": r["launch"],
                            "algorithmic_GBps": r["algorithmic_GBps"],
                            "speedup_vs_f32": r["mlups"] / res["mlups"],
                            "kernels": r["kernels"]}
            note("%s %.0f MLUPS" % (st, r["mlups"]))
    copy_gbs = copy_bandwidth()
    single_field = separate_lattices = None
    if not args.no_variants:
        single_field = run_single_field(max(args.steps // 3, 1), args.warmup, args.n)
        separate_lattices = run_separate_lattices(max(args.steps // 3, 1), args.warmup, args.n)
        note("single-field and separate-lattice legs done")
    multiseed = None
    if not args.no_multiseed:
        multiseed = run_multiseed(args.multiseed_steps)
        note("multi-seed leg done")
    ensemble = None
    if not args.no_ensemble:
        ensemble = run_ensemble(args.ensemble_steps, max(args.ensemble_steps // 4, 1))
        note("ensemble leg done")
    errors = None
    if not args.no_errors and args.n == 256:
        errors = oracle_errors(["f32"] + ([] if args.no_variants else ["f16", "bf16"]))
        for st, e in errors.items():
            if st in variants:
                variants[st]["error_vs_oracle"] = e
        note("errors against the oracle done")

    dom = max(res["kernels"], key=lambda k: res["kernels"][k]["avg_ms"])
    kd = res["kernels"][dom]
    traffic = measured_traffic(dom, "f32")
    roofline = {"bound": "hbm", "kernel": dom, "achieved": kd["GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": kd["GBps"] / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": kd["bytes_per_launch"],
                "avg_launch_ms": kd["avg_ms"], "copy_kernel_GBps": copy_gbs}

    cpu = None
    if rank == 0 and not args.no_cpu:
        cpu = cpu_baseline(args.n)

    line = {
        "metric": METRIC, "value": res["mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "centred seed R=10, %d^3 D3Q19, phi/U/theta, Delta=0.6, "
                               "eps=0.05, k=0.15, no-flux walls, dt/tau0=0.15 (dt=tau0 is unstable), "
                               "FP64 reductions every 100 steps" % args.n,
                   "nodes": args.n ** 3, "lattice": "D3Q19", "storage": "f32"},
        "algorithmic_GBps": res["algorithmic_GBps"],
        "launch": res["launch"],
        "kernels": res["kernels"],
        "host_io": res["host_io"],
        "error_vs_oracle": errors.get("f32") if errors else None,
        "variants": variants,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "single_field": single_field,
        "separate_lattices": separate_lattices,
        "ensemble": ensemble,
        "multiseed": multiseed,
        "health": {"solid_fraction": res["solid_fraction"], "phi_range": res["phi_range"]},
    }
    if rank == 0:
        print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
