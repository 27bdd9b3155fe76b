"""HBM bandwidth reference on one GPU: read-only, write-only and copy kernels
of the library (lbpf_bench_bandwidth) over a sweep of access width, cache
hint and grid size.  The best rate of each mode is the practical ceiling the
step kernels are compared with; the roofline peak stays the published 8 TB/s.

    python -m paper_1602_07483_amd.bandwidth [--gib 2] [--reps 10] [--json out.json]

Bytes counted: nbytes per read-only or write-only launch, 2 nbytes per copy.
Timed with events on torch's current stream, on which the kernels run.
"""
import argparse
import json
import sys

MODES = ("read", "write", "copy")
WIDTHS = (2, 4, 8, 16)
GRIDS = (1024, 2048, 4096, 8192, 16384, 32768)


def sweep(gib=2.0, reps=10, widths=WIDTHS, grids=GRIDS, log=print):
    import torch
    from paper_1602_07483_amd import lbpf
    nbytes = int(gib * (1 << 30)) // 64 * 64
    a = torch.zeros(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.zeros(nbytes // 4, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    for mode, name in enumerate(MODES):
        for width in widths:
            for nt in (0, 1):
                for blocks in grids:
                    def launch():
                        st = lbpf.lbpf_bench_bandwidth(mode, width, nt, blocks, b.data_ptr(), a.data_ptr(),
                                                       nbytes, stream)
                        if st != 0:
                            raise RuntimeError("lbpf_bench_bandwidth failed: %d" % st)
                    launch()
                    launch()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        launch()
                    e1.record()
                    e1.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    moved = (2 if mode == 2 else 1) * nbytes
                    gbps = moved / (ms * 1e-3) / 1e9
                    rows.append({"mode": name, "width": width, "nontemporal": nt, "blocks": blocks,
                                 "ms": ms, "GBps": gbps})
                    log("%-5s width %2d nt %d blocks %5d: %8.4f ms %7.0f GB/s" % (name, width, nt, blocks, ms, gbps))
    best = {}
    for name in MODES:
        r = max((x for x in rows if x["mode"] == name), key=lambda x: x["GBps"])
        best[name] = r
    return {"bytes": nbytes, "reps": reps, "rows": rows, "best": best}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--json", default="")
    a = ap.parse_args(argv)
    res = sweep(a.gib, a.reps)
    for name, r in res["best"].items():
        print("best %-5s: %.0f GB/s (width %d, nontemporal %d, %d blocks)" % (name, r["GBps"], r["width"],
                                                                           r["nontemporal"], r["blocks"]))
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(res, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
