"""Benchmark of the reordering hot path on one MI355X.

Workload: the 1920x1080 bounce-2 diffuse wavefront (2,073,600 rays) on the
~1M-triangle grid city, resident in HBM.  One step is the whole reordered
path on that wavefront through the C ABI: Two Point 64-bit keys
(rr_compute_keys), the key/index sort (rr_sort), the ray gather (rr_gather)
and the closest-hit trace of the sorted rays (rr_trace).  HIP events on the
working stream bracket each phase inside the timed region; the unsorted
trace of the same rays is timed the same way for the comparison.

Prints one JSON line: MRays/s including the reorder overhead (value), the
unsorted trace MRays/s, per-phase milliseconds, the sort's bandwidth, the
trace kernel's roofline figures and the CPU oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MRays/s incl. reorder vs unsorted trace; sort GB/s; p50/p99 batch latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--key", default="ot64", choices=["od32", "od64", "ot32", "ot64"])
    ap.add_argument("--builder", type=int, default=1, help="0 median split, 1 binned SAH")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the other key variants")
    ap.add_argument("--phases", default="all", choices=["all", "trace"],
                    help="'trace' times only the sorted and unsorted traces (for counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


KEYS = {"od32": (1, 32), "od64": (1, 64), "ot32": (2, 32), "ot64": (2, 64)}


def sort_algorithmic_bytes(n: int, key_bits: int) -> int:
    """One key read for the histograms plus, per 8-bit pass, a read and a
    write of (key, index)."""
    k = key_bits // 8
    return n * (k + (key_bits // 8) * 2 * (k + 4))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported in this build "
              "(the path shards by ray ranges with no exchange, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_11273_amd as rr
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rr.load()

    w = W.bounce2_1080p()
    n = w.rays.shape[0]
    scene = rr.Scene(w.tris, builder=args.builder)
    lo, hi = scene.bounds()
    kind, bits = KEYS[args.key]
    params = rr.key_params(kind, bits, lo, hi, 0.25)

    stream = torch.cuda.current_stream()
    rays = torch.from_numpy(w.rays).to(dev)
    kd = torch.int64 if bits == 64 else torch.int32
    keys = torch.empty(n, dtype=kd, device=dev)
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    srays = torch.empty((n, 8), dtype=torch.float32, device=dev)
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    uhits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    sws = rr.workspace(rr.sort_workspace_size(n, bits), dev)

    def step(ev=None):
        if ev: ev[0].record(stream)
        rr.rr_compute_keys(rays, params, keys=keys, idx=idx)
        if ev: ev[1].record(stream)
        rr.rr_sort(keys, idx, key_bits=bits, ws=sws)
        if ev: ev[2].record(stream)
        rr.rr_gather(rays, idx, out=srays)
        if ev: ev[3].record(stream)
        rr.rr_trace(scene, srays, hits=hits)
        if ev: ev[4].record(stream)

    def unsorted(ev=None):
        if ev: ev[0].record(stream)
        rr.rr_trace(scene, rays, hits=uhits)
        if ev: ev[1].record(stream)

    if args.phases == "trace":
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for _ in range(args.steps):
            rr.rr_trace(scene, srays, hits=hits)
            unsorted()
        torch.cuda.synchronize()
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"phases": "trace", "steps": args.steps}))
        return

    for _ in range(args.warmup):
        step()
        unsorted()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    phase = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(4)] for k in range(args.steps)])
    keys_ms, sort_ms, gather_ms, trace_ms = np.median(phase, axis=0)

    uev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
    for k in range(args.steps):
        unsorted(uev[k])
    torch.cuda.synchronize()
    unsorted_ms = float(np.median([e[0].elapsed_time(e[1]) for e in uev]))

    # correctness of what was timed: the sorted hits scattered back equal the unsorted hits
    back = rr.rr_scatter_hits(hits, idx)
    torch.cuda.synchronize()
    same = bool(torch.equal(back.view(torch.int32), uhits.view(torch.int32)))

    value = n / (ms_per_step * 1e-3) / 1e6
    trace_bytes = n * (32 + 16)
    sort_bytes = sort_algorithmic_bytes(n, bits)
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "MRays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "bounce2_diffuse_1920x1080_grid_city_1M_tris", "rays": int(n),
                   "triangles": int(w.tris.shape[0]), "key": args.key, "term_ratio": 0.25,
                   "bvh": ["median", "sah"][args.builder], "step": "keys+sort+gather+trace (sorted hits)"},
        "unsorted_trace_mrays": round(n / (unsorted_ms * 1e-3) / 1e6, 2),
        "trace_speedup_sorted_vs_unsorted": round(unsorted_ms / trace_ms, 3),
        "reorder_vs_unsorted": round(unsorted_ms / ms_per_step, 3),
        "phase_ms": {"keys": round(keys_ms, 4), "sort": round(sort_ms, 4), "gather": round(gather_ms, 4),
                     "trace_sorted": round(trace_ms, 4), "trace_unsorted": round(unsorted_ms, 4)},
        "sort_gbs": round(sort_bytes / (sort_ms * 1e-3) / 1e9, 1),
        "sort_roofline_frac": round(sort_bytes / (sort_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
        "hits_scatter_back_equal_unsorted": same,
        "roofline": {"kernel": "k_trace (sorted rays)", "bound": "hbm",
                     "achieved": round(trace_bytes / (trace_ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(trace_bytes / (trace_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                     "traffic": None, "algorithmic_bytes_per_ray": 48},
    }
    if not args.no_variants:
        result["variants"] = variants(torch, rr, scene, rays, n, lo, hi, dev, stream, args.steps, unsorted_ms)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.key)
    if args.copy_calibration:
        copy_calibration(torch, dev)
    scene.close()
    print(json.dumps(result))


def variants(torch, rr, scene, rays, n, lo, hi, dev, stream, steps, unsorted_ms):
    """The fused entry point for each key kind (sorted-order hits), and with
    the hits scattered back to ray order."""
    out = {}
    for name, (kind, bits) in [("none", (0, 32)), ("od32", (1, 32)), ("od64", (1, 64)), ("ot32", (2, 32)),
                               ("ot64", (2, 64))]:
        p = rr.key_params(kind, bits, lo, hi, 0.25)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
        cnt = torch.empty(1, dtype=torch.int32, device=dev)
        for flags, tag in ((0, ""), (rr.RR_HITS_ORIGINAL_ORDER, "_scatter_back"), (rr.RR_INDIRECT, "_indirect")):
            for _ in range(2):
                rr.rr_reorder_and_trace(scene, rays, p, flags=flags, hits=hits, count=cnt, ws=ws, want_perm=False)
            ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
            for k in range(steps):
                ev[k][0].record(stream)
                rr.rr_reorder_and_trace(scene, rays, p, flags=flags, hits=hits, count=cnt, ws=ws, want_perm=False)
                ev[k][1].record(stream)
            torch.cuda.synchronize()
            ms = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
            out[name + tag] = {"ms": round(ms, 4), "mrays": round(n / (ms * 1e-3) / 1e6, 2),
                               "vs_unsorted": round(unsorted_ms / ms, 3)}
        del ws
    return out


def cpu_baseline(w, key):
    """The CPU oracle on the whole wavefront: keys, sort, gather and trace
    over its median-split BVH (the build itself is not timed)."""
    import oracle as O
    threads = os.cpu_count() or 1
    kind, bits = KEYS[key]
    lo, hi = O.scene_box(w.tris)
    bvh = O.BVH(w.tris)
    n = w.rays.shape[0]
    t = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.reorder_and_trace(bvh, w.rays, kind, bits, lo, hi, 0.25, threads=threads)
        t.append(time.perf_counter() - t0)
    s = float(np.median(t))
    return {"value": round(n / s / 1e6, 3), "unit": "MRays/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole {n}-ray wavefront, median of 3 runs ({s:.2f} s each); keys and trace "
                      f"threaded over {threads} host threads, sort single-threaded (numpy lexsort)"}


def copy_calibration(torch, dev):
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
