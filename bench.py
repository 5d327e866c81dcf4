"""Benchmark of the reordering hot path on one MI355X.

Headline workload: the 1920x1080 bounce-2 diffuse wavefront (2,073,600 rays)
on the ~1M-triangle grid city, resident in HBM.  One step is the whole
reordered path on that wavefront through the C ABI: Two Point 64-bit keys
(rr_compute_keys), the key/index sort (rr_sort), the ray gather (rr_gather)
and the closest-hit trace of the sorted rays (rr_trace).  HIP events on the
working stream bracket each phase inside the timed region; the unsorted trace
of the same rays is timed the same way for the comparison.

Further sections (each can be skipped): the fused entry point per key
variant; the 3840x2160 bounce-3 wavefront (8,294,400 slots, terminated rays
compacted before the sort); 64 wavefronts of mixed bounces reordered and
traced in one graph launch with autotuned launch shape; a Poisson stream of
requests served with continuous batching on the ~4M-triangle city, with
p50/p99 latency; and the CPU oracle on the host cores.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MRays/s incl. reorder vs unsorted trace; sort GB/s; p50/p99 batch latency"
KEYS = {"none": (0, 32), "od32": (1, 32), "od64": (1, 64), "ot32": (2, 32), "ot64": (2, 64)}
# the figure's other layouts (32-bit) and the Two Point termination estimates
METHODS = {"origin": (3, 32), "costa": (4, 32), "aila": (5, 32), "aila_compact": (6, 32), "octahedron": (7, 32),
           "tp_adaptive32": (8, 32), "tp_adaptive64": (8, 64), "tp_real32": (9, 32)}
# HBM traffic of the sorted trace launch, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes scaled by a plain copy's readings; valid only while the sources that
# decide the trace's memory traffic are unchanged (checked by digest).
TRAFFIC_PROFILE = os.path.join("profiles", "k_trace4_bounce2_1080p_traffic.txt")
TRAFFIC_SOURCES = ("paper_2506_11273_amd/csrc/trace.hip", "paper_2506_11273_amd/csrc/scene.cpp",
                   "paper_2506_11273_amd/csrc/common.hpp", "paper_2506_11273_amd/csrc/keys_dev.hpp",
                   "paper_2506_11273_amd/csrc/keys.hip", "workloads/gen.c")
SECTIONS = ("config1", "variants", "orders", "shuffled", "shadow", "bounce3", "sorts", "batch", "serve", "cpu")


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--key", default="ot64", choices=[k for k in KEYS if k != "none"])
    ap.add_argument("--builder", type=int, default=1, help="0 median split, 1 binned SAH")
    ap.add_argument("--skip", default="", help="comma list of sections to skip: " + ",".join(SECTIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-loads", default="0.5,0.8,0.95",
                    help="offered loads, fractions of the measured batched capacity")
    ap.add_argument("--phases", default="all", choices=["all", "trace", "trace4m", "sort", "batch"],
                    help="'trace' times only the sorted and unsorted traces of the headline wavefront, "
                         "'trace4m' the shuffled, key-sorted and generation orders of first-bounce rays "
                         "in the 4M-triangle city, 'sort' only sorts, 'batch' only runs the 64-wavefront "
                         "batch graph in a fixed launch shape (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for the HBM byte counters)")
    a = ap.parse_args(argv)
    a.skip = set(s for s in a.skip.split(",") if s)
    unknown = sorted(a.skip - set(SECTIONS))
    if unknown:
        ap.error(f"--skip: unknown section(s) {','.join(unknown)}; known: {','.join(SECTIONS)}")
    if a.no_cpu_baseline:
        a.skip.add("cpu")
    if a.no_variants:
        a.skip.add("variants")
    return a


def sort_algorithmic_bytes(n: int, key_bits: int) -> int:
    """One key read for the histograms plus, per 8-bit pass, a read and a
    write of (key, index)."""
    k = key_bits // 8
    return n * (k + (key_bits // 8) * 2 * (k + 4))


def median_ms(torch, stream, fn, reps):
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
    for k in range(reps):
        ev[k][0].record(stream)
        fn()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    return float(np.median([e[0].elapsed_time(e[1]) for e in ev]))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard by ray ranges with no exchange)", file=sys.stderr)
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
    if args.phases == "trace4m":
        trace_orders_4m(torch, rr, W, dev, args)
        return
    if args.phases == "sort":
        sorts_only(torch, rr, W, dev, args)
        return

    w = W.bounce2_1080p()
    n = w.rays.shape[0]
    scene = rr.Scene(w.tris, builder=args.builder)
    if args.phases == "batch":
        batch_only(torch, rr, W, scene, w, dev, args)
        return
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

    # the headline step: one fused call (keys, the sort with the ray gather in
    # its last pass, the trace), hits in key order
    fhits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    fws = rr.workspace(rr.reorder_workspace_size(n, params), dev)

    def fused():
        rr.rr_reorder_and_trace(scene, rays, params, flags=0, hits=fhits, ws=fws, want_perm=False, want_count=False)

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
        print(json.dumps({"phases": "trace", "steps": args.steps, "warmup": args.warmup,
                          "sources_sha256": sources_digest()}))
        return

    for _ in range(args.warmup):
        fused()
        step()
        unsorted()
    torch.cuda.synchronize()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        fused()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # the same work as separate calls, for the per-phase times
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    phase = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(4)] for k in range(args.steps)])
    keys_ms, sort_ms, gather_ms, trace_ms = np.median(phase, axis=0)
    unsorted_ms = median_ms(torch, stream, unsorted, args.steps)

    # what was timed is correct: the fused call's hits equal the separate
    # calls' hits, and scattered back they equal the unsorted trace's hits
    same_fused = bool(torch.equal(fhits.view(torch.int32), hits.view(torch.int32)))
    back = rr.rr_scatter_hits(hits, idx)
    torch.cuda.synchronize()
    same = bool(torch.equal(back.view(torch.int32), uhits.view(torch.int32))) and same_fused
    prof = rr.rr_trace_profile(scene, srays)
    uprof = rr.rr_trace_profile(scene, rays)

    value = n / (ms_per_step * 1e-3) / 1e6
    trace_bytes = n * TRACE_BYTES_PER_RAY
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
                   "bvh": ["median", "sah"][args.builder] + " collapsed to 4-wide",
                   "step": "rr_reorder_and_trace: keys, sort (ray gather fused into its last pass), trace; "
                           "hits in key order"},
        "unsorted_trace_mrays": round(n / (unsorted_ms * 1e-3) / 1e6, 2),
        "trace_speedup_sorted_vs_unsorted": round(unsorted_ms / trace_ms, 3),
        "reorder_vs_unsorted": round(unsorted_ms / ms_per_step, 3),
        "phase_ms": {"keys": round(keys_ms, 4), "sort": round(sort_ms, 4), "gather": round(gather_ms, 4),
                     "trace_sorted": round(trace_ms, 4), "trace_unsorted": round(unsorted_ms, 4),
                     "separate_calls_total": round(keys_ms + sort_ms + gather_ms + trace_ms, 4)},
        "sort_gbs": round(sort_bytes / (sort_ms * 1e-3) / 1e9, 1),
        "sort_roofline_frac": round(sort_bytes / (sort_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
        "hbm_copy_gbs": copy_bandwidth(torch, dev, stream),
        "simd_efficiency": {"sorted": round(prof["simd_efficiency"], 3),
                            "unsorted": round(uprof["simd_efficiency"], 3)},
        "per_ray": {"inner_visits": round(prof["inner_visits"] / n, 2), "leaf_visits": round(prof["leaf_visits"] / n, 2),
                    "tri_tests": round(prof["tri_tests"] / n, 2)},
        "hits_scatter_back_equal_unsorted": same,
        "fused_hits_equal_separate_calls": same_fused,
        "roofline": trace_roofline(trace_bytes, trace_ms, n, profiled_traffic(args.key, args.builder),
                                   profiled_valu(args.key, args.builder), prof["inner_visits"], prof["tri_tests"]),
    }
    if "config1" not in args.skip:
        result["config1_soup_65k"] = config1(torch, rr, W, dev, stream)
    if "variants" not in args.skip:
        result["variants"] = variants(torch, rr, scene, rays, n, lo, hi, dev, stream, args.steps, unsorted_ms, uhits)
    if "orders" not in args.skip:
        result["coherence"] = orders(torch, rr, scene, rays, n, lo, hi, dev, stream, args.steps, uhits)
    if "shuffled" not in args.skip:
        result["shuffled_input"] = shuffled_input(torch, rr, W, scene, rays, n, dev, stream, args.steps)
    if "shadow" not in args.skip:
        result["shadow_1080p"] = shadow(torch, rr, W, scene, dev, stream, args.steps)
    if "bounce3" not in args.skip:
        result["bounce3_2160p"] = bounce3(torch, rr, W, scene, dev, stream, max(5, args.steps // 2))
    if "sorts" not in args.skip:
        result["sort_sizes"] = sort_sizes(torch, rr, dev, stream)
    if "batch" not in args.skip:
        result["batched_64_wavefronts"] = batched(torch, rr, W, scene, w, dev, stream)
    scene.close()
    if "serve" not in args.skip:
        loads = [float(x) for x in args.serve_loads.split(",") if x]
        result["served"] = served(torch, rr, W, dev, args.serve_requests, loads)
        main_load = min(result["served"]["loads"], key=lambda r: abs(r["offered_load"] - 0.8))
        result["p50_ms"] = main_load["p50_ms"]
        result["p99_ms"] = main_load["p99_ms"]
        base = min(result["served"]["unsorted_loads"], key=lambda r: abs(r["offered_load"] - 0.8))
        result["unsorted_served_p50_ms"] = base["p50_ms"]
        result["unsorted_served_p99_ms"] = base["p99_ms"]
    if "cpu" not in args.skip:
        result["cpu_baseline"] = cpu_baseline(w, args.key)
    if args.copy_calibration:
        copy_calibration(torch, dev)
    print(json.dumps(result))


def sources_digest() -> str:
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        h.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _profile_values(key: str, builder: int) -> dict:
    """key: value lines of the committed counter summary, or {} when it was
    taken on other sources or another configuration."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_PROFILE)) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith(" "))
    except OSError:
        return {}
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("sources_sha256") != sources_digest() or kv.get("key") != key or kv.get("builder") != str(builder):
        return {}
    return kv


def profiled_traffic(key: str, builder: int):
    """Bytes per sorted-trace launch from the committed counter summary, or
    None when it was taken on other sources or another configuration."""
    try:
        return int(_profile_values(key, builder)["traffic_bytes_per_launch_sorted"])
    except (KeyError, ValueError):
        return None


def profiled_valu(key: str, builder: int):
    """VALU wave instructions per sorted-trace launch (SQ_INSTS_VALU), from
    the same committed summary, or None."""
    try:
        return int(_profile_values(key, builder)["valu_wave_instructions_per_launch_sorted"])
    except (KeyError, ValueError):
        return None


# FP32 operations (add, mul, min/max and compare count 1, fused multiply-add
# 2) of one quantised inner-node test (4 children: 72 for the three axes'
# plane distances, 36 for the slab tests, 5 compares to order the hits) and
# of one triangle test (the full Moller-Trumbore test with its range checks).
FLOPS_PER_INNER_VISIT = 113
FLOPS_PER_TRI_TEST = 54
# FP32 vector peak without packed FP32 instructions (the library is built
# without them): 256 CUs x 4 SIMDs x 16 lanes x 2 (fused multiply-add) x
# 2.4 GHz.  The 157.3 TFLOP/s figure counts packed FP32 issue.
FP32_VECTOR_PEAK_TFLOPS = 78.6
TRACE_BYTES_PER_RAY = 32 + 16  # the ray read, the hit written


def trace_roofline(trace_bytes, trace_ms, n, traffic, valu_instr, inner_visits=None, tri_tests=None):
    """The trace kernel against the HBM roofline: its algorithmic bytes are
    the ray read and the hit written (48 per ray), over the live HIP-event
    launch time.  BVH node and triangle fetches are not algorithmic; the
    measured HBM traffic of a launch (counters) sits in `traffic`.  The
    kernel's counters show VALU instructions issued on nearly every cycle,
    so the arithmetic view (node and triangle tests, visit counts from the
    profiling kernel on the same rays, against the non-packed FP32 vector
    peak) is reported beside it as `alu_view`."""
    gbs = trace_bytes / (trace_ms * 1e-3) / 1e9
    r = {"kernel": "k_trace4 (sorted rays)", "bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5), "traffic": traffic,
         "algorithmic_bytes_per_launch": trace_bytes, "algorithmic_bytes_per_ray": TRACE_BYTES_PER_RAY,
         "launch_ms": round(trace_ms, 4)}
    if traffic:
        r["traffic_over_algorithmic"] = round(traffic / trace_bytes, 2)
    if inner_visits is not None:
        flops = FLOPS_PER_INNER_VISIT * inner_visits + FLOPS_PER_TRI_TEST * tri_tests
        tf = flops / (trace_ms * 1e-3) / 1e12
        r["alu_view"] = {"achieved": round(tf, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "flops_per_launch": int(flops),
                         "flops_per_ray": round(flops / n, 1)}
    # VALU wave instructions per launch (SQ_INSTS_VALU of the committed
    # counter run) and per ray
    r["valu_wave_instructions"] = valu_instr
    r["valu_wave_instructions_per_ray"] = round(valu_instr / n, 1) if valu_instr else None
    return r


def config1(torch, rr, W, dev, stream, reps=50):
    """The small configuration of the method: 65,536 rays (origins uniform
    in the unit cube, directions uniform on the sphere) against 4,096 random
    triangles, median-split BVH, 32-bit origin-direction keys.  Per fused
    call: device time (HIP events, median), wall time per call with the
    calls issued back to back, and the host time to issue one call (no
    synchronisation inside the issuing loop); the unsorted trace alike, and
    that trace through the persistent one-lane kernel for comparison."""
    w = W.soup(seed=1)
    n = w.rays.shape[0]
    out = {"rays": int(n), "triangles": int(w.tris.shape[0]), "bvh": "median split collapsed to 4-wide",
           "key": "od32"}
    with rr.Scene(w.tris, builder=0) as sc:
        lo, hi = sc.bounds()
        p = rr.key_params(1, 32, lo, hi, 0.25)
        rays = torch.from_numpy(w.rays).to(dev)
        hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)

        def fused():
            rr.rr_reorder_and_trace(sc, rays, p, flags=0, hits=hits, ws=ws, want_perm=False, want_count=False)

        def unsorted():
            rr.rr_trace(sc, rays, hits=hits)

        for name, fn in (("fused", fused), ("unsorted_trace", unsorted)):
            for _ in range(5):
                fn()
            dev_ms = median_ms(torch, stream, fn, reps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            t1 = time.perf_counter()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            out[name] = {"device_ms": round(dev_ms, 4), "mrays": round(n / (dev_ms * 1e-3) / 1e6, 2),
                         "wall_ms_per_call": round((t2 - t0) * 1e3 / reps, 4),
                         "host_issue_us_per_call": round((t1 - t0) * 1e6 / reps, 1)}
        out["reorder_vs_unsorted"] = round(out["unsorted_trace"]["device_ms"] / out["fused"]["device_ms"], 3)
        # the same trace through the persistent one-lane kernel (rr_trace_ex),
        # which rr_trace leaves for launches of this size to the four-lane one
        one = torch.empty_like(hits)
        rr.rr_trace(sc, rays, hits=one, refill=8)
        ms1 = median_ms(torch, stream, lambda: rr.rr_trace(sc, rays, hits=one, refill=8), reps)
        rr.rr_trace(sc, rays, hits=hits)
        torch.cuda.synchronize()
        out["unsorted_trace_one_lane_kernel_ms"] = round(ms1, 4)
        out["four_lane_vs_one_lane"] = round(ms1 / out["unsorted_trace"]["device_ms"], 3)
        out["four_lane_hits_equal_one_lane"] = bool(torch.equal(one.view(torch.int32), hits.view(torch.int32)))
    return out


def variants(torch, rr, scene, rays, n, lo, hi, dev, stream, steps, unsorted_ms, uhits):
    """The fused entry point for each key kind: hits in key order, hits
    scattered back to ray order, and tracing through the sorted index; then
    the figure's other layouts and the adaptive and real Two Point
    estimates, hits in key order.  The adaptive table is warmed by two calls
    on the wavefront first and keeps learning in the timed calls (each call
    adds its traced lengths); the real estimate reads the unsorted trace's
    hits."""
    out = {}
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    for name, (kind, bits) in KEYS.items():
        p = rr.key_params(kind, bits, lo, hi, 0.25)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        for flags, tag in ((0, ""), (rr.RR_HITS_ORIGINAL_ORDER, "_scatter_back"), (rr.RR_INDIRECT, "_indirect")):
            def run():
                rr.rr_reorder_and_trace(scene, rays, p, flags=flags, hits=hits, ws=ws, want_perm=False,
                                        want_count=False)
            run(); run()
            ms = median_ms(torch, stream, run, steps)
            out[name + tag] = {"ms": round(ms, 4), "mrays": round(n / (ms * 1e-3) / 1e6, 2),
                               "vs_unsorted": round(unsorted_ms / ms, 3)}
        del ws
    # local (block-wise) sorting instead of the device-wide sort
    for name in ("od32", "ot32", "ot64"):
        kind, bits = KEYS[name]
        p = rr.key_params(kind, bits, lo, hi, 0.25)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        for flag, block in ((rr.RR_LOCAL_SORT_1024, 1024), (rr.RR_LOCAL_SORT_2048, 2048),
                            (rr.RR_LOCAL_SORT_4096, 4096)):
            def run():
                rr.rr_reorder_and_trace(scene, rays, p, flags=flag, hits=hits, ws=ws, want_perm=False, want_count=False)
            run(); run()
            ms = median_ms(torch, stream, run, steps)
            k, idx, _ = rr.rr_compute_keys(rays, p)
            sort_ms = median_ms(torch, stream, lambda: rr.rr_local_sort(k, idx, block=block, key_bits=bits), steps)
            out[f"{name}_local{block}"] = {"ms": round(ms, 4), "mrays": round(n / (ms * 1e-3) / 1e6, 2),
                                           "vs_unsorted": round(unsorted_ms / ms, 3), "sort_ms": round(sort_ms, 4)}
        del ws
    for name, (kind, bits) in METHODS.items():
        aux = None
        if kind == rr.RR_KEY_TWO_POINT_ADAPTIVE:
            aux = rr.LengthTable(rr.key_params(kind, bits, lo, hi, 0.25))
        elif kind == rr.RR_KEY_TWO_POINT_REAL:
            aux = uhits
        p = rr.key_params(kind, bits, lo, hi, 0.25, aux=aux)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        def run():
            rr.rr_reorder_and_trace(scene, rays, p, flags=0, hits=hits, ws=ws, want_perm=False, want_count=False)
        run(); run()
        ms = median_ms(torch, stream, run, steps)
        # the trace alone on this method's order
        k, idx, _ = rr.rr_compute_keys(rays, p)
        rr.rr_sort(k, idx, key_bits=bits)
        srays = rr.rr_gather(rays, idx)
        tms = median_ms(torch, stream, lambda: rr.rr_trace(scene, srays, hits=hits), steps)
        out[name] = {"ms": round(ms, 4), "mrays": round(n / (ms * 1e-3) / 1e6, 2),
                     "vs_unsorted": round(unsorted_ms / ms, 3), "trace_ms": round(tms, 4),
                     "trace_speedup": round(unsorted_ms / tms, 3)}
        del ws
    return out


def orders(torch, rr, scene, rays, n, lo, hi, dev, stream, steps, uhits):
    """Trace time and coherence measure M^64_CPS (Section 4.3) of the
    wavefront in each order: pixel (as generated), shuffled (a seeded random
    permutation, an incoherent order), and sorted by every key method; both
    also relative to pixel order."""
    import numpy as np
    base = rr.key_params(0, 32, lo, hi)
    out = {}
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)

    def measure(r):
        ms = median_ms(torch, stream, lambda: rr.rr_trace(scene, r, hits=hits), steps)
        rr.rr_trace(scene, r, hits=hits)
        _, m = rr.coherence_m64(r, hits, base)
        return ms, float(m.cpu()[0])

    perm = torch.from_numpy(np.random.default_rng(7).permutation(n)).to(dev)
    table = rr.LengthTable(rr.key_params(8, 32, lo, hi))
    # the adaptive table learns from one trace of the wavefront (as after a previous pass)
    table.accumulate(rays, uhits)
    rows = {"pixel": rays, "shuffled": rays.index_select(0, perm).contiguous()}
    for name, (kind, bits) in list(KEYS.items())[1:] + list(METHODS.items()):
        aux = table if kind == 8 else (uhits if kind == 9 else None)
        p = rr.key_params(kind, bits, lo, hi, 0.25, aux=aux)
        k, idx, _ = rr.rr_compute_keys(rays, p)
        rr.rr_sort(k, idx, key_bits=bits)
        rows[name] = rr.rr_gather(rays, idx)
    for name, r in rows.items():
        ms, m = measure(r)
        out[name] = {"trace_ms": round(ms, 4), "m64": round(m, 3)}
    p0 = out["pixel"]
    for v in out.values():
        v["rel_trace"] = round(v["trace_ms"] / p0["trace_ms"], 4)
        v["rel_m64"] = round(v["m64"] / p0["m64"], 4)
    return {"orders": out}


def shuffled_input(torch, rr, W, scene, rays, n, dev, stream, steps):
    """Rays that arrive in an incoherent order (a seeded random permutation
    of the wavefront): their trace against the fused reorder-and-trace call
    on the same input, which sorts them first.  On the headline wavefront
    and on first-bounce rays at 3840x2160 in the 4M-triangle city."""
    def study(sc, r, nrays):
        lo, hi = sc.bounds()
        perm = torch.from_numpy(np.random.default_rng(7).permutation(nrays)).to(dev)
        sh = r.index_select(0, perm).contiguous()
        hits = torch.empty((nrays, 4), dtype=torch.float32, device=dev)
        t_pixel = median_ms(torch, stream, lambda: rr.rr_trace(sc, r, hits=hits), steps)
        t_sh = median_ms(torch, stream, lambda: rr.rr_trace(sc, sh, hits=hits), steps)
        out = {"rays": int(nrays), "trace_generation_order_ms": round(t_pixel, 4),
               "trace_shuffled_ms": round(t_sh, 4), "fused_from_shuffled": {}}
        for name in ("od32", "origin", "ot64"):
            kind, bits = METHODS[name] if name in METHODS else KEYS[name]
            p = rr.key_params(kind, bits, lo, hi, 0.25)
            ws = rr.workspace(rr.reorder_workspace_size(nrays, p), dev)

            def run():
                rr.rr_reorder_and_trace(sc, sh, p, flags=0, hits=hits, ws=ws, want_perm=False, want_count=False)
            run()
            ms = median_ms(torch, stream, run, steps)
            out["fused_from_shuffled"][name] = {"ms": round(ms, 4), "vs_shuffled_trace": round(t_sh / ms, 3)}
            del ws
        del sh, hits
        return out

    res = {"city1M_bounce2_1080p": study(scene, rays, n)}
    c, r = city4m_bounce1_2160p(W)
    with rr.Scene(c.tris) as sc4:
        rd = torch.from_numpy(r).to(dev)
        res["city4M_bounce1_2160p"] = study(sc4, rd, r.shape[0])
        del rd
    torch.cuda.empty_cache()
    return res


def city4m_bounce1_2160p(W):
    """The 4M-triangle city (the grid city scaled 2x2) and its first-bounce
    rays at 3840x2160 that left a surface (the dead slots dropped)."""
    c = W.city(5, 200, 200, 3_520_000)
    r = W.camera_rays(5, 3840, 2160, (100.0, 120.0, 100.0))
    r, alive = W.bounce(c, 5, 300, r, np.ones(r.shape[0], np.uint8))
    return c, np.ascontiguousarray(r[alive.astype(bool)])


def trace_orders_4m(torch, rr, W, dev, args):
    """For counter runs: the first-bounce rays of the 4M-triangle city traced
    in three orders, a seeded random permutation (shuffled), that order
    sorted by origin-direction 32-bit keys (keys, sort and gather run once
    before), and the generation order.  The trace launches come in that
    order, warmup and steps alike, so dispatch i is order i mod 3."""
    c, r = city4m_bounce1_2160p(W)
    n = r.shape[0]
    with rr.Scene(c.tris) as sc:
        lo, hi = sc.bounds()
        gen = torch.from_numpy(r).to(dev)
        perm = torch.from_numpy(np.random.default_rng(7).permutation(n)).to(dev)
        sh = gen.index_select(0, perm).contiguous()
        p = rr.key_params(1, 32, lo, hi, 0.25)
        k, idx, _ = rr.rr_compute_keys(sh, p)
        rr.rr_sort(k, idx, key_bits=32)
        srt = rr.rr_gather(sh, idx)
        hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        for _ in range(args.warmup + args.steps):
            for rays in (sh, srt, gen):
                rr.rr_trace(sc, rays, hits=hits)
        torch.cuda.synchronize()
        if args.copy_calibration:
            copy_calibration(torch, dev)
        print(json.dumps({"phases": "trace4m", "rays": int(n), "triangles": int(c.tris.shape[0]),
                          "orders": ["shuffled", "od32_sorted", "generation"], "steps": args.steps,
                          "warmup": args.warmup, "sources_sha256": sources_digest()}))


# the batch's launch shape for profiler runs: the autotuner's choice on the
# 64-wavefront batch (8-bit digits, 8 keys per thread, refill 8, fixed tile
# order, 256-thread trace blocks)
BATCH_PROFILE_SHAPE = {"digit_bits": 8, "keys_per_thread": 8, "refill": 8, "tile_order": 1, "trace_block": 256}


def batch_only(torch, rr, W, scene, w, dev, args):
    """For profiler runs: the 64-wavefront batch graph in BATCH_PROFILE_SHAPE,
    warmup + steps launches."""
    segs, keep, total, _ = batch_segments(torch, rr, W, scene, w, dev)
    with rr.Batch(scene, max_rays=total, max_segments=len(segs), config=BATCH_PROFILE_SHAPE) as b:
        for _ in range(args.warmup + args.steps):
            b.run(segs, flags=0)
        torch.cuda.synchronize()
    print(json.dumps({"phases": "batch", "segments": len(segs), "rays": total, "shape": BATCH_PROFILE_SHAPE,
                      "steps": args.steps, "warmup": args.warmup}))


def sorts_only(torch, rr, W, dev, args):
    """For counter runs: device-wide sorts of 64-bit pairs, warmup and steps
    alike, in this order: the headline's Two Point keys (2,073,600), random
    keys (2,073,600), random keys (8,294,400), random keys (67,108,864, more
    than the 256 MB MALL holds); each input sorted by the most-significant-
    digit sort (rr_sort_msd: setup, histogram, two scatter passes with a
    histogram between them, then both bucket kernels, of which one returns
    at once: the wave kernel when no bucket holds more than 512 keys, else
    the batch kernel) and then by the LSD sort (rr_sort_ex with rr_sort's
    tile size: setup, histogram, 8 scatter passes)."""
    w = W.bounce2_1080p()
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
    rays = torch.from_numpy(w.rays).to(dev)
    k_real, _, _ = rr.rr_compute_keys(rays, rr.key_params(2, 64, lo, hi, 0.25))
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    cases = [("ot64_headline", k_real),
             ("random_2M", torch.randint(-(1 << 62), 1 << 62, (k_real.shape[0],), dtype=torch.int64, device=dev,
                                         generator=g)),
             ("random_8M", torch.randint(-(1 << 62), 1 << 62, (8294400,), dtype=torch.int64, device=dev,
                                         generator=g)),
             ("random_64M", torch.randint(-(1 << 62), 1 << 62, (1 << 26,), dtype=torch.int64, device=dev,
                                          generator=g))]
    work = []
    for name, k0 in cases:
        m = k0.shape[0]
        work.append((k0, k0.clone(), torch.empty(m, dtype=torch.int32, device=dev),
                     rr.workspace(rr.sort_workspace_size(m, 64), dev)))
    torch.cuda.synchronize()
    for _ in range(args.warmup + args.steps):
        for k0, k, idx, ws in work:
            for msd in (True, False):
                k.copy_(k0)
                torch.arange(k0.shape[0], dtype=torch.int32, device=dev, out=idx)
                if msd:
                    rr.rr_sort(k, idx, ws=ws, msd=True)
                else:
                    rr.rr_sort(k, idx, ws=ws, keys_per_thread=16 if k0.shape[0] >= 1 << 24 else 8)
    torch.cuda.synchronize()
    if args.copy_calibration:
        copy_calibration(torch, dev)
    print(json.dumps({"phases": "sort", "cases": [c[0] for c in cases], "steps": args.steps, "warmup": args.warmup}))


def shadow(torch, rr, W, scene, dev, stream, steps):
    """Two shadow rays per primary hit point of the 1080p view (4,147,200
    rays) toward a square light of side 5% of the extent, traced any-hit:
    unsorted, and reordered by each 32-bit key method (trace alone and the
    fused call)."""
    ws_ = W.shadow_1080p()
    n = ws_.rays.shape[0]
    rays = torch.from_numpy(ws_.rays).to(dev)
    lo, hi = scene.bounds()
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    un = median_ms(torch, stream, lambda: rr.rr_trace_any(scene, rays, hits=hits), steps)
    occluded = float((hits[:, 1].view(torch.int32) >= 0).float().mean().cpu())
    out = {"rays": int(n), "occluded_fraction": round(occluded, 4), "unsorted_trace_ms": round(un, 4),
           "unsorted_mrays": round(n / (un * 1e-3) / 1e6, 2), "methods": {}}
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    for name, (kind, bits) in [("od32", (1, 32)), ("ot32", (2, 32)), ("origin", (3, 32)), ("costa", (4, 32)),
                               ("aila", (5, 32)), ("aila_compact", (6, 32)), ("octahedron", (7, 32))]:
        p = rr.key_params(kind, bits, lo, hi, 0.25)
        k, idx, _ = rr.rr_compute_keys(rays, p)
        rr.rr_sort(k, idx, key_bits=bits)
        srays = rr.rr_gather(rays, idx)
        tms = median_ms(torch, stream, lambda: rr.rr_trace_any(scene, srays, hits=hits), steps)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        def run():
            rr.rr_reorder_and_trace(scene, rays, p, flags=rr.RR_ANY_HIT, hits=hits, count=cnt, ws=ws,
                                    want_perm=False)
        run()
        ms = median_ms(torch, stream, run, steps)
        out["methods"][name] = {"trace_ms": round(tms, 4), "trace_speedup": round(un / tms, 3),
                                "fused_ms": round(ms, 4), "fused_vs_unsorted": round(un / ms, 3)}
        del ws, srays
    return out


def bounce3(torch, rr, W, scene, dev, stream, steps):
    """3840x2160 bounce-3 slots on the same city; terminated rays are
    compacted before the sort.  Rates count live rays."""
    w3 = W.bounce3_2160p()
    rays = torch.from_numpy(w3.rays).to(dev)
    alive = torch.from_numpy(w3.alive).to(dev)
    n = w3.rays.shape[0]
    live = int(w3.alive.sum())
    lo, hi = scene.bounds()
    out = {"slots": int(n), "live": live}
    hits = torch.empty((n, 4), dtype=torch.float32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    for name in ("none", "od32", "od64", "ot64"):
        kind, bits = KEYS[name]
        p = rr.key_params(kind, bits, lo, hi, 0.25)
        ws = rr.workspace(rr.reorder_workspace_size(n, p), dev)
        for flags, tag in ((0, ""), (rr.RR_HITS_ORIGINAL_ORDER, "_scatter_back")):
            def run():
                rr.rr_reorder_and_trace(scene, rays, p, alive=alive, flags=flags, hits=hits, count=cnt, ws=ws,
                                        want_perm=False)
            run()
            ms = median_ms(torch, stream, run, steps)
            out[name + tag] = {"ms": round(ms, 4), "mrays": round(live / (ms * 1e-3) / 1e6, 2)}
        assert int(cnt.cpu()[0]) == live
        del ws
    return out


def sort_sizes(torch, rr, dev, stream, reps=15):
    """rr_sort of seeded uniform random keys with indices 0..n-1 at the two
    wavefront sizes and at 64M pairs (beyond the 256 MB last-level cache),
    32- and 64-bit keys, against the HBM roofline of the 8-bit schedule; for
    64-bit keys also rr_sort_msd of the same keys (entries ending in _msd).
    Every sort starts from the same input, restored by a copy: the time is
    the median of copy and sort issued back to back, minus the median of the
    copy alone (a single call bracketed by events would also time the host
    issuing its kernels, longer than a sort of 2M pairs).  Each result is
    checked (keys non-decreasing as unsigned words, equal keys in ascending
    index order, indices a permutation)."""
    out = {}
    for n in (2073600, 8294400, 67108864):
        for bits in (32, 64):
            g = torch.Generator(device=dev)
            g.manual_seed(n + bits)
            dt = torch.int64 if bits == 64 else torch.int32
            lo, hi = (-(1 << 63), (1 << 63) - 1) if bits == 64 else (-(1 << 31), (1 << 31) - 1)
            k0 = torch.randint(lo, hi, (n,), dtype=dt, device=dev, generator=g)
            i0 = torch.arange(n, dtype=torch.int32, device=dev)
            k = torch.empty_like(k0)
            i = torch.empty_like(i0)
            ws = rr.workspace(rr.sort_workspace_size(n, bits), dev)
            def restore():
                k.copy_(k0)
                i.copy_(i0)

            for msd in ((False, True) if bits == 64 else (False,)):
                def run():
                    restore()
                    rr.rr_sort(k, i, key_bits=bits, ws=ws, msd=msd)

                run()
                ms = median_ms(torch, stream, run, reps) - median_ms(torch, stream, restore, reps)
                run()
                torch.cuda.synchronize()
                flip = k ^ torch.tensor(lo, dtype=dt, device=dev)  # unsigned order as signed order
                ok = bool((flip[1:] >= flip[:-1]).all())
                ties = flip[1:] == flip[:-1]
                ok = ok and bool((i[1:][ties] > i[:-1][ties]).all())
                ok = ok and bool(torch.equal(torch.sort(i).values, i0))
                ok = ok and bool(torch.equal(k0[i.long()], k))
                b = sort_algorithmic_bytes(n, bits)
                out[f"u{bits}_n{n}" + ("_msd" if msd else "")] = {
                    "ms": round(ms, 4), "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                    "roofline_frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3), "ok": ok}
                del flip, ties
            del k0, i0, k, i, ws
            torch.cuda.empty_cache()
    return out


def batch_segments(torch, rr, W, scene, w, dev):
    """The 64 wavefronts of the batched section: sizes log-uniform in
    [4K, 2M], each drawn from the primary or bounce 1-4 rays of the 1920x1080
    city view, Two Point 64-bit keys.  Returns (segments, tensors kept alive,
    total rays, the key parameters)."""
    c = w.city
    pools = []
    r = W.camera_rays(4, 1920, 1080, (c.nx / 2.0, 0.6 * max(c.nx, c.nz), c.nz / 2.0))
    alive = np.ones(r.shape[0], np.uint8)
    pools.append(r)
    for k in range(4):
        r, alive = W.bounce(c, 4, 200 + k, r, alive)
        pools.append(np.ascontiguousarray(r[alive.astype(bool)]))
    sizes = W.segment_sizes(4)
    lo, hi = scene.bounds()
    key = rr.key_params(2, 64, lo, hi, 0.25)
    segs, keep = [], []
    for i, m in enumerate(sizes):
        depth = int(W.rngu(4, 41, i) * 5)
        pool = pools[depth]
        ix = W.sample_indices(4, 1000 + i, int(m), pool.shape[0])
        rays = torch.from_numpy(np.ascontiguousarray(pool[ix])).to(dev)
        hits = torch.empty((int(m), 4), dtype=torch.float32, device=dev)
        keep.append((rays, hits))
        segs.append(rr.segment(rays, hits, key))
    return segs, keep, int(sizes.sum()), key


def batched(torch, rr, W, scene, w, dev, stream):
    """The 64 wavefronts reordered and traced in one graph launch (shape
    from the autotuner), against the same wavefronts one call each."""
    segs, keep, total, key = batch_segments(torch, rr, W, scene, w, dev)
    out = {"segments": len(segs), "rays": total}
    with rr.Batch(scene, max_rays=total, max_segments=len(segs)) as b:
        t0 = time.perf_counter()
        best, tuned_ms = b.autotune(segs, reps=2)
        out["autotune_s"] = round(time.perf_counter() - t0, 2)
        out["config"] = best
        try:
            rr.save_tuned(total, 64, best, tuned_ms)
        except OSError:
            pass
        b.run(segs, flags=0)
        ms = median_ms(torch, stream, lambda: b.run(segs, flags=0), 10)
        out["graph_ms"] = round(ms, 3)
        out["mrays"] = round(total / (ms * 1e-3) / 1e6, 2)
        # the same graph with every segment unsorted (key kind none): the
        # same-form baseline of the reordered batch
        none = rr.key_params(0, 32, *scene.bounds())
        usegs = [rr.segment(r, h, none) for r, h in keep]
        b.run(usegs, flags=0)
        ms_n = median_ms(torch, stream, lambda: b.run(usegs, flags=0), 10)
        out["graph_unsorted_ms"] = round(ms_n, 3)
        out["graph_unsorted_mrays"] = round(total / (ms_n * 1e-3) / 1e6, 2)
        out["graph_reorder_vs_unsorted"] = round(ms_n / ms, 3)
        ms_o = median_ms(torch, stream, lambda: b.run(segs, flags=rr.RR_HITS_ORIGINAL_ORDER), 5)
        out["graph_scatter_back_ms"] = round(ms_o, 3)
        # the same wavefronts one call each
        wss = {}
        def per_call():
            for (rays, hits) in keep:
                m = rays.shape[0]
                if m not in wss:
                    wss[m] = rr.workspace(rr.reorder_workspace_size(m, key), dev)
                rr.rr_reorder_and_trace(scene, rays, key, flags=0, hits=hits, ws=wss[m], want_perm=False)
        per_call()
        ms_p = median_ms(torch, stream, per_call, 3)
        out["per_call_ms"] = round(ms_p, 3)
        out["per_call_mrays"] = round(total / (ms_p * 1e-3) / 1e6, 2)
        # host time to issue the 64 calls (no synchronisation in between)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        per_call()
        t1 = time.perf_counter()
        torch.cuda.synchronize()
        out["per_call_host_issue_ms"] = round((t1 - t0) * 1e3, 3)
        # unsorted trace of the same rays, one call each
        def unsorted():
            for (rays, hits) in keep:
                rr.rr_trace(scene, rays, hits=hits)
        ms_u = median_ms(torch, stream, unsorted, 3)
        out["unsorted_trace_mrays"] = round(total / (ms_u * 1e-3) / 1e6, 2)
    return out


# the server's shape in the served section: 3 slots, batches of at most 2M
# rays, requests in ray order above 512K rays served as parts of 512K (every
# request of a batch completes with the batch, and concurrent batches share
# the device, so smaller batches shorten the latency tail)
SERVE_SHAPE = dict(slots=3, hbm_budget_bytes=32 << 30, max_batch_rays=1 << 21, max_batch_requests=16,
                   split_rays=1 << 19)
# the earlier shape (2 slots, no parts), run at 0.8 load for comparison
SERVE_SHAPE_2SLOTS = dict(slots=2, hbm_budget_bytes=32 << 30, max_batch_rays=1 << 23, max_batch_requests=16,
                          split_rays=0)


def served(torch, rr, W, dev, n_req, loads):
    """Poisson streams of requests (ray counts log-uniform in [16K, 4M], key
    kind drawn per request from none / OD-32 / OD-64 / OT-64, rays drawn
    from the primary, bounce-1 and bounce-2 rays of a 3840x2160 view) against
    the grid city scaled 2x2 (~4M triangles), served with continuous
    batching (SERVE_SHAPE) under a 32 GB workspace budget, at each offered
    load (a fraction of the measured batched capacity).  The same stream
    with every request unsorted (key kind none) is served at the same loads
    and arrival times: the same-form baseline; and the mixed stream with the
    2-slot shape without parts at 0.8 load."""
    c = W.city(5, 200, 200, 3_520_000)
    scene = rr.Scene(c.tris)
    lo, hi = scene.bounds()
    r = W.camera_rays(5, 3840, 2160, (100.0, 120.0, 100.0))
    pools = [torch.from_numpy(r).to(dev)]
    alive = np.ones(r.shape[0], np.uint8)
    for k in range(2):
        r, alive = W.bounce(c, 5, 300 + k, r, alive)
        pools.append(torch.from_numpy(np.ascontiguousarray(r[alive.astype(bool)])).to(dev))
    kinds = ["none", "od32", "od64", "ot64"]
    none = rr.key_params(0, 32, lo, hi, 0.25)
    warm = 50
    reqs = []
    for i in range(n_req + warm):
        m = int(math.floor(math.exp(math.log(16384) + W.rngu(5, 50, i) * (math.log(1 << 22) - math.log(16384)))))
        kname = kinds[int(W.rngu(5, 51, i) * 4)]
        pool = pools[int(W.rngu(5, 52, i) * 3)]
        ix = torch.from_numpy(W.sample_indices(5, 2000 + i, m, pool.shape[0])).to(dev)
        rays = pool.index_select(0, ix).contiguous()
        hits = torch.empty((m, 4), dtype=torch.float32, device=dev)
        kind, bits = KEYS[kname]
        reqs.append((rays, hits, rr.key_params(kind, bits, lo, hi, 0.25), kname))
    torch.cuda.synchronize()
    # batched capacity on this scene, to set the arrival rates
    segs = [rr.segment(a, b, k) for a, b, k, _ in reqs[warm:warm + 8]]
    stream = torch.cuda.current_stream()
    with rr.Batch(scene, max_rays=sum(int(s.n) for s in segs), max_segments=8) as b:
        b.run(segs)
        ms = median_ms(torch, stream, lambda: b.run(segs), 3)
    cap_rays_s = sum(int(s.n) for s in segs) / (ms * 1e-3)
    mean_n = float(np.mean([x[0].shape[0] for x in reqs[warm:]]))
    out = {"scene_triangles": int(c.tris.shape[0]), "requests": n_req, "shape": SERVE_SHAPE,
           "capacity_mrays": round(cap_rays_s / 1e6, 1), "mean_request_rays": int(mean_n), "loads": [],
           "unsorted_loads": []}

    def stream_run(cfg, load, li, unsorted):
        lam = load * cap_rays_s / mean_n
        with rr.Server(scene, **cfg) as sv:
            sv.start()
            for rays, hits, key, _ in reqs[:warm]:
                sv.submit(rays, hits, none if unsorted else key, sync=False)
            sv.drain(300.0)
        with rr.Server(scene, **cfg) as sv:
            t = 0.02
            for i, (rays, hits, key, _) in enumerate(reqs[warm:]):
                sv.submit(rays, hits, none if unsorted else key, arrival_s=t, sync=False)
                t += -math.log(1.0 - W.rngu(5, 60 + li, i)) / lam
            sv.start()
            sv.drain(600.0)
            st = sv.stats()
        row = {"offered_load": load, "arrival_rate_per_s": round(lam, 1)}
        row.update({k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()})
        return row

    for li, load in enumerate(loads):
        out["loads"].append(stream_run(SERVE_SHAPE, load, li, False))
        out["unsorted_loads"].append(stream_run(SERVE_SHAPE, load, li, True))
    li8 = min(range(len(loads)), key=lambda i: abs(loads[i] - 0.8)) if loads else 0
    if loads:
        out["two_slots_no_parts_at_0.8"] = stream_run(SERVE_SHAPE_2SLOTS, loads[li8], li8, False)
    scene.close()
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
    return {"value": round(n / s / 1e6, 3), "unit": "MRays/s", "cores": threads, "cpu": cpu_model(),
            "kind": "oracle",
            "sample": f"the whole {n}-ray wavefront, median of 3 runs ({s:.2f} s each); keys and trace "
                      f"threaded over {threads} host threads, sort single-threaded (numpy lexsort)"}


def copy_bandwidth(torch, dev, stream):
    """Measured device-copy bandwidth beside the 8 TB/s vendor peak: a plain
    1 GiB device-to-device copy, bytes read plus bytes written over its
    median time of 5 (after one warm-up)."""
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    ms = median_ms(torch, stream, lambda: b.copy_(a), 5)
    del a, b
    return round(2 * (1 << 30) / (ms * 1e-3) / 1e9, 1)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
