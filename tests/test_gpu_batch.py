"""GPU tests of the batched and serving layers.

Invariants: every segment of a batch gives exactly the results of the
per-call path on that wavefront alone (hits bit for bit, permutation equal to
the oracle's stable order); every launch shape gives the same results; the
captured graph replayed many times (with eager work and synchronisations in
between) matches the eager launches; a served request's hits equal the
request traced alone, whatever else was in flight.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2506_11273_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def city(rr):
    w = W.city_small(seed=21, width=200, height=120, depth=1, n=16, n_clutter=20000)
    scene = rr.Scene(w.tris)
    yield w, scene
    scene.close()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


KINDS = [(0, 32), (1, 32), (1, 64), (2, 32), (2, 64)]


def make_segments(rr, w, scene, sizes, seed=0):
    """Segments cut from a pool of rays, each with its own key method."""
    lo, hi = scene.bounds()
    rng = np.random.default_rng(seed)
    pool = w.rays
    out = []
    for k, n in enumerate(sizes):
        idx = rng.integers(0, pool.shape[0], n)
        rays = to_dev(pool[idx]) if n else torch.empty((0, 8), dtype=torch.float32, device=DEV)
        kind, bits = KINDS[k % len(KINDS)]
        out.append({"rays": rays, "rays_np": pool[idx], "key": rr.key_params(kind, bits, lo, hi, 0.25),
                    "kind": kind, "bits": bits, "lo": lo, "hi": hi,
                    "hits": torch.empty((n, 4), dtype=torch.float32, device=DEV),
                    "perm": torch.empty(max(n, 1), dtype=torch.int32, device=DEV)})
    return out


def seg_structs(rr, segs):
    return [rr.segment(s["rays"], s["hits"], s["key"], perm=s["perm"], n=s["rays"].shape[0]) for s in segs]


def expected(rr, scene, s):
    """Per-call results on the segment alone: hits in ray order and the
    oracle's stable permutation."""
    n = s["rays"].shape[0]
    hits = rr.hits_to_numpy(rr.rr_trace(scene, s["rays"])) if n else np.empty(0, O.HIT_DTYPE)
    if s["kind"] == 0:
        perm = np.arange(n, dtype=np.uint32)
    else:
        k = O.keys(s["rays_np"], s["kind"], s["bits"], s["lo"], s["hi"], 0.25)
        _, perm = O.sort_pairs(k)
    return hits, perm


def check(rr, scene, segs, what=""):
    torch.cuda.synchronize()
    for j, s in enumerate(segs):
        n = s["rays"].shape[0]
        hits, perm = expected(rr, scene, s)
        got = rr.hits_to_numpy(s["hits"][:n])
        assert got.tobytes() == hits.tobytes(), f"{what} segment {j} hits"
        assert np.array_equal(s["perm"][:n].cpu().numpy().view(np.uint32), perm), f"{what} segment {j} perm"


SIZES = [5000, 0, 1, 4097, 30000, 777, 65536, 12345, 2, 100000]


def test_batch_equals_per_call(rr, city):
    w, scene = city
    segs = make_segments(rr, w, scene, SIZES, seed=1)
    with rr.Batch(scene, max_rays=sum(SIZES), max_segments=16) as b:
        b.run(seg_structs(rr, segs))
        check(rr, scene, segs, "graph")
        for s in segs:
            s["hits"].fill_(7.0)
        b.run(seg_structs(rr, segs), flags=rr.RR_HITS_ORIGINAL_ORDER | rr.RR_BATCH_EAGER)
        check(rr, scene, segs, "eager")


def test_batch_all_32bit_keys_and_sorted_order_hits(rr, city):
    w, scene = city
    segs = make_segments(rr, w, scene, [3000, 9000, 20000], seed=2)
    lo, hi = scene.bounds()
    for s in segs:
        s["key"] = rr.key_params(1, 32, lo, hi)
        s["kind"], s["bits"] = 1, 32
    with rr.Batch(scene, max_rays=40000, max_segments=4) as b:
        b.run(seg_structs(rr, segs), flags=0)
        torch.cuda.synchronize()
        for s in segs:
            hits, perm = expected(rr, scene, s)
            got = rr.hits_to_numpy(s["hits"])
            assert got.tobytes() == hits[perm].tobytes()  # sorted order = ray order through perm


def test_graph_replays_match_eager(rr, city):
    w, scene = city
    segs = make_segments(rr, w, scene, [20000, 3000, 50000, 1], seed=3)
    with rr.Batch(scene, max_rays=80000, max_segments=8) as b:
        b.run(seg_structs(rr, segs), flags=rr.RR_HITS_ORIGINAL_ORDER | rr.RR_BATCH_EAGER)
        torch.cuda.synchronize()
        ref = [(s["hits"].clone(), s["perm"].clone()) for s in segs]
        for rep in range(5):
            for s in segs:
                s["hits"].zero_()
                s["perm"].zero_()
            torch.cuda.synchronize()
            b.run(seg_structs(rr, segs))
            torch.cuda.synchronize()
            for (h, p), s in zip(ref, segs):
                assert torch.equal(s["hits"].view(torch.int32), h.view(torch.int32)), rep
                assert torch.equal(s["perm"], p), rep
            # unrelated eager work between replays
            x = torch.randn(1 << 16, device=DEV)
            assert float(x.sum()) == pytest.approx(float(x.cpu().sum()), rel=1e-3, abs=1e-2)


def test_batch_mix_changes_between_runs(rr, city):
    w, scene = city
    with rr.Batch(scene, max_rays=200000, max_segments=16) as b:
        for seed, sizes in enumerate([[1000, 2000], [150000, 3, 40000], [64], [0, 0, 5000]]):
            segs = make_segments(rr, w, scene, sizes, seed=10 + seed)
            b.run(seg_structs(rr, segs))
            check(rr, scene, segs, f"mix {seed}")


def test_every_launch_shape_gives_identical_results(rr, city):
    w, scene = city
    segs = make_segments(rr, w, scene, [30000, 7000, 60000], seed=4)
    with rr.Batch(scene, max_rays=100000, max_segments=4) as b:
        outs = []
        for db in (8, 4):
            for kpt in (16, 8):
                for refill in (1, 16, 64):
                    for order in (rr.RR_TILES_COUNTER, rr.RR_TILES_FIXED):
                        for block in (128, 256, 512):
                            b.set_config({"digit_bits": db, "keys_per_thread": kpt, "refill": refill,
                                          "tile_order": order, "trace_block": block})
                            cfg = b.info()["config"]
                            assert cfg["tile_order"] == order and cfg["trace_block"] == block
                            b.run(seg_structs(rr, segs))
                            torch.cuda.synchronize()
                            outs.append([(s["hits"].cpu().numpy().tobytes(), s["perm"].cpu().numpy().tobytes())
                                         for s in segs])
        assert all(o == outs[0] for o in outs)
        for bad in ({"tile_order": 2}, {"trace_block": 64}, {"trace_block": 1024}):
            with pytest.raises(rr.RRError):
                b.set_config(dict({"digit_bits": 8, "keys_per_thread": 16, "refill": 8}, **bad))
        best, ms = b.autotune(seg_structs(rr, segs), reps=2)
        assert best["digit_bits"] in (4, 8) and best["tile_order"] in (0, 1) and ms > 0
        assert best["trace_block"] in (128, 256, 512)
        b.run(seg_structs(rr, segs))
        check(rr, scene, segs, "tuned")


def test_batch_rejects_bad_input(rr, city):
    w, scene = city
    segs = make_segments(rr, w, scene, [1000, 1000], seed=5)
    with rr.Batch(scene, max_rays=1500, max_segments=1) as b:
        with pytest.raises(rr.RRError):
            b.run(seg_structs(rr, segs))          # more segments than the batch holds
    with rr.Batch(scene, max_rays=1500, max_segments=4) as b:
        with pytest.raises(rr.RRError) as e:
            b.run(seg_structs(rr, segs))          # more rays than the capacity
        assert e.value.status == -6


# ---------------------------------------------------------------- serving

def test_server_results_equal_alone_and_overlap(rr, city):
    w, scene = city
    rng = np.random.default_rng(6)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(500), np.log(60000), 24))]
    segs = make_segments(rr, w, scene, sizes, seed=6)
    with rr.Server(scene, slots=3, hbm_budget_bytes=8 << 30, max_batch_rays=150000, max_batch_requests=8) as sv:
        sv.start()
        ids = []
        for k, s in enumerate(segs):
            ids.append(sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.002 * k))
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
        stats = sv.stats()
    assert all(x["status"] == 0 and x["done"] for x in st)
    assert stats["completed"] == len(segs) and stats["failed"] == 0
    assert stats["p99_ms"] >= stats["p50_ms"] > 0 and stats["rays"] == sum(sizes)
    # each request's hits equal the request traced alone
    for j, s in enumerate(segs):
        hits, _ = expected(rr, scene, s)
        assert rr.hits_to_numpy(s["hits"]).tobytes() == hits.tobytes(), j
    # latency is measured from arrival, and nothing starts before it arrives
    for x in st:
        assert x["start_s"] >= x["arrival_s"] - 1e-6 and x["finish_s"] >= x["start_s"]


def test_server_sample_against_the_oracle(rr, city):
    """A seeded sample of 32 served requests (mixed sizes and key methods,
    overlapping on three slots): each request's hits, in ray order, equal
    the oracle's trace of that request bit for bit."""
    w, scene = city
    bvh = O.BVH(w.tris)
    rng = np.random.default_rng(32)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(64), np.log(20000), 32))]
    segs = make_segments(rr, w, scene, sizes, seed=32)
    with rr.Server(scene, slots=3, hbm_budget_bytes=8 << 30, max_batch_rays=60000, max_batch_requests=6) as sv:
        sv.start()
        ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.001 * k) for k, s in enumerate(segs)]
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
    assert all(x["status"] == 0 and x["done"] for x in st)
    torch.cuda.synchronize()
    for j, s in enumerate(segs):
        want = bvh.trace(s["rays_np"])
        assert rr.hits_to_numpy(s["hits"]).tobytes() == want.tobytes(), j


def test_direct_calls_beside_a_busy_server(rr, city):
    """The caller's own fused calls and batches, on a stream of its own,
    while the server's thread runs batches on its streams: both give the
    results each gives alone (the per-call sort waits through its bounded
    look-back fallback when the server holds CUs)."""
    w, scene = city
    lo, hi = scene.bounds()
    rng = np.random.default_rng(41)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(2000), np.log(80000), 24))]
    segs = make_segments(rr, w, scene, sizes, seed=41)
    direct = to_dev(w.rays[:150001])
    p = rr.key_params(O.KIND_OT, 64, lo, hi, 0.25)
    want_direct = rr.hits_to_numpy(rr.rr_reorder_and_trace(scene, direct, p, flags=rr.RR_HITS_ORIGINAL_ORDER)[0])
    own = make_segments(rr, w, scene, [3000, 40000, 777], seed=42)
    own_structs = seg_structs(rr, own)
    side = torch.cuda.Stream()
    with rr.Server(scene, slots=2, hbm_budget_bytes=8 << 30, max_batch_rays=120000, max_batch_requests=8) as sv, \
            rr.Batch(scene, max_rays=50000, max_segments=4) as b:
        sv.start()
        ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.0005 * k) for k, s in enumerate(segs)]
        got = []
        with torch.cuda.stream(side):
            for _ in range(6):
                h, _, _ = rr.rr_reorder_and_trace(scene, direct, p, flags=rr.RR_HITS_ORIGINAL_ORDER)
                b.run(own_structs)
                got.append(h)
        side.synchronize()
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
    assert all(x["status"] == 0 and x["done"] for x in st)
    for h in got:
        assert rr.hits_to_numpy(h).tobytes() == want_direct.tobytes()
    check(rr, scene, own, "own batch")
    for j, s in enumerate(segs):
        hits, _ = expected(rr, scene, s)
        assert rr.hits_to_numpy(s["hits"]).tobytes() == hits.tobytes(), j


def test_server_batches_and_overlaps_under_load(rr, city):
    w, scene = city
    sizes = [40000] * 16
    segs = make_segments(rr, w, scene, sizes, seed=7)
    with rr.Server(scene, slots=2, hbm_budget_bytes=8 << 30, max_batch_rays=120000, max_batch_requests=4) as sv:
        sv.start()
        ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.0) for s in segs]
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
        stats = sv.stats()
    assert max(x["batch_requests"] for x in st) > 1          # requests were batched together
    assert stats["batches"] < len(segs)
    # two batches were on the device at the same time
    spans = sorted({(x["start_s"], x["finish_s"]) for x in st})
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    for j, s in enumerate(segs):
        hits, _ = expected(rr, scene, s)
        assert rr.hits_to_numpy(s["hits"]).tobytes() == hits.tobytes(), j


def test_server_admission_and_rejection(rr, city):
    w, scene = city
    # a budget too small for one slot
    with pytest.raises(rr.RRError) as e:
        rr.Server(scene, slots=1, hbm_budget_bytes=1 << 20, max_batch_rays=100000)
    assert e.value.status == -6
    segs = make_segments(rr, w, scene, [5000, 200000, 3000], seed=8)
    with rr.Server(scene, slots=1, hbm_budget_bytes=8 << 30, max_batch_rays=100000) as sv:
        sv.start()
        a = sv.submit(segs[0]["rays"], segs[0]["hits"], segs[0]["key"])
        with pytest.raises(rr.RRError) as e:
            sv.submit(segs[1]["rays"], segs[1]["hits"], segs[1]["key"])   # larger than any batch
        assert e.value.status == -6
        host = torch.zeros((10, 8))
        lib = rr.load()
        import ctypes
        rid = ctypes.c_int64()
        bad = lib.rr_server_submit(sv.handle, host.data_ptr(), 10, ctypes.byref(segs[0]["key"]),
                                   segs[0]["hits"].data_ptr(), 1, -1.0, ctypes.byref(rid))
        assert bad == -1                                                   # host memory refused at submit
        c = sv.submit(segs[2]["rays"], segs[2]["hits"], segs[2]["key"])
        sv.drain(60.0)
        assert sv.wait(a)["status"] == 0 and sv.wait(c)["status"] == 0
        assert sv.stats()["rejected"] == 1
    for s in (segs[0], segs[2]):
        hits, _ = expected(rr, scene, s)
        assert rr.hits_to_numpy(s["hits"]).tobytes() == hits.tobytes()


def test_server_hit_order_per_request(rr, city):
    """Requests asking for hits in key order (flags 0) and in ray order,
    interleaved: each batch holds one hit order, and every request gets its
    own order (key order = the ray-order hits permuted by the oracle's stable
    order)."""
    w, scene = city
    rng = np.random.default_rng(51)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(300), np.log(30000), 16))]
    segs = make_segments(rr, w, scene, sizes, seed=51)
    with rr.Server(scene, slots=2, hbm_budget_bytes=8 << 30, max_batch_rays=100000, max_batch_requests=8) as sv:
        sv.start()
        ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.0003 * k,
                         flags=0 if k % 2 else rr.RR_HITS_ORIGINAL_ORDER) for k, s in enumerate(segs)]
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
    assert all(x["status"] == 0 and x["done"] for x in st)
    for k, s in enumerate(segs):
        hits, perm = expected(rr, scene, s)
        want = hits[perm] if k % 2 else hits
        assert rr.hits_to_numpy(s["hits"]).tobytes() == want.tobytes(), k


def test_server_destroy_releases_waiting_threads(rr, city):
    """rr_server_destroy while other threads block in rr_server_wait on
    requests that never start (the loop was not started): every waiter
    returns with a failure status before the server is freed."""
    import threading
    w, scene = city
    segs = make_segments(rr, w, scene, [1000, 2000, 3000], seed=52)
    sv = rr.Server(scene, slots=1, hbm_budget_bytes=8 << 30, max_batch_rays=10000)
    ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.0) for s in segs]
    out = {}

    def waiter(i):
        try:
            sv.wait(i, timeout_s=30.0)
            out[i] = "ok"
        except rr.RRError as e:
            out[i] = e.status

    th = [threading.Thread(target=waiter, args=(i,)) for i in ids]
    for t in th:
        t.start()
    import time
    time.sleep(0.2)
    sv.close()
    for t in th:
        t.join(10.0)
    assert all(not t.is_alive() for t in th)
    assert sorted(out) == sorted(ids) and all(v != "ok" for v in out.values())


def test_server_requests_larger_than_a_batch_as_parts(rr, city):
    """A request in ray order larger than the largest batch is served as
    parts of the split size (its hits equal the request traced alone); one
    in key order, which cannot be split, is refused; a split size larger
    than the largest batch is refused at create."""
    w, scene = city
    with pytest.raises(rr.RRError) as e:
        rr.Server(scene, slots=2, hbm_budget_bytes=8 << 30, max_batch_rays=20000, split_rays=30000)
    assert e.value.status == -1
    segs = make_segments(rr, w, scene, [50000, 50000, 7000], seed=71)
    with rr.Server(scene, slots=2, hbm_budget_bytes=8 << 30, max_batch_rays=20000, max_batch_requests=4,
                   split_rays=5000) as sv:
        sv.start()
        a = sv.submit(segs[0]["rays"], segs[0]["hits"], segs[0]["key"])
        with pytest.raises(rr.RRError) as e:
            sv.submit(segs[1]["rays"], segs[1]["hits"], segs[1]["key"], flags=0)
        assert e.value.status == -6
        c = sv.submit(segs[2]["rays"], segs[2]["hits"], segs[2]["key"], flags=0)
        sv.drain(60.0)
        assert sv.wait(a)["status"] == 0 and sv.wait(c)["status"] == 0
        assert sv.stats()["rejected"] == 1
    hits, _ = expected(rr, scene, segs[0])
    assert rr.hits_to_numpy(segs[0]["hits"]).tobytes() == hits.tobytes()
    hits, perm = expected(rr, scene, segs[2])
    assert rr.hits_to_numpy(segs[2]["hits"]).tobytes() == hits[perm].tobytes()


def test_server_splits_large_requests(rr, city):
    """With a split size, requests in ray order larger than it are served as
    parts (several batches, possibly on several slots at once); requests in
    key order are not split.  Every request's hits equal the request traced
    alone."""
    w, scene = city
    rng = np.random.default_rng(53)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(200), np.log(40000), 20))] + [39999, 12001, 5000, 5001]
    segs = make_segments(rr, w, scene, sizes, seed=53)
    with rr.Server(scene, slots=3, hbm_budget_bytes=8 << 30, max_batch_rays=60000, max_batch_requests=4,
                   split_rays=5000) as sv:
        sv.start()
        ids = [sv.submit(s["rays"], s["hits"], s["key"], arrival_s=0.0002 * k,
                         flags=0 if k % 5 == 4 else rr.RR_HITS_ORIGINAL_ORDER) for k, s in enumerate(segs)]
        sv.drain(120.0)
        st = [sv.wait(i) for i in ids]
        stats = sv.stats()
    assert all(x["status"] == 0 and x["done"] for x in st)
    assert stats["completed"] == len(segs) and stats["rays"] == sum(sizes)
    # parts of 5000 rays, at most 4 per batch: more batches than requests
    assert stats["batches"] >= sum(-(-n // 5000) if k % 5 != 4 else 1 for k, n in enumerate(sizes)) // 4
    for k, s in enumerate(segs):
        hits, perm = expected(rr, scene, s)
        want = hits[perm] if k % 5 == 4 else hits
        assert rr.hits_to_numpy(s["hits"]).tobytes() == want.tobytes(), k
    for x in st:
        assert x["finish_s"] >= x["start_s"] >= x["arrival_s"] - 1e-6
