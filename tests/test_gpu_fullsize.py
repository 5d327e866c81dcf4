"""GPU parity at the full sizes the bench times, in its launch configuration:
the 1920x1080 bounce-2 wavefront on the ~1M-triangle grid city (2,073,600
rays), the 3840x2160 bounce-3 wavefront on the same city (8,294,400 slots,
compacted before the sort), the 64-wavefront batch (17.4M rays) and the
served configuration on the ~4M-triangle city (requests of 16K to 4M rays).
Keys, permutations and every hit are checked against the oracle (hits with
the near-tie rule), and hits scattered back to ray order against the unsorted
trace bit for bit."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from hitcheck import assert_hits_match

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
    """The headline wavefront, its scene on the device and the oracle's BVH."""
    w = W.bounce2_1080p()
    scene = rr.Scene(w.tris)
    yield w, scene, O.BVH(w.tris)
    scene.close()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def keys_np(t, bits):
    a = t.cpu().numpy()
    return a.view(np.uint32) if bits == 32 else a.view(np.uint64)


@pytest.mark.parametrize("kind,bits", [(O.KIND_OT, 64), (O.KIND_OD, 64)])
def test_headline_keys_and_fused_call(rr, city, kind, bits):
    w, scene, bvh = city
    lo, hi = scene.bounds()
    n = w.rays.shape[0]
    rays = to_dev(w.rays)
    p = rr.key_params(kind, bits, lo, hi, 0.25)
    want_keys = O.keys(w.rays, kind, bits, lo, hi, 0.25)
    k, _, _ = rr.rr_compute_keys(rays, p)
    assert np.array_equal(keys_np(k, bits), want_keys)
    _, want_perm = O.sort_pairs(want_keys)
    # the bench's step: keys and histograms in one kernel, the gather in the
    # sort's last pass, hits in key order
    hits, perm, cnt = rr.rr_reorder_and_trace(scene, rays, p, flags=0)
    assert int(cnt.cpu().numpy()[0]) == n
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), want_perm)
    h = rr.hits_to_numpy(hits)
    # every hit, in key order, against the oracle's trace of the sorted rays
    sorted_rays = np.ascontiguousarray(w.rays[want_perm])
    assert_hits_match(h, bvh.trace(sorted_rays), sorted_rays, w.tris, f"headline kind {kind}")
    # hits scattered back equal the unsorted trace, every ray
    back, _, _ = rr.rr_reorder_and_trace(scene, rays, p, flags=rr.RR_HITS_ORIGINAL_ORDER)
    plain = rr.hits_to_numpy(rr.rr_trace(scene, rays))
    assert rr.hits_to_numpy(back).tobytes() == plain.tobytes()
    assert h.tobytes() == plain[want_perm].tobytes()


def test_large_launch_refill(rr, city):
    """A launch of more than 512 rays per resident wave (the headline rays
    three times over, 6.2M rays), where rr_trace takes its larger refill
    threshold: the same hits bit for bit as rr_trace_ex with refill 8, and
    each copy the same as the trace of the wavefront alone (whose hits the
    headline test checks against the oracle)."""
    w, scene, _ = city
    n = w.rays.shape[0]
    rays = to_dev(np.concatenate([w.rays] * 3))
    auto = rr.rr_trace(scene, rays)
    fixed = rr.rr_trace(scene, rays, refill=8)
    assert torch.equal(auto.view(torch.int32), fixed.view(torch.int32))
    one = rr.rr_trace(scene, rays[:n])
    for c in range(3):
        assert torch.equal(auto[c * n:(c + 1) * n].view(torch.int32), one.view(torch.int32)), c


def test_bounce3_compacted(rr, city):
    w, scene, bvh = city
    w3 = W.bounce3_2160p()
    assert np.array_equal(w3.tris, w.tris)  # the same city
    lo, hi = scene.bounds()
    live = O.compact(w3.alive)
    p = rr.key_params(O.KIND_OT, 64, lo, hi, 0.25)
    hits, perm, cnt = rr.rr_reorder_and_trace(scene, to_dev(w3.rays), p, alive=to_dev(w3.alive), flags=0)
    c = int(cnt.cpu().numpy()[0])
    assert c == len(live)
    k = O.keys(w3.rays[live], O.KIND_OT, 64, lo, hi, 0.25)
    order = np.lexsort((live, k))
    want_perm = live[order].astype(np.uint32)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32)[:c], want_perm)
    h = rr.hits_to_numpy(hits)[:c]
    sorted_rays = np.ascontiguousarray(w3.rays[want_perm])
    assert_hits_match(h, bvh.trace(sorted_rays), sorted_rays, w.tris, "bounce-3")


def test_batch_64_wavefronts(rr, city):
    """The bench's batch (its segments built by the bench's own code), in the
    default launch shape and in the autotuner's usual one."""
    w, scene, bvh = city
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    segs, keep, total, key = bench.batch_segments(torch, rr, W, scene, w, torch.device(DEV))
    assert len(segs) == 64 and total > 10_000_000
    lo, hi = scene.bounds()
    perms = [torch.empty(r.shape[0], dtype=torch.int32, device=DEV) for r, _ in keep]
    with_perm = [rr.segment(r, h, key, perm=q) for (r, h), q in zip(keep, perms)]
    rays_np = [r.cpu().numpy() for r, _ in keep]
    want = []
    want_hits = []
    for rn in rays_np:
        _, wp = O.sort_pairs(O.keys(rn, O.KIND_OT, 64, lo, hi, 0.25))
        want.append(wp)
        want_hits.append(bvh.trace(np.ascontiguousarray(rn[wp])))
    for shape in (None, bench.BATCH_PROFILE_SHAPE):
        with rr.Batch(scene, max_rays=total, max_segments=len(segs), config=shape) as b:
            b.run(with_perm, flags=0)
            torch.cuda.synchronize()
        for j, ((r, h), q) in enumerate(zip(keep, perms)):
            assert np.array_equal(q.cpu().numpy().view(np.uint32), want[j]), (shape, j)
            got = rr.hits_to_numpy(h)
            assert_hits_match(got, want_hits[j], rays_np[j][want[j]], w.tris, f"{shape} segment {j}")


def test_served_4m_city(rr):
    """The serving configuration of the bench (~4M-triangle city, requests
    of 16K to 4M rays with mixed key methods; three slots, batches of at most
    2M rays, requests above 512K rays served as parts; 32 GB budget): every
    served hit equals the unsorted trace of its request and the oracle's
    trace of the request."""
    c = W.city(5, 200, 200, 3_520_000)
    r = W.camera_rays(5, 3840, 2160, (100.0, 120.0, 100.0))
    r, alive = W.bounce(c, 5, 300, r, np.ones(r.shape[0], np.uint8))
    pool = np.ascontiguousarray(r[alive.astype(bool)])
    bvh = O.BVH(c.tris)
    sizes = [16384, 100_000, 500_000, 1_000_000, 2_000_000, 1 << 22]
    kinds = [(0, 32), (1, 32), (1, 64), (2, 64)]
    with rr.Scene(c.tris) as scene:
        lo, hi = scene.bounds()
        reqs = []
        for j, n in enumerate(sizes):
            ix = W.sample_indices(5, 7000 + j, n, pool.shape[0])
            rn = np.ascontiguousarray(pool[ix])
            kind, bits = kinds[j % len(kinds)]
            reqs.append((rn, to_dev(rn), torch.empty((n, 4), dtype=torch.float32, device=DEV),
                         rr.key_params(kind, bits, lo, hi, 0.25)))
        with rr.Server(scene, slots=3, hbm_budget_bytes=32 << 30, max_batch_rays=1 << 21,
                       max_batch_requests=16, split_rays=1 << 19) as sv:
            sv.start()
            ids = [sv.submit(rd, h, p, arrival_s=0.0005 * j) for j, (_, rd, h, p) in enumerate(reqs)]
            sv.drain(300.0)
            st = [sv.wait(i) for i in ids]
        assert all(x["status"] == 0 and x["done"] for x in st)
        torch.cuda.synchronize()
        for j, (rn, rd, h, _) in enumerate(reqs):
            got = rr.hits_to_numpy(h)
            assert got.tobytes() == rr.hits_to_numpy(rr.rr_trace(scene, rd)).tobytes(), j
            assert_hits_match(got, bvh.trace(rn), rn, c.tris, f"request {j}")
