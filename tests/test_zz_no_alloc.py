"""rr_reorder_and_trace_noalloc (the fused call with its workspace in the
library's static device array, for callers that cannot allocate) against
rr_reorder_and_trace with a caller workspace, through the C ABI: two calls
in a row, the second with a smaller input, other key method, compaction and
hit order (so the second call runs on what the first left in the array),
then a third with the most-significant-digit sort forced;
keys, permutation, count and hits must be identical.  A call whose workspace
exceeds the array is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

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


def call_noalloc(rr, scene, rays, p, flags, alive=None):
    L = rr.load()
    n = rays.shape[0]
    hits = torch.full((n, 4), -7.0, dtype=torch.float32, device=DEV)
    perm = torch.full((n,), -7, dtype=torch.int32, device=DEV)
    count = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    st = L.rr_reorder_and_trace_noalloc(scene.handle, ctypes.c_void_p(rays.data_ptr()), n,
                                        ctypes.c_void_p(alive.data_ptr() if alive is not None else None),
                                        ctypes.byref(p), ctypes.c_void_p(hits.data_ptr()),
                                        ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(count.data_ptr()),
                                        flags, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, hits, perm, count


def call_with_workspace(rr, scene, rays, p, flags, alive=None):
    n = rays.shape[0]
    hits = torch.full((n, 4), -7.0, dtype=torch.float32, device=DEV)
    perm = torch.full((n,), -7, dtype=torch.int32, device=DEV)
    count = torch.full((1,), -7, dtype=torch.int32, device=DEV)
    rr.rr_reorder_and_trace(scene, rays, p, alive=alive, flags=flags, hits=hits, perm=perm, count=count)
    return hits, perm, count


def same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_noalloc_equals_the_fused_call(rr):
    w = W.bounce2_1080p()
    with rr.Scene(w.tris) as scene:
        lo, hi = scene.bounds()
        rays = torch.from_numpy(w.rays).to(DEV)
        # first call: the whole 1080p wavefront, Two Point 64-bit, hits in key order
        p1 = rr.key_params(2, 64, lo, hi, 0.25)
        st, h1, q1, c1 = call_noalloc(rr, scene, rays, p1, 0)
        assert st == 0, rr.load().rr_status_string(st)
        e1, f1, d1 = call_with_workspace(rr, scene, rays, p1, 0)
        torch.cuda.synchronize()
        assert same(q1, f1) and same(c1, d1) and same(h1, e1)
        # second call: fewer rays, origin-direction 32-bit, compacted, hits
        # scattered back to ray order
        m = 300007
        r2 = rays[:m].contiguous()
        alive = torch.from_numpy((np.random.default_rng(3).random(m) < 0.6).astype(np.uint8)).to(DEV)
        p2 = rr.key_params(1, 32, lo, hi, 0.25)
        st, h2, q2, c2 = call_noalloc(rr, scene, r2, p2, rr.RR_HITS_ORIGINAL_ORDER, alive)
        assert st == 0, rr.load().rr_status_string(st)
        e2, f2, d2 = call_with_workspace(rr, scene, r2, p2, rr.RR_HITS_ORIGINAL_ORDER, alive)
        torch.cuda.synchronize()
        live = int(d2.cpu()[0])
        assert int(c2.cpu()[0]) == live == int(alive.sum().cpu())
        assert same(q2[:live], f2[:live]) and same(h2, e2)
        # third call: the most-significant-digit sort forced (its bucket
        # kernel and plan live in the array too)
        m3 = 500009
        r3 = rays[-m3:].contiguous()
        st, h4, q4, c4 = call_noalloc(rr, scene, r3, p1, rr.RR_SORT_MSD)
        assert st == 0, rr.load().rr_status_string(st)
        e4, f4, d4 = call_with_workspace(rr, scene, r3, p1, rr.RR_SORT_MSD)
        torch.cuda.synchronize()
        assert same(q4, f4) and same(c4, d4) and same(h4, e4)
        # more rays than the array holds: refused, outputs untouched
        big = torch.zeros((3_000_000, 8), dtype=torch.float32, device=DEV)
        st, h3, q3, c3 = call_noalloc(rr, scene, big, p1, 0)
        torch.cuda.synchronize()
        assert st == -5  # RR_ERR_WORKSPACE_TOO_SMALL
        assert bool((q3 == -7).all()) and bool((c3 == -7).all())
