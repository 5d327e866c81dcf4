"""GPU parity of the any-hit (occlusion) trace used for shadow rays: the
occluded flag equals the oracle's (a ray is occluded exactly when its closest
hit exists), and the record reported for an occluded ray is the oracle's
exact triangle test of that triangle (which triangle is reported depends on
the traversal and is not unique)."""
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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check_any(h, ref, rays, tris, what):
    occluded = ref["prim"] >= 0
    assert np.array_equal(h["prim"] >= 0, occluded), what
    miss = ~occluded
    assert np.all(np.isinf(h["t"][miss])) and np.all(h["u"][miss] == 0) and np.all(h["v"][miss] == 0), what
    for i in np.nonzero(occluded)[0]:
        ok, t, u, v = O.mt(rays[i], tris[int(h["prim"][i])])
        assert ok and rays[i, 3] < t < rays[i, 7], (what, i)
        assert np.float32(t) == h["t"][i] and np.float32(u) == h["u"][i] and np.float32(v) == h["v"][i], (what, i)


def test_any_hit_soup(rr, soup65k):
    w = soup65k
    rays = w.rays.copy()
    rng = np.random.default_rng(3)
    rays[:, 7] = rng.uniform(0.05, 1.0, rays.shape[0]).astype(np.float32)   # finite shadow-ray lengths
    ref = O.brute_force(w.tris, rays)
    assert 0.05 < np.mean(ref["prim"] >= 0) < 0.95
    with rr.Scene(w.tris) as sc:
        h = rr.hits_to_numpy(rr.rr_trace_any(sc, to_dev(rays)))
        check_any(h, ref, rays, w.tris, "soup")


def test_any_hit_city_shadow_rays(rr):
    w = W.city_small(seed=8, width=160, height=90, depth=1)
    c = w.city
    s = W.shadow_rays(8, 400, w.rays, (c.nx / 2.0, 30.0, c.nz / 2.0), 0.05 * c.extent)
    bvh = O.BVH(w.tris)
    ref = bvh.trace(s)
    assert 0.01 < np.mean(ref["prim"] >= 0) < 0.99
    lo, hi = O.scene_box(w.tris)
    with rr.Scene(w.tris) as sc:
        rays = to_dev(s)
        check_any(rr.hits_to_numpy(rr.rr_trace_any(sc, rays)), ref, s, w.tris, "city")
        # reordered shadow rays through the fused call
        for kind, bits, flags in ((O.KIND_OCTAHEDRON, 32, rr.RR_ANY_HIT),
                                  (O.KIND_OD, 32, rr.RR_ANY_HIT | rr.RR_HITS_ORIGINAL_ORDER),
                                  (O.KIND_OT, 64, rr.RR_ANY_HIT | rr.RR_INDIRECT)):
            p = rr.key_params(kind, bits, lo, hi)
            hits, perm, _ = rr.rr_reorder_and_trace(sc, rays, p, flags=flags)
            _, want = O.sort_pairs(O.keys(s, kind, bits, lo, hi))
            assert np.array_equal(perm.cpu().numpy().view(np.uint32), want)
            h = rr.hits_to_numpy(hits)
            if flags & rr.RR_HITS_ORIGINAL_ORDER:
                check_any(h, ref, s, w.tris, f"fused {kind}")
            else:
                check_any(h, ref[want], s[want], w.tris, f"fused {kind}")
        table = rr.LengthTable(rr.key_params(8, 32, lo, hi))
        with pytest.raises(rr.RRError):
            rr.rr_reorder_and_trace(sc, rays, rr.key_params(8, 32, lo, hi, aux=table), flags=rr.RR_ANY_HIT)
