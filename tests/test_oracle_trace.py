"""Pins for the oracle's sort, gather, compaction and closest-hit trace.

* sort: against Python's sorted() on (key, index) tuples and the stability
  properties of Section 3.2's key/index sort;
* gather/scatter: the identity gather-then-scatter;
* Moller-Trumbore: closed-form hand cases and a float64 linear solve;
* BVH trace: brute force over every triangle, bit for bit;
* the workload generator's analytic city hit distance against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W


# ------------------------------------------------------------------ sort

def test_sort_matches_tuple_sort():
    rng = np.random.default_rng(0)
    for n, hi in ((1, 4), (7, 3), (300, 16), (1000, 1 << 32)):
        k = rng.integers(0, hi, n, dtype=np.uint64).astype(np.uint32)
        idx = rng.permutation(n).astype(np.uint32)
        ks, ix = O.sort_pairs(k, idx)
        ref = sorted(zip(k.tolist(), idx.tolist()))
        assert ks.tolist() == [a for a, _ in ref]
        assert ix.tolist() == [b for _, b in ref]


def test_sort_properties_u64():
    rng = np.random.default_rng(1)
    n = 50000
    k = rng.integers(0, 1 << 12, n, dtype=np.uint64) << np.uint64(50)  # many equal keys
    ks, ix = O.sort_pairs(k)
    assert np.all(ks[1:] >= ks[:-1])
    assert np.array_equal(np.sort(ix), np.arange(n, dtype=np.uint32))
    eq = ks[1:] == ks[:-1]
    assert np.all(ix[1:][eq] > ix[:-1][eq])  # stable: ties keep index order
    assert np.array_equal(k[ix], ks)


def test_gather_scatter_identity():
    rng = np.random.default_rng(2)
    rays = rng.normal(size=(1000, 8)).astype(np.float32)
    idx = rng.permutation(1000).astype(np.uint32)
    g = O.gather(rays, idx)
    assert np.array_equal(g[5], rays[idx[5]])
    assert np.array_equal(O.scatter(g, idx), rays)


def test_compact():
    a = np.array([0, 1, 1, 0, 0, 1, 0, 1], np.uint8)
    assert O.compact(a).tolist() == [1, 2, 5, 7]
    assert O.compact(np.zeros(5, np.uint8)).size == 0
    assert O.compact(np.ones(3, np.uint8)).tolist() == [0, 1, 2]


# ---------------------------------------------------------- triangle test

def ray(o, d, tmin=0.0, tmax=np.inf):
    return np.array([*o, tmin, *d, tmax], np.float32)


def test_mt_closed_form():
    tri = np.array([0, 0, 0.5, 1, 0, 0.5, 0, 1, 0.5], np.float32)
    hit, t, u, v = O.mt(ray((0.25, 0.25, 0), (0, 0, 1)), tri)
    assert hit and t == 0.5 and u == 0.25 and v == 0.25
    # barycentrics follow the edges v1 - v0 (u) and v2 - v0 (v)
    hit, t, u, v = O.mt(ray((0.5, 0.125, 2), (0, 0, -1)), tri)
    assert hit and t == 1.5 and u == 0.5 and v == 0.125
    # outside: u + v > 1, and a ray parallel to the plane
    assert not O.mt(ray((0.75, 0.5, 0), (0, 0, 1)), tri)[0]
    assert not O.mt(ray((0.2, 0.2, 0.5), (1, 0, 0)), tri)[0]
    # two-sided: the same triangle wound the other way
    tri2 = tri.reshape(3, 3)[[0, 2, 1]].ravel()
    hit, t, u, v = O.mt(ray((0.25, 0.125, 0), (0, 0, 1)), tri2)
    assert hit and t == 0.5 and u == 0.125 and v == 0.25


def test_mt_against_float64_solve():
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(3000):
        v = rng.uniform(-1, 1, (3, 3))
        o = rng.uniform(-2, 2, 3)
        target = v[0] + rng.uniform(-0.2, 1.2) * (v[1] - v[0]) + rng.uniform(-0.2, 1.2) * (v[2] - v[0])
        d = target - o
        d /= np.linalg.norm(d)
        r = ray(o, d)
        tri = v.astype(np.float32).ravel()
        # float64 solve of o + t d = v0 + u e1 + v e2 on the rounded inputs
        rf = r.astype(np.float64)
        tf = tri.astype(np.float64).reshape(3, 3)
        e1, e2 = tf[1] - tf[0], tf[2] - tf[0]
        A = np.stack([-rf[4:7], e1, e2], axis=1)
        if abs(np.linalg.det(A)) < 1e-3:
            continue
        t, uu, vv = np.linalg.solve(A, rf[0:3] - tf[0])
        hit, t32, u32, v32 = O.mt(r, tri)
        margin = min(uu, vv, 1 - uu - vv)
        if abs(margin) < 1e-4:
            continue  # too close to an edge to demand the same decision
        assert hit == (margin > 0), (uu, vv)
        if hit:
            assert abs(t32 - t) <= 1e-4 * max(1.0, abs(t))
            assert abs(u32 - uu) <= 1e-4 and abs(v32 - vv) <= 1e-4
            checked += 1
    assert checked > 500


def test_tie_goes_to_lower_primitive():
    # two coplanar triangles sharing the edge x + y = 1 in the plane z = 0.5;
    # a ray through the shared edge hits both at t = 0.5 exactly
    a = [1, 0, 0.5, 0, 1, 0.5, 1, 1, 0.5]
    b = [0, 0, 0.5, 1, 0, 0.5, 0, 1, 0.5]
    r = ray((0.5, 0.5, 0), (0, 0, 1))[None]
    for tris in ([a, b], [b, a]):
        T = np.array(tris, np.float32)
        assert O.mt(r[0], T[0])[0] and O.mt(r[0], T[1])[0]
        h = O.brute_force(T, r)[0]
        assert h["t"] == 0.5 and h["prim"] == 0
        assert O.BVH(T).trace(r)[0]["prim"] == 0


def test_ray_interval_is_open():
    tri = np.array([[0, 0, 0.5, 1, 0, 0.5, 0, 1, 0.5]], np.float32)
    assert O.brute_force(tri, ray((0.2, 0.2, 0), (0, 0, 1), tmax=0.5)[None])[0]["prim"] == -1
    assert O.brute_force(tri, ray((0.2, 0.2, 0), (0, 0, 1), tmin=0.5)[None])[0]["prim"] == -1
    assert O.brute_force(tri, ray((0.2, 0.2, 0), (0, 0, 1), tmax=0.50001)[None])[0]["prim"] == 0
    h = O.brute_force(tri, ray((0.2, 0.2, 0), (0, 0, -1))[None])[0]
    assert h["prim"] == -1 and np.isinf(h["t"]) and h["u"] == 0 and h["v"] == 0


# ------------------------------------------------------------ BVH trace

def test_bvh_equals_brute_force_soup(soup65k):
    w = soup65k
    bf = O.brute_force(w.tris, w.rays)
    bvh = O.BVH(w.tris)
    h = bvh.trace(w.rays)
    assert h.tobytes() == bf.tobytes()
    assert 0.2 < np.mean(bf["prim"] >= 0) < 0.4


def test_bvh_equals_brute_force_small_city():
    # axis-aligned boxes and a ground quad: flat boxes, axis-parallel rays
    w = W.city_small(seed=11, width=96, height=64, depth=1)
    rays = w.rays
    extra = np.array([[3.5, 2.0, 3.5, 0, 0, -1, 0, np.inf],   # straight down
                      [0.5, 0.05, 5.0, 0, 1, 0, 0, np.inf],   # along +x at ground level
                      [6.0, 0.5, 6.0, 0, 0, 0, 1, np.inf]], np.float32)
    extra = extra[:, [0, 1, 2, 3, 4, 5, 6, 7]]
    extra[:, 4:7] = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    rays = np.concatenate([rays, extra])
    bf = O.brute_force(w.tris, rays)
    h = O.BVH(w.tris).trace(rays)
    assert h.tobytes() == bf.tobytes()
    assert np.mean(bf["prim"] >= 0) > 0.5


@pytest.mark.parametrize("scale", [1.0, 2.0 ** -40, 2.0 ** 40])
def test_bvh_equals_brute_force_degenerate(scale):
    """Zero-area and duplicate triangles, rays in the plane of axis-aligned
    triangles, axis-aligned and negative-zero directions, empty and inverted
    intervals: the BVH finds brute force's hits, bit for bit, at three
    scales.  Scaling up by a power of two changes no hit's primitive; at
    2^-40 products of the near-degenerate edges fall into the subnormal
    range, lose precision, and a few hits may change."""
    T, rays = W.degenerate(12, 3000, 8192, scale)
    bf = O.brute_force(T, rays)
    assert O.BVH(T).trace(rays).tobytes() == bf.tobytes()
    assert (bf["prim"] >= 0).sum() > 1000
    if scale >= 1.0:
        T1, rays1 = W.degenerate(12, 3000, 8192, 1.0)
        assert np.array_equal(bf["prim"], O.brute_force(T1, rays1)["prim"])


def test_bvh_indirect_equals_gather():
    w = W.soup(seed=4, n_rays=4000, n_tris=500)
    bvh = O.BVH(w.tris)
    idx = np.random.default_rng(4).permutation(4000).astype(np.uint32)
    assert bvh.trace(w.rays, idx=idx).tobytes() == bvh.trace(O.gather(w.rays, idx)).tobytes()


def test_bvh_is_balanced():
    # median split: depth = ceil(log2(ceil(n / 4)))
    for n in (1, 4, 5, 100, 4096):
        tris = W.random_tris(9, n)
        b = O.BVH(tris)
        leaves = -(-n // 4)
        assert b.depth == int(np.ceil(np.log2(leaves))) if leaves > 1 else b.depth == 0


def test_generator_hits_agree_with_oracle():
    # the generator's analytic box/ground intersection and the oracle's
    # triangle trace must see the same first surface in a clutter-free city
    c = W.city(5, 10, 10, 0)
    rays = W.camera_rays(5, 64, 36, (5.0, 6.0, 5.0))
    b1, _ = W.bounce(c, 5, 100, rays)
    for rr in (rays, b1):
        ta = W.city_hit_t(c, rr)
        h = O.BVH(c.tris).trace(rr)
        hit_a = np.isfinite(ta)
        assert np.array_equal(hit_a, h["prim"] >= 0)
        assert np.allclose(h["t"][hit_a], ta[hit_a], rtol=1e-5, atol=1e-5)


def test_pipeline_scatter_back_matches_unsorted(soup65k):
    w = soup65k
    bvh = O.BVH(w.tris)
    lo, hi = O.scene_box(w.tris)
    base = bvh.trace(w.rays)
    for kind, bits in ((O.KIND_OD, 32), (O.KIND_OT, 64)):
        res = O.reorder_and_trace(bvh, w.rays, kind, bits, lo, hi)
        assert O.scatter(res["hits"], res["idx"]).tobytes() == base.tobytes()
