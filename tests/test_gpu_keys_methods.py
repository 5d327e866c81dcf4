"""GPU parity of the figure's other key layouts (Origin, Costa, Aila, Aila
Compact, Octahedron) and of Two Point with the adaptive and the real
termination estimate (Section 3.1.6), against the CPU oracle: keys bit for
bit, the length table byte for byte, permutations exactly."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"
LAYOUTS = [O.KIND_ORIGIN, O.KIND_COSTA, O.KIND_AILA, O.KIND_AILA_COMPACT, O.KIND_OCTAHEDRON]


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2506_11273_amd as m
    m.load()
    return m


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def keys_np(t, bits):
    a = t.cpu().numpy()
    return a.view(np.uint32) if bits == 32 else a.view(np.uint64)


def edge_rays(n, seed):
    rng = np.random.default_rng(seed)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = rng.uniform(-0.5, 1.5, (n, 3))
    d = rng.normal(size=(n, 3))
    r[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r[:, 7] = np.where(rng.uniform(size=n) < 0.3, rng.uniform(0, 0.3, n), np.inf)
    axes = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, 0, 0], [0.6, 0, -0.8]]
    m = min(n, len(axes))
    r[:m, 4:7] = axes[:m]
    if n > 10:
        r[8, 0:3] = [1, 1, 1]
        r[9, 0] = np.nan
        r[10, 4] = np.nan
    return r


@pytest.mark.parametrize("kind", LAYOUTS)
def test_layout_keys_bit_exact(rr, soup65k, kind):
    w = soup65k
    lo, hi = O.scene_box(w.tris)
    p = rr.key_params(kind, 32, lo, hi)
    k, idx, _ = rr.rr_compute_keys(to_dev(w.rays), p)
    assert np.array_equal(keys_np(k, 32), O.keys(w.rays, kind, 32, lo, hi))
    for n in (1, 11, 257, 1000):
        r = edge_rays(n, n)
        p = rr.key_params(kind, 32, (0, 0, 0), (1, 1, 1))
        k, _, _ = rr.rr_compute_keys(to_dev(r), p)
        assert np.array_equal(keys_np(k, 32), O.keys(r, kind, 32, (0, 0, 0), (1, 1, 1))), (kind, n)


def test_layout_golden_values(rr):
    import test_oracle_layouts as T
    for name, kind, o, d, expected in T.golden():
        if kind == "CELL":
            continue
        r = np.array([[*o, 0, *d, np.inf]], np.float32)
        p = rr.key_params(T.KINDS[kind], 32, (0, 0, 0), (1, 1, 1))
        k, _, _ = rr.rr_compute_keys(to_dev(r), p)
        assert int(keys_np(k, 32)[0]) == expected, name


def test_layouts_with_compaction(rr):
    w = W.city_small(seed=3, width=128, height=72, depth=2)
    lo, hi = O.scene_box(w.tris)
    live = O.compact(w.alive)
    for kind in LAYOUTS:
        p = rr.key_params(kind, 32, lo, hi)
        k, idx, cnt = rr.rr_compute_keys(to_dev(w.rays), p, alive=to_dev(w.alive))
        c = int(cnt.cpu().numpy()[0])
        assert c == len(live)
        assert np.array_equal(keys_np(k, 32)[:c], O.keys(w.rays[live], kind, 32, lo, hi))


def test_layouts_refuse_64_bits_and_missing_tables(rr):
    r = to_dev(edge_rays(16, 1))
    for kind in LAYOUTS:
        with pytest.raises(rr.RRError) as e:
            rr.rr_compute_keys(r, rr.key_params(kind, 64, (0, 0, 0), (1, 1, 1)))
        assert e.value.status == -4
    for kind in (rr.RR_KEY_TWO_POINT_ADAPTIVE, rr.RR_KEY_TWO_POINT_REAL):
        with pytest.raises(rr.RRError) as e:
            rr.rr_compute_keys(r, rr.key_params(kind, 32, (0, 0, 0), (1, 1, 1)))
        assert e.value.status == -1
        host = torch.zeros((16, 4))
        with pytest.raises(rr.RRError) as e:
            rr.rr_compute_keys(r, rr.key_params(kind, 32, (0, 0, 0), (1, 1, 1), aux=host))
        assert e.value.status == -1


@pytest.mark.parametrize("bits", [32, 64])
def test_two_point_real(rr, soup65k, bits):
    w = soup65k
    lo, hi = O.scene_box(w.tris)
    with rr.Scene(w.tris) as sc:
        rays = to_dev(w.rays)
        hits = rr.rr_trace(sc, rays)
        p = rr.key_params(rr.RR_KEY_TWO_POINT_REAL, bits, lo, hi, aux=hits)
        k, _, _ = rr.rr_compute_keys(rays, p)
        ref = O.keys(w.rays, O.KIND_TP_REAL, bits, lo, hi, aux=rr.hits_to_numpy(hits))
        assert np.array_equal(keys_np(k, bits), ref)
        h = rr.hits_to_numpy(hits)
        assert 0 < np.mean(h["prim"] >= 0) < 1   # both the hit and the miss branch are exercised


def test_length_table_init_accumulate_and_keys(rr):
    w = W.city_small(seed=9, width=160, height=90, depth=2)
    lo, hi = O.scene_box(w.tris)
    live = O.compact(w.alive)
    rays_np = np.ascontiguousarray(w.rays[live])
    with rr.Scene(w.tris) as sc:
        rays = to_dev(rays_np)
        p = rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, 32, lo, hi, 0.25)
        table = rr.LengthTable(p)
        p.aux = table.cells.data_ptr()
        p._aux_ref = table.cells
        ref = O.LengthTable(lo, hi, 0.25)
        assert table.numpy().tobytes() == ref.cells.tobytes()
        # a fresh table gives the fixed estimate
        for bits in (32, 64):
            pb = rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, bits, lo, hi, 0.25, aux=table)
            k, _, _ = rr.rr_compute_keys(rays, pb)
            assert np.array_equal(keys_np(k, bits), O.keys(rays_np, O.KIND_OT, bits, lo, hi))
        # accumulate traced lengths twice (the second time through a permutation)
        hits = rr.rr_trace(sc, rays)
        hn = rr.hits_to_numpy(hits)
        table.accumulate(rays, hits)
        ref.accumulate(rays_np, hn)
        perm = np.random.default_rng(1).permutation(len(rays_np)).astype(np.int32)
        table.accumulate(rays, hits[to_dev(perm).long()], idx=to_dev(perm))
        ref.accumulate(rays_np[perm], hn[perm])
        torch.cuda.synchronize()
        assert table.numpy().tobytes() == ref.cells.tobytes()
        assert np.max(ref.cells["count"]) > 2
        for bits in (32, 64):
            pb = rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, bits, lo, hi, 0.25, aux=table)
            k, _, _ = rr.rr_compute_keys(rays, pb)
            got = keys_np(k, bits)
            want = O.keys(rays_np, O.KIND_TP_ADAPTIVE, bits, lo, hi, aux=ref)
            assert np.array_equal(got, want)
            assert not np.array_equal(got, O.keys(rays_np, O.KIND_OT, bits, lo, hi))


def test_fused_adaptive_updates_the_table(rr):
    w = W.city_small(seed=10, width=128, height=72, depth=2)
    lo, hi = O.scene_box(w.tris)
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        rays, alive = to_dev(w.rays), to_dev(w.alive)
        p = rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, 32, lo, hi, 0.25)
        table = rr.LengthTable(p)
        p = rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, 32, lo, hi, 0.25, aux=table)
        ref = O.LengthTable(lo, hi, 0.25)
        live = O.compact(w.alive)
        for it, flags in enumerate((0, rr.RR_HITS_ORIGINAL_ORDER, rr.RR_INDIRECT)):
            k = O.keys(w.rays[live], O.KIND_TP_ADAPTIVE, 32, lo, hi, aux=ref)
            order = np.lexsort((live, k))
            want_perm = live[order]
            want_hits = bvh.trace(w.rays[want_perm])
            hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, alive=alive, flags=flags)
            c = int(cnt.cpu().numpy()[0])
            assert c == len(live)
            assert np.array_equal(perm.cpu().numpy().view(np.uint32)[:c], want_perm), it
            h = rr.hits_to_numpy(hits)
            hs = h[want_perm] if flags & rr.RR_HITS_ORIGINAL_ORDER else h[:c]
            assert hs.tobytes() == want_hits.tobytes(), it
            ref.accumulate(w.rays[want_perm], want_hits)
            torch.cuda.synchronize()
            assert table.numpy().tobytes() == ref.cells.tobytes(), it


def test_fused_dense_every_key_method(rr):
    """Without compaction the fused call computes the keys and counts the
    sort's digit histograms in one kernel: every key method and width gives
    the oracle's permutation, and the hits scattered back equal the unsorted
    trace bit for bit."""
    w = W.city_small(seed=17, width=160, height=90, depth=1)
    lo, hi = O.scene_box(w.tris)
    n = w.rays.shape[0]
    with rr.Scene(w.tris) as sc:
        rays = to_dev(w.rays)
        base = rr.rr_trace(sc, rays)
        base_np = rr.hits_to_numpy(base)
        assert 0 < np.mean(base_np["prim"] >= 0) < 1
        cases = [(k, 32) for k in LAYOUTS] + [(rr.RR_KEY_TWO_POINT_ADAPTIVE, b) for b in (32, 64)] + \
                [(rr.RR_KEY_TWO_POINT_REAL, b) for b in (32, 64)]
        for kind, bits in cases:
            aux = oaux = None
            if kind == rr.RR_KEY_TWO_POINT_ADAPTIVE:
                # a table with traced lengths in it, mirrored by the oracle's
                aux = rr.LengthTable(rr.key_params(kind, bits, lo, hi, 0.25))
                oaux = O.LengthTable(lo, hi, 0.25)
                aux.accumulate(rays, base)
                oaux.accumulate(w.rays, base_np)
                torch.cuda.synchronize()
                assert aux.numpy().tobytes() == oaux.cells.tobytes()
            elif kind == rr.RR_KEY_TWO_POINT_REAL:
                aux, oaux = base, base_np
            p = rr.key_params(kind, bits, lo, hi, 0.25, aux=aux)
            want = O.keys(w.rays, kind, bits, lo, hi, aux=oaux)
            _, want_perm = O.sort_pairs(want)
            hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, flags=rr.RR_HITS_ORIGINAL_ORDER)
            assert int(cnt.cpu().numpy()[0]) == n
            assert np.array_equal(perm.cpu().numpy().view(np.uint32), want_perm), (kind, bits)
            assert rr.hits_to_numpy(hits).tobytes() == base_np.tobytes(), (kind, bits)


def test_fused_dense_past_2_24_rays(rr):
    """From 2^24 keys on the sort takes 16 keys per thread; the fused call's
    keys-and-histogram kernel feeds that schedule too.  Permutation against
    the oracle's keys and stable order; hits on a sample against the
    oracle's trace, all hits scattered back against the unsorted trace."""
    w = W.city_small(seed=23, width=64, height=36, depth=1, n=8, n_clutter=2000)
    lo, hi = O.scene_box(w.tris)
    n = (1 << 24) + 4097
    rng = np.random.default_rng(24)
    r = np.empty((n, 8), np.float32)
    r[:, 0:3] = rng.uniform(lo, hi, (n, 3))
    d = rng.normal(size=(n, 3))
    r[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r[:, 3] = 0.0
    r[:, 7] = np.inf
    for bits in (64, 32):
        kind = O.KIND_OT if bits == 64 else O.KIND_OD
        want = O.keys(r, kind, bits, lo, hi)
        want_perm = np.lexsort((np.arange(n, dtype=np.uint32), want)).astype(np.uint32)
        with rr.Scene(w.tris) as sc:
            rays = to_dev(r)
            p = rr.key_params(kind, bits, lo, hi)
            hits, perm, _ = rr.rr_reorder_and_trace(sc, rays, p, flags=0)
            got_perm = perm.cpu().numpy().view(np.uint32)
            assert np.array_equal(got_perm, want_perm), bits
            back = rr.rr_scatter_hits(hits, perm)
            assert torch.equal(back.view(torch.int32), rr.rr_trace(sc, rays).view(torch.int32)), bits
            h = rr.hits_to_numpy(hits)
            sample = rng.choice(n, 4096, replace=False)
            ref = O.BVH(w.tris).trace(r[want_perm[sample]])
            assert h[sample].tobytes() == ref.tobytes(), bits
            del rays, hits, perm, back
            torch.cuda.empty_cache()


def test_batch_mixes_key_methods(rr):
    w = W.city_small(seed=21, width=200, height=120, depth=1, n=16, n_clutter=20000)
    lo, hi = O.scene_box(w.tris)
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
        rng = np.random.default_rng(3)
        table = rr.LengthTable(rr.key_params(rr.RR_KEY_TWO_POINT_ADAPTIVE, 32, lo, hi))
        kinds = [(k, 32) for k in LAYOUTS] + [(rr.RR_KEY_TWO_POINT_ADAPTIVE, 64), (rr.RR_KEY_TWO_POINT_REAL, 32),
                                              (rr.RR_KEY_ORIGIN_TERMINATION, 64)]
        segs, keep = [], []
        for j, (kind, bits) in enumerate(kinds):
            n = int(rng.integers(100, 20000))
            rn = np.ascontiguousarray(w.rays[rng.integers(0, len(w.rays), n)])
            rays = to_dev(rn)
            aux = table if kind == rr.RR_KEY_TWO_POINT_ADAPTIVE else (
                rr.rr_trace(sc, rays) if kind == rr.RR_KEY_TWO_POINT_REAL else None)
            key = rr.key_params(kind, bits, lo, hi, aux=aux)
            hits = torch.empty((n, 4), dtype=torch.float32, device=DEV)
            perm = torch.empty(n, dtype=torch.int32, device=DEV)
            keep.append((rn, rays, hits, perm, kind, bits, aux, key))
            segs.append(rr.segment(rays, hits, key, perm=perm))
        with rr.Batch(sc, max_rays=sum(x[0].shape[0] for x in keep), max_segments=len(keep)) as b:
            b.run(segs)
            torch.cuda.synchronize()
        otab = O.LengthTable(lo, hi)
        for rn, rays, hits, perm, kind, bits, aux, key in keep:
            oa = otab if kind == rr.RR_KEY_TWO_POINT_ADAPTIVE else (
                rr.hits_to_numpy(aux) if kind == rr.RR_KEY_TWO_POINT_REAL else None)
            k = O.keys(rn, kind, bits, lo, hi, aux=oa)
            _, want = O.sort_pairs(k)
            assert np.array_equal(perm.cpu().numpy().view(np.uint32), want), kind
            alone = rr.hits_to_numpy(rr.rr_trace(sc, rays))
            assert rr.hits_to_numpy(hits).tobytes() == alone.tobytes(), kind


# ------------------------------------------------------- coherence measure

def test_coherence_m64_matches_oracle(rr):
    w = W.city_small(seed=12, width=160, height=90, depth=2)
    lo, hi = O.scene_box(w.tris)
    live = O.compact(w.alive)
    with rr.Scene(w.tris) as sc:
        p = rr.key_params(rr.RR_KEY_NONE, 32, lo, hi)
        for n in (1, 63, 64, 65, 1000, len(live)):
            rn = np.ascontiguousarray(w.rays[live[:n]])
            rays = to_dev(rn)
            hits = rr.rr_trace(sc, rays)
            g, m = rr.coherence_m64(rays, hits, p)
            gr, mr = O.coherence_m64(rn, rr.hits_to_numpy(hits), lo, hi)
            gg = g.cpu().numpy()
            assert len(gg) == len(gr)
            np.testing.assert_allclose(gg, gr, rtol=1e-9, atol=1e-12)
            assert abs(float(m.cpu()[0]) - mr) <= 1e-9 * abs(mr) + 1e-12
        # the measure is deterministic run to run
        g2, m2 = rr.coherence_m64(rays, hits, p)
        assert torch.equal(g, g2) and torch.equal(m, m2)
        e, me = rr.coherence_m64(rays[:0], hits[:0], p)
        assert float(me.cpu()[0]) == 0.0
