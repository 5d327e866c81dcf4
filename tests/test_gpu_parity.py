"""GPU parity: every step of the HIP path against the CPU oracle.

Keys and sort permutations must match bit for bit; hits must match exactly
(the triangle test is evaluated in the same binary32 operation order on both
sides), with the near-tie rule as the only allowed difference: a differing
primitive is accepted only if the oracle's own test of the GPU's primitive
passes with t within 1e-5 relative of the oracle's t.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from hitcheck import assert_hits_match

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    import paper_2506_11273_amd as m
    m.load()
    return m


DEV = "cuda"
KINDS = [(O.KIND_OD, 32), (O.KIND_OD, 64), (O.KIND_OT, 32), (O.KIND_OT, 64)]


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def keys_np(t, bits):
    a = t.cpu().numpy()
    return a.view(np.uint32) if bits == 32 else a.view(np.uint64)


def idx_np(t):
    return t.cpu().numpy().view(np.uint32)


# ------------------------------------------------------------------- keys

@pytest.mark.parametrize("kind,bits", KINDS)
def test_keys_bit_exact_soup(rr, soup65k, kind, bits):
    w = soup65k
    lo, hi = O.scene_box(w.tris)
    p = rr.key_params(kind, bits, lo, hi, 0.25)
    k, idx, _ = rr.rr_compute_keys(to_dev(w.rays), p)
    torch.cuda.synchronize()
    ref = O.keys(w.rays, kind, bits, lo, hi, 0.25)
    assert np.array_equal(keys_np(k, bits), ref)
    assert np.array_equal(idx_np(idx), np.arange(len(ref), dtype=np.uint32))


@pytest.mark.parametrize("n", [1, 63, 255, 257, 1000])
def test_keys_ragged_sizes_and_edge_values(rr, n):
    rng = np.random.default_rng(n)
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = rng.uniform(-0.5, 1.5, (n, 3))     # includes out-of-box origins
    d = rng.normal(size=(n, 3))
    rays[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    rays[:, 7] = np.where(rng.uniform(size=n) < 0.3, rng.uniform(0, 0.3, n), np.inf)
    rays[0, 0:3] = [1.0, 1.0, 1.0]                     # on the upper face
    rays[0, 4:7] = [0.0, 0.0, -1.0]
    if n > 3:
        rays[1, 0] = np.nan
        rays[2, 4:7] = [1.0, 0.0, 0.0]
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    for kind, bits in KINDS:
        for ratio in (0.25, 0.0):
            p = rr.key_params(kind, bits, lo, hi, ratio)
            k, _, _ = rr.rr_compute_keys(to_dev(rays), p)
            ref = O.keys(rays, kind, bits, lo, hi, ratio)
            assert np.array_equal(keys_np(k, bits), ref), (kind, bits, ratio)


def test_keys_golden_values(rr):
    import test_oracle_keys as T
    for name, kind, bits, o, d, ratio, expected in T.load_golden():
        r = np.array([[*o, 0, *d, np.inf]], np.float32)
        p = rr.key_params(kind, bits, (0, 0, 0), (1, 1, 1), ratio)
        k, _, _ = rr.rr_compute_keys(to_dev(r), p)
        assert int(keys_np(k, bits)[0]) == expected, name


def test_keys_compaction(rr):
    w = W.city_small(seed=3, width=128, height=72, depth=2)
    lo, hi = O.scene_box(w.tris)
    live = O.compact(w.alive)
    assert 0 < len(live) < len(w.alive)
    for kind, bits in KINDS:
        p = rr.key_params(kind, bits, lo, hi)
        k, idx, cnt = rr.rr_compute_keys(to_dev(w.rays), p, alive=to_dev(w.alive))
        c = int(cnt.cpu().numpy().view(np.uint32)[0])
        assert c == len(live)
        assert np.array_equal(idx_np(idx)[:c], live)
        assert np.array_equal(keys_np(k, bits)[:c], O.keys(w.rays[live], kind, bits, lo, hi))


def test_keys_compaction_all_dead_and_all_live(rr):
    rays = W.random_rays(5, 3000)
    p = rr.key_params(rr.RR_KEY_ORIGIN_DIRECTION, 32, (0, 0, 0), (1, 1, 1))
    for alive in (np.zeros(3000, np.uint8), np.ones(3000, np.uint8)):
        k, idx, cnt = rr.rr_compute_keys(to_dev(rays), p, alive=to_dev(alive))
        c = int(cnt.cpu().numpy()[0])
        assert c == int(alive.sum())
        assert np.array_equal(idx_np(idx)[:c], O.compact(alive))


# ------------------------------------------------------------------- sort

def _random_keys(n, bits, seed, dup_bits):
    rng = np.random.default_rng(seed)
    if bits == 32:
        k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        k &= np.uint32(~((1 << dup_bits) - 1) & 0xFFFFFFFF)
    else:
        k = rng.integers(0, 1 << 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
        k &= ~np.uint64((1 << dup_bits) - 1)
    return k


@pytest.mark.parametrize("n", [1, 2, 100, 4095, 4096, 4097, 65553, 300007])
@pytest.mark.parametrize("bits", [32, 64])
def test_sort_matches_stable_order(rr, n, bits):
    for dup in (0, bits - 6):  # distinct-ish keys, then only 64 distinct values
        k = _random_keys(n, bits, n + bits + dup, dup)
        dt = torch.int32 if bits == 32 else torch.int64
        kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
        idx = torch.arange(n, dtype=torch.int32, device=DEV)
        rr.rr_sort(kd, idx)
        ks, ix = O.sort_pairs(k)
        assert kd.dtype == dt
        assert np.array_equal(keys_np(kd, bits), ks), (n, bits, dup)
        assert np.array_equal(idx_np(idx), ix), (n, bits, dup)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("digit_bits,kpt", [(8, 16), (8, 8), (4, 16), (4, 8)])
def test_sort_every_configuration_identical(rr, bits, digit_bits, kpt):
    n = 123457
    k = _random_keys(n, bits, 99, bits - 10)
    kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
    idx = torch.arange(n, dtype=torch.int32, device=DEV)
    rr.rr_sort(kd, idx, digit_bits=digit_bits, keys_per_thread=kpt)
    ks, ix = O.sort_pairs(k)
    assert np.array_equal(idx_np(idx), ix)
    assert np.array_equal(keys_np(kd, bits), ks)



def _edge_keys(case, n, bits, rng):
    """Key distributions at the ends of what the digit passes meet."""
    top = (1 << bits) - 1
    dt = np.uint32 if bits == 32 else np.uint64
    if case == "all_equal":
        return np.full(n, 0x5A5A5A5A5A5A5A5A & top, dt)
    if case == "ascending":
        return np.sort(rng.integers(0, top, n, dtype=np.uint64, endpoint=True).astype(dt) >> dt(3))
    if case == "descending":
        return np.sort(rng.integers(0, top, n, dtype=np.uint64, endpoint=True).astype(dt))[::-1].copy()
    if case == "extremes":
        return np.where(rng.integers(0, 2, n) == 1, dt(top), dt(0)).astype(dt)
    if case == "low_byte_only":
        return (rng.integers(0, 256, n, dtype=np.uint64) | np.uint64(0x1234567800000000 & top)).astype(dt)
    if case == "top_byte_only":
        return (rng.integers(0, 256, n, dtype=np.uint64) << np.uint64(bits - 8)).astype(dt)
    if case == "one_hot_value":
        k = rng.integers(0, top, n, dtype=np.uint64, endpoint=True).astype(dt)
        k[rng.random(n) < 0.9] = dt(0x00FF00FF00FF00FF & top)
        return k
    raise ValueError(case)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("case", ["all_equal", "ascending", "descending", "extremes", "low_byte_only",
                                  "top_byte_only", "one_hot_value"])
def test_sort_edge_distributions(rr, bits, case):
    """Stability by input position with indices that do not ascend (reversed,
    then a random permutation), in the default configuration and two others."""
    n = 300007
    rng = np.random.default_rng(bits * 100 + len(case))
    k = _edge_keys(case, n, bits, rng)
    _, perm = O.sort_pairs(k)  # stable order of the positions
    ks = k[perm]
    for idx_in, cfg in ((np.arange(n, dtype=np.uint32)[::-1].copy(), {}),
                        (rng.permutation(n).astype(np.uint32), {"digit_bits": 8, "keys_per_thread": 16}),
                        (rng.permutation(n).astype(np.uint32), {"digit_bits": 4, "keys_per_thread": 8})):
        kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
        idx = to_dev(idx_in.view(np.int32))
        rr.rr_sort(kd, idx, **cfg)
        assert np.array_equal(keys_np(kd, bits), ks), (case, cfg)
        assert np.array_equal(idx_np(idx), idx_in[perm]), (case, cfg)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("n", [1_228_801, 2_621_443])
def test_sort_tile_runs_per_xcd(rr, n, bits):
    """Sizes where the fixed tile order deals runs of 16 tiles to the XCDs:
    ~300 tiles (whole spans of 128 tiles, then blocks that keep their own
    tile) and ~640 tiles (more tiles than resident blocks, a partial last
    round); reversed input indices, 2^20 distinct keys."""
    k = _random_keys(n, bits, n + bits, bits - 20)
    idx_in = np.arange(n, dtype=np.uint32)[::-1].copy()
    _, perm = O.sort_pairs(k)
    kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
    idx = to_dev(idx_in.view(np.int32))
    rr.rr_sort(kd, idx)
    assert np.array_equal(keys_np(kd, bits), k[perm])
    assert np.array_equal(idx_np(idx), idx_in[perm])


def test_sort_past_2_24_with_device_count(rr):
    """The 16-keys-per-thread configuration rr_sort takes from 2^24 keys on,
    with a device count below the capacity and 2^20 distinct 64-bit keys."""
    n_max, n = (1 << 24) + 4097, (1 << 24) + 1001
    k = _random_keys(n_max, 64, 77, 44)
    kd = to_dev(k.view(np.int64))
    idx = torch.arange(n_max, dtype=torch.int32, device=DEV)
    cnt = torch.tensor([n], dtype=torch.int32, device=DEV)
    rr.rr_sort(kd, idx, count=cnt)
    ks, ix = O.sort_pairs(k[:n])
    got_k = keys_np(kd, 64)
    assert np.array_equal(idx_np(idx)[:n], ix)
    assert np.array_equal(got_k[:n], ks)
    assert np.array_equal(got_k[n:], k[n:])


def test_sort_device_count(rr):
    n_max, n = 50000, 31337
    k = _random_keys(n_max, 64, 5, 20)
    kd = to_dev(k.view(np.int64))
    idx = torch.arange(n_max, dtype=torch.int32, device=DEV)
    cnt = torch.tensor([n], dtype=torch.int32, device=DEV)
    rr.rr_sort(kd, idx, count=cnt)
    ks, ix = O.sort_pairs(k[:n])
    assert np.array_equal(idx_np(idx)[:n], ix)
    assert np.array_equal(keys_np(kd, 64)[:n], ks)
    # the tail beyond the count is untouched
    assert np.array_equal(keys_np(kd, 64)[n:], k[n:])


def test_sort_twice_is_deterministic(rr):
    n = 200000
    k = _random_keys(n, 32, 8, 12)
    outs = []
    for _ in range(2):
        kd = to_dev(k.view(np.int32))
        idx = torch.arange(n, dtype=torch.int32, device=DEV)
        rr.rr_sort(kd, idx)
        outs.append(idx_np(idx).copy())
    assert np.array_equal(outs[0], outs[1])


# ----------------------------------------------------------------- gather

def test_gather_and_scatter(rr):
    rng = np.random.default_rng(3)
    n = 100003
    rays = rng.normal(size=(n, 8)).astype(np.float32)
    perm = rng.permutation(n).astype(np.uint32)
    g = rr.rr_gather(to_dev(rays), to_dev(perm.view(np.int32)))
    assert np.array_equal(g.cpu().numpy(), rays[perm])
    hits = rng.normal(size=(n, 4)).astype(np.float32)
    s = rr.rr_scatter_hits(to_dev(hits), to_dev(perm.view(np.int32)))
    assert np.array_equal(s.cpu().numpy()[perm], hits)


# ------------------------------------------------------------------ trace

@pytest.mark.parametrize("builder", [0, 1])
def test_trace_soup_matches_brute_force(rr, soup65k, builder):
    w = soup65k
    ref = O.brute_force(w.tris, w.rays)
    with rr.Scene(w.tris, builder=builder) as sc:
        h = rr.hits_to_numpy(rr.rr_trace(sc, to_dev(w.rays)))
    assert_hits_match(h, ref, w.rays, w.tris, f"soup builder {builder}")


def test_trace_small_city_matches_oracle(rr):
    w = W.city_small(seed=11, width=160, height=90, depth=1)
    ref = O.BVH(w.tris).trace(w.rays)
    for builder in (0, 1):
        with rr.Scene(w.tris, builder=builder) as sc:
            h = rr.hits_to_numpy(rr.rr_trace(sc, to_dev(w.rays)))
        assert_hits_match(h, ref, w.rays, w.tris, f"city builder {builder}")


def test_trace_ragged_counts_and_refill(rr, soup65k):
    """Ray counts around the 64-ray packets and the XCD shares of the
    persistent waves (fewer blocks than XCDs, ragged last packets), a device
    count below the capacity (slots past it untouched), and several refill
    thresholds: the same hits every time."""
    w = soup65k
    N = 30011
    rays = np.ascontiguousarray(w.rays[:N])
    ref = O.brute_force(w.tris, rays)
    with rr.Scene(w.tris, builder=1) as sc:
        for n in (1, 63, 64, 65, 511, 2049, 4097, 12345, N):
            h = rr.hits_to_numpy(rr.rr_trace(sc, to_dev(rays[:n])))
            assert_hits_match(h, ref[:n], rays[:n], w.tris, f"n={n}")
        dr = to_dev(rays)
        full = rr.rr_trace(sc, dr)
        cnt = torch.tensor([7777], dtype=torch.int32, device=DEV)
        out = torch.full((N, 4), -3.0, dtype=torch.float32, device=DEV)
        rr.rr_trace(sc, dr, count=cnt, hits=out)
        assert torch.equal(out[:7777].view(torch.int32), full[:7777].view(torch.int32))
        assert bool((out[7777:] == -3.0).all())
        for refill in (1, 8, 33, 64):
            h = rr.rr_trace(sc, dr, refill=refill)
            assert torch.equal(h.view(torch.int32), full.view(torch.int32)), f"refill {refill}"
    assert_hits_match(rr.hits_to_numpy(full), ref, rays, w.tris, "full")


def test_persistent_trace_device_counts(rr, soup65k):
    """The one-lane persistent trace (rr_trace with a refill threshold) under a
    device-side ray count below the capacity.  The count sets where the XCD
    shares end, and the waves of a block take rays from the block's packets
    through a shared counter until the share is used up.  Counts of 0 and 1,
    around packets and blocks, and just below the capacity, each at three
    refill thresholds: the oracle's hits for the counted rays, and the slots
    past the count left untouched."""
    w = soup65k
    N = 30011
    rays = np.ascontiguousarray(w.rays[:N])
    ref = O.brute_force(w.tris, rays)
    dr = to_dev(rays)
    out = torch.empty((N, 4), dtype=torch.float32, device=DEV)
    with rr.Scene(w.tris, builder=1) as sc:
        for count in (0, 1, 255, 257, 6161, 16385, N - 1, N):
            cnt = torch.tensor([count], dtype=torch.int32, device=DEV)
            for refill in (1, 16, 64):
                out.fill_(-3.0)
                rr.rr_trace(sc, dr, count=cnt, hits=out, refill=refill)
                torch.cuda.synchronize()
                assert bool((out[count:] == -3.0).all()), (count, refill)
                if count:
                    assert_hits_match(rr.hits_to_numpy(out[:count]), ref[:count], rays[:count], w.tris,
                                      f"count={count} refill={refill}")


def test_four_lane_trace_equals_the_persistent_kernel(rr):
    """rr_trace traces small launches with four lanes per ray (up to what one
    resident wave of its blocks holds, about 98K rays) and larger ones with
    one lane per ray; rr_trace_ex always takes the latter.  On bounce-2 rays
    of the city both give the same hits bit for bit on both sides of the
    switch, with a device count below the capacity, and through an index
    (the fused call's indirect trace); a sample is checked against the
    oracle."""
    w = W.city_small(seed=11, width=480, height=270, depth=1)
    rays = np.ascontiguousarray(w.rays)
    n_all = rays.shape[0]
    assert n_all > 110000
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        dr = to_dev(rays)
        for n in (1, 3, 64, 65, 4097, 65536, 98303, 98304, 98305, 110001):
            r = dr[:n]
            a = rr.rr_trace(sc, r)
            b = rr.rr_trace(sc, r, refill=8)
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), n
        n = 90000
        cnt = torch.tensor([54321], dtype=torch.int32, device=DEV)
        out = torch.full((n, 4), -3.0, dtype=torch.float32, device=DEV)
        rr.rr_trace(sc, dr[:n], count=cnt, hits=out)
        full = rr.rr_trace(sc, dr[:n], refill=8)
        assert torch.equal(out[:54321].view(torch.int32), full[:54321].view(torch.int32))
        assert bool((out[54321:] == -3.0).all())
        sample = W.sample_indices(11, 7, 4096, n)
        assert_hits_match(rr.hits_to_numpy(full)[sample], bvh.trace(rays[sample]), rays[sample], w.tris, "sample")
        lo, hi = sc.bounds()
        p = rr.key_params(O.KIND_OD, 32, lo, hi, 0.25)
        for flags in (rr.RR_INDIRECT, rr.RR_INDIRECT | rr.RR_HITS_ORIGINAL_ORDER, rr.RR_HITS_ORIGINAL_ORDER):
            h, _, _ = rr.rr_reorder_and_trace(sc, dr[:n], p, flags=flags)
            if flags & rr.RR_HITS_ORIGINAL_ORDER:
                assert torch.equal(h.view(torch.int32), full.view(torch.int32)), flags


def test_trace_tiny_scenes_and_ties(rr):
    # one triangle (the root is a leaf); shared-edge tie goes to the lower id
    a = [1, 0, 0.5, 0, 1, 0.5, 1, 1, 0.5]
    b = [0, 0, 0.5, 1, 0, 0.5, 0, 1, 0.5]
    rays = np.array([[0.5, 0.5, 0, 0, 0, 0, 1, np.inf],
                     [0.25, 0.25, 0, 0, 0, 0, 1, np.inf],
                     [0.25, 0.25, 0, 0, 0, 0, -1, np.inf],
                     [0.25, 0.25, 0, 0, 0, 0, 1, 0.5]], np.float32)
    for tris in ([b], [a, b], [b, a]):
        T = np.array(tris, np.float32)
        ref = O.brute_force(T, rays)
        with rr.Scene(T) as sc:
            h = rr.hits_to_numpy(rr.rr_trace(sc, to_dev(rays)))
        assert h.tobytes() == ref.tobytes()



@pytest.mark.parametrize("scale", [1.0, 2.0 ** -40, 2.0 ** 40])
def test_trace_degenerate_geometry(rr, scale):
    """Zero-area and duplicate triangles, rays parallel to triangles, axis-
    aligned and negative-zero directions, empty and inverted intervals, at
    three scales (powers of two, so the scaled inputs are exact): hits
    bit-identical to brute force with both builders, alone and through the
    fused call."""
    T, rays = W.degenerate(12, 3000, 8192, scale)
    ref = O.brute_force(T, rays)
    assert (ref["prim"] >= 0).sum() > 1000  # the scene is hit
    for builder in (0, 1):
        with rr.Scene(T, builder=builder) as sc:
            rd = to_dev(rays)
            h = rr.hits_to_numpy(rr.rr_trace(sc, rd))
            assert h.tobytes() == ref.tobytes(), (scale, builder)
            # reordered by the Two Point key, hits scattered back to ray order
            lo, hi = sc.bounds()
            p = rr.key_params(O.KIND_OT, 64, lo, hi, 0.25)
            back, _, _ = rr.rr_reorder_and_trace(sc, rd, p, flags=rr.RR_HITS_ORIGINAL_ORDER)
            assert rr.hits_to_numpy(back).tobytes() == ref.tobytes(), (scale, builder)


def stacked_scene(n, n_rays, seed):
    """n near-parallel triangles stacked in z over one unit footprint (ids in
    random order), and rays that cross the stack: from below, from above,
    and from inside it in random directions.  Every box of a descent is hit,
    so a traversal pushes three entries per level of the 4-wide tree."""
    rng = np.random.default_rng(seed)
    z = (np.arange(n) + rng.uniform(0.1, 0.9, n)) / n
    a = rng.uniform(-0.01, 0.01, (n, 2))
    T = np.zeros((n, 9), np.float32)
    T[:, 0], T[:, 1], T[:, 2] = a[:, 0], a[:, 1], z
    T[:, 3], T[:, 4], T[:, 5] = a[:, 0] + 1.0, a[:, 1], z
    T[:, 6], T[:, 7], T[:, 8] = a[:, 0], a[:, 1] + 1.0, z
    T = np.ascontiguousarray(T[rng.permutation(n)])
    m = n_rays // 3
    xy = rng.uniform(0.02, 0.45, (n_rays, 2))
    o = np.zeros((n_rays, 3))
    d = np.zeros((n_rays, 3))
    o[:, :2] = xy
    o[:m, 2] = -0.5
    d[:m] = np.c_[rng.normal(0, 0.05, (m, 2)), np.ones(m)]
    o[m:2 * m, 2] = 1.5
    d[m:2 * m] = np.c_[rng.normal(0, 0.05, (m, 2)), -np.ones(m)]
    o[2 * m:, 2] = rng.uniform(0.0, 1.0, n_rays - 2 * m)
    d[2 * m:] = rng.normal(size=(n_rays - 2 * m, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n_rays, 8), np.float32)
    rays[:, 0:3], rays[:, 4:7] = o, d
    rays[:, 3], rays[:, 7] = 0.0, np.inf
    return T, rays


@pytest.mark.parametrize("builder", [0, 1, 1 | 2])
def test_trace_deep_stack_spills_to_scratch(rr, builder):
    """A scene whose traversals need more stack entries than the 16 held in
    LDS: the profiling counters show the scratch part in use, and every hit
    equals brute force (with both builders and full-precision nodes)."""
    T, rays = stacked_scene(1 << 17, 3072, 61)
    ref = O.brute_force(T, rays)
    assert (ref["prim"] >= 0).mean() > 0.5
    with rr.Scene(T, builder=builder) as sc:
        rd = to_dev(rays)
        prof = rr.rr_trace_profile(sc, rd)
        assert prof["max_stack"] > 16 and prof["spill_pushes"] > 0, prof
        h = rr.hits_to_numpy(rr.rr_trace(sc, rd))
        assert_hits_match(h, ref, rays, T, f"stack builder {builder}")
        # the persistent one-lane-per-ray kernel (rr_trace_ex; rr_trace takes the
        # four-lane kernel at this size) spills too and gives the same hits
        h1 = rr.hits_to_numpy(rr.rr_trace(sc, rd, refill=8))
        assert h1.tobytes() == h.tobytes()
        # the profiling variant returns the same hits
        hp = torch.empty((rays.shape[0], 4), dtype=torch.float32, device=DEV)
        rr.rr_trace_profile(sc, rd, hits=hp)
        assert rr.hits_to_numpy(hp).tobytes() == h.tobytes()
        # reordered (and traced in key order) the hits are unchanged
        lo, hi = sc.bounds()
        back, _, _ = rr.rr_reorder_and_trace(sc, rd, rr.key_params(O.KIND_OT, 64, lo, hi, 0.25),
                                             flags=rr.RR_HITS_ORIGINAL_ORDER)
        assert rr.hits_to_numpy(back).tobytes() == h.tobytes()


# ---------------------------------------------------------- fused pipeline

@pytest.mark.parametrize("kind,bits", KINDS + [(O.KIND_NONE, 32)])
def test_reorder_and_trace_soup(rr, soup65k, kind, bits):
    w = soup65k
    bvh = O.BVH(w.tris)
    lo, hi = O.scene_box(w.tris)
    ref = O.reorder_and_trace(bvh, w.rays, kind, bits, lo, hi)
    with rr.Scene(w.tris) as sc:
        rays = to_dev(w.rays)
        p = rr.key_params(kind, bits, lo, hi)
        base = rr.hits_to_numpy(rr.rr_trace(sc, rays))
        for flags in (0, rr.RR_INDIRECT, rr.RR_HITS_ORIGINAL_ORDER, rr.RR_HITS_ORIGINAL_ORDER | rr.RR_INDIRECT):
            hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, flags=flags)
            h = rr.hits_to_numpy(hits)
            assert np.array_equal(idx_np(perm), ref["idx"]), flags
            assert int(cnt.cpu().numpy()[0]) == len(w.rays)
            if flags & rr.RR_HITS_ORIGINAL_ORDER:
                assert h.tobytes() == base.tobytes(), flags      # scatter-back == unsorted, bit for bit
            else:
                assert_hits_match(h, ref["hits"], ref["rays"], w.tris, f"sorted {kind}/{bits}/{flags}")


def test_reorder_and_trace_with_compaction(rr):
    w = W.city_small(seed=5, width=128, height=72, depth=2)
    bvh = O.BVH(w.tris)
    lo, hi = O.scene_box(w.tris)
    with rr.Scene(w.tris) as sc:
        rays, alive = to_dev(w.rays), to_dev(w.alive)
        full = rr.hits_to_numpy(rr.rr_trace(sc, rays))
        for kind, bits in [(O.KIND_NONE, 32), (O.KIND_OD, 32), (O.KIND_OT, 64)]:
            ref = O.reorder_and_trace(bvh, w.rays, kind, bits, lo, hi, alive=w.alive)
            p = rr.key_params(kind, bits, lo, hi)
            hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, alive=alive, flags=rr.RR_HITS_ORIGINAL_ORDER)
            c = int(cnt.cpu().numpy()[0])
            assert c == len(ref["idx"])
            assert np.array_equal(idx_np(perm)[:c], ref["idx"])
            h = rr.hits_to_numpy(hits)
            live = w.alive.astype(bool)
            assert h[live].tobytes() == full[live].tobytes()
            assert np.all(h["prim"][~live] == -1) and np.all(np.isinf(h["t"][~live]))


def test_reorder_and_trace_dense_ragged_sizes(rr, soup65k):
    """The dense fused call (keys and digit histograms in one kernel, 4096
    rays per histogram unit) at ragged sizes around the unit and the sort
    tile, one ray included: permutation against the oracle's stable order of
    its keys, key-order hits against the plain trace through it."""
    w = soup65k
    lo, hi = O.scene_box(w.tris)
    with rr.Scene(w.tris) as sc:
        for n in (1, 2, 63, 4095, 4096, 4097, 8193, 12289):
            rays_np = np.ascontiguousarray(w.rays[:n])
            rays = to_dev(rays_np)
            base = rr.hits_to_numpy(rr.rr_trace(sc, rays))
            for kind, bits in [(O.KIND_OD, 32), (O.KIND_OT, 64)]:
                _, want = O.sort_pairs(O.keys(rays_np, kind, bits, lo, hi))
                p = rr.key_params(kind, bits, lo, hi)
                hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, flags=0)
                assert int(cnt.cpu().numpy()[0]) == n
                assert np.array_equal(idx_np(perm), want), (n, kind, bits)
                assert rr.hits_to_numpy(hits).tobytes() == base[want].tobytes(), (n, kind, bits)


def test_reorder_and_trace_compaction_edges_every_flag(rr, soup65k):
    """Live sets at the edges (none, only the first slot, only the last slot,
    every other slot, all) through the fused call with the gather in the
    sort's last pass, the gather kernel (local sort) and the indirect trace,
    hits in key order and in ray order: the live hits equal the plain trace,
    the key-order hits follow the permutation, and the count is exact."""
    w = soup65k
    n = 5003
    rays_np = np.ascontiguousarray(w.rays[:n])
    lo, hi = O.scene_box(w.tris)
    masks = {"none": np.zeros(n, np.uint8), "first": np.eye(1, n, 0, dtype=np.uint8)[0],
             "last": np.eye(1, n, n - 1, dtype=np.uint8)[0], "alternate": (np.arange(n) % 2).astype(np.uint8),
             "all": np.ones(n, np.uint8)}
    with rr.Scene(w.tris) as sc:
        rays = to_dev(rays_np)
        full = rr.hits_to_numpy(rr.rr_trace(sc, rays))
        for kind, bits in [(O.KIND_OD, 32), (O.KIND_OT, 64)]:
            p = rr.key_params(kind, bits, lo, hi)
            for mname, m in masks.items():
                live = np.nonzero(m)[0]
                ref_idx = live.astype(np.uint32)
                if len(live):
                    cidx = O.compact(m)
                    _, ref_idx = O.sort_pairs(O.keys(rays_np[cidx], kind, bits, lo, hi), cidx)
                for flags in (0, rr.RR_HITS_ORIGINAL_ORDER, rr.RR_INDIRECT, rr.RR_LOCAL_SORT_2048):
                    what = f"kind {kind}/{bits} mask {mname} flags {flags}"
                    hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, alive=to_dev(m), flags=flags)
                    c = int(cnt.cpu().numpy()[0])
                    assert c == len(live), what
                    pi = idx_np(perm)[:c]
                    if flags & rr.RR_LOCAL_SORT_2048:
                        assert np.array_equal(np.sort(pi), live), what
                    else:
                        assert np.array_equal(pi, ref_idx), what
                    h = rr.hits_to_numpy(hits)
                    if flags & rr.RR_HITS_ORIGINAL_ORDER:
                        assert h[live].tobytes() == full[live].tobytes(), what
                        dead = m == 0
                        assert np.all(h["prim"][dead] == -1) and np.all(np.isinf(h["t"][dead])), what
                    else:
                        assert h[:c].tobytes() == full[pi].tobytes(), what


def test_zero_rays(rr, soup65k):
    w = soup65k
    with rr.Scene(w.tris[:10]) as sc:
        rays = torch.empty((0, 8), dtype=torch.float32, device=DEV)
        p = rr.key_params(rr.RR_KEY_ORIGIN_DIRECTION, 32, (0, 0, 0), (1, 1, 1))
        hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, ws=rr.workspace(256, DEV))
        assert int(cnt.cpu().numpy()[0]) == 0
        assert rr.rr_trace(sc, rays).shape == (0, 4)


def test_host_pointer_rejected(rr, soup65k):
    with rr.Scene(soup65k.tris[:10]) as sc:
        host = torch.zeros((10, 8), dtype=torch.float32)
        with pytest.raises(ValueError):
            rr.rr_trace(sc, host)
        lib = rr.load()
        hits = torch.empty((10, 4), dtype=torch.float32, device=DEV)
        st = lib.rr_trace(sc.handle, host.data_ptr(), 10, None, hits.data_ptr(), None)
        assert st == -1
