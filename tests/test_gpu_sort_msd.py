"""GPU parity of the most-significant-digit sort (rr_sort_msd, and the fused
call with RR_SORT_MSD): two stable scatter passes on the two highest digits
in which the keys differ, then the buckets of equal top digits sorted on
their other digits: each by one wave when no bucket holds more than 512
keys, else in batches in LDS, a bucket larger than a batch by one block in
chunks through global memory.  Its result must be the stable order of the
oracle (Section 3.2), and the LSD sort's (rr_sort and rr_sort_ex) bit for
bit, whatever the key distribution: buckets of 1 to 512 keys and one of 513,
buckets that straddle the batch kernel's windows, buckets too large for LDS
with an odd or even number of differing digits below the top two, keys
differing in one digit only, input indices that do not ascend, a device
count below the capacity, evenly spread keys at wavefront sizes."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from hitcheck import assert_hits_match

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda"
WAVE_CAP = 512  # largest bucket that one wave sorts


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


def run_all(rr, k, bits, idx_in=None, count=None, ways=None):
    """The MSD sort (64-bit keys), rr_sort and the LSD sort (rr_sort_ex) of
    the same pairs; each must give the oracle's stable order by input
    position, so all agree bit for bit."""
    n = k.shape[0]
    idx_in = np.arange(n, dtype=np.uint32) if idx_in is None else idx_in
    m = n if count is None else count
    _, perm = O.sort_pairs(k[:m])
    if ways is None:
        ways = ("msd", "auto", "lsd") if bits == 64 else ("auto", "lsd")
    for way in ways:
        kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
        idx = to_dev(idx_in.view(np.int32))
        cnt = None if count is None else torch.tensor([count], dtype=torch.int32, device=DEV)
        rr.rr_sort(kd, idx, count=cnt, key_bits=bits, msd=way == "msd", keys_per_thread=8 if way == "lsd" else None)
        gk, gi = keys_np(kd, bits), idx.cpu().numpy().view(np.uint32)
        assert np.array_equal(gk[:m], k[:m][perm]), ("keys", way)
        assert np.array_equal(gi[:m], idx_in[:m][perm]), ("idx", way)
        assert np.array_equal(gk[m:], k[m:]) and np.array_equal(gi[m:], idx_in[m:]), ("tail", way)


def bucket_max(k):
    """The largest bucket of the MSD sort for 64-bit keys k: keys of equal
    digits dh and dl, dh the highest 8-bit digit in which the keys differ and
    dl the next lower one that differs (dh alone when none does)."""
    k = k.astype(np.uint64)
    x = int(np.bitwise_or.reduce(k ^ k[0]))
    digs = [d for d in range(8) if (x >> (8 * d)) & 255]
    if not digs:
        return int(k.size)
    dh = max(digs)
    b = (k >> np.uint64(8 * dh)) & np.uint64(255)
    low = [d for d in digs if d < dh]
    if low:
        b = b * np.uint64(256) + ((k >> np.uint64(8 * max(low))) & np.uint64(255))
    return int(np.bincount(b.astype(np.int64)).max())


def wave_bucket_keys(seed, extra=()):
    """Buckets (distinct top 16 bits) of 1 to 512 keys, the sizes around
    every multiple of 64 (a wave's rows of keys) among them, plus the sizes in
    extra.  In each bucket a random subset of the six lower digits varies
    (none: all keys equal; all six: six in-wave passes).  Positions
    shuffled."""
    rng = np.random.default_rng(seed)
    edges = [1, 2, 511, 512] + [64 * r + e for r in range(1, 8) for e in (-1, 0, 1)]
    sizes = np.concatenate([rng.integers(1, 513, 300), edges, list(extra)]).astype(np.int64)
    rng.shuffle(sizes)
    prefixes = rng.choice(1 << 16, sizes.shape[0], replace=False).astype(np.uint64)
    masks = np.zeros(sizes.shape[0], np.uint64)
    for i in range(sizes.shape[0]):
        for d in range(6):
            if rng.random() < 0.6:
                masks[i] |= np.uint64(255 << (8 * d))
    masks[:3] = 0
    masks[3:6] = np.uint64((1 << 48) - 1)
    n = int(sizes.sum())
    k = np.repeat(prefixes << np.uint64(48), sizes) | (rng.integers(0, 1 << 48, n, dtype=np.uint64)
                                                       & np.repeat(masks, sizes))
    return k[rng.permutation(n)], rng


def test_every_bucket_sorted_by_one_wave(rr):
    """Buckets of at most 512 keys: every bucket is sorted by one wave."""
    k, rng = wave_bucket_keys(512)
    assert bucket_max(k) == WAVE_CAP
    run_all(rr, k, 64, idx_in=rng.permutation(k.shape[0]).astype(np.uint32))


def test_one_bucket_of_513_keys(rr):
    """The same kind of buckets and one of 513 keys: the batch kernel sorts
    them all."""
    k, rng = wave_bucket_keys(513, extra=(WAVE_CAP + 1,))
    assert bucket_max(k) == WAVE_CAP + 1
    run_all(rr, k, 64, idx_in=rng.permutation(k.shape[0]).astype(np.uint32))


@pytest.mark.parametrize("n", [2_073_600, 8_294_400])
def test_evenly_spread_keys_at_wavefront_sizes(rr, n):
    """Uniform 64-bit keys of 1080p and 2160p wavefronts (buckets of ~32 and
    ~127 keys, every one sorted by a wave) with a device count one below the
    capacity."""
    rng = np.random.default_rng(n)
    k = rng.integers(0, (1 << 64) - 1, n, dtype=np.uint64, endpoint=True)
    assert bucket_max(k[: n - 1]) <= WAVE_CAP
    run_all(rr, k, 64, count=n - 1)


def big_bucket_keys(n, bits, low_bits, frac, seed):
    """A fraction `frac` of the keys share their top 16 bits and differ only
    in their low `low_bits` bits (one bucket far larger than a batch); the
    rest are uniform."""
    rng = np.random.default_rng(seed)
    top = (1 << bits) - 1
    k = rng.integers(0, top, n, dtype=np.uint64, endpoint=True)
    sel = rng.random(n) < frac
    prefix = np.uint64(0x00AB << (bits - 16))
    k[sel] = prefix | rng.integers(0, 1 << low_bits, int(sel.sum()), dtype=np.uint64)
    return k.astype(np.uint32 if bits == 32 else np.uint64)


@pytest.mark.parametrize("low_bits", [24, 16, 40])
def test_buckets_larger_than_a_batch(rr, low_bits):
    """One bucket of ~180K keys (an odd and an even number of differing
    digits below the top two), with reversed input indices."""
    n = 300007
    k = big_bucket_keys(n, 64, low_bits, 0.6, 7 + low_bits)
    run_all(rr, k, 64, idx_in=np.arange(n, dtype=np.uint32)[::-1].copy())


def test_bucket_sizes_around_the_batch(rr):
    """Buckets of 1 to ~12K keys (sizes spread over the whole range, some
    just above and below a batch of 8192 and straddling the kernel's 8192-key
    windows), keys differing in every digit inside a bucket, shuffled input
    indices."""
    rng = np.random.default_rng(64)
    sizes = np.concatenate([rng.integers(1, 12000, 40), [8191, 8192, 8193, 1, 2, 4095, 4097]])
    rng.shuffle(sizes)
    n = int(sizes.sum())
    prefixes = np.sort(rng.choice(1 << 16, sizes.shape[0], replace=False)).astype(np.uint64)
    k = np.repeat(prefixes << np.uint64(48), sizes)
    k |= rng.integers(0, 1 << 48, n, dtype=np.uint64)
    k = k[rng.permutation(n)]
    run_all(rr, k, 64, idx_in=rng.permutation(n).astype(np.uint32))


@pytest.mark.parametrize("n", [1, 2, 3, 100, 8191, 8192, 8193, 16385, 65537])
def test_small_and_window_sizes(rr, n):
    """Sizes ragged against the bucket kernel's 8,192-key windows."""
    rng = np.random.default_rng(n)
    k = rng.integers(0, (1 << 64) - 1, n, dtype=np.uint64, endpoint=True)
    k = k >> np.uint64(rng.integers(0, 63))
    run_all(rr, k, 64)


@pytest.mark.parametrize("digit", [0, 1, 3])
def test_one_or_two_differing_digits(rr, digit):
    """Keys that differ in one digit only, or in that digit and the top one:
    the two scatter passes alone order them."""
    n = 200003
    rng = np.random.default_rng(digit * 3 + 64)
    base = np.uint64(0x0123456789ABCDEF)
    d = rng.integers(0, 256, n, dtype=np.uint64)
    k1 = (base & ~np.uint64(255 << (8 * digit))) | (d << np.uint64(8 * digit))
    run_all(rr, k1, 64)
    top = rng.integers(0, 4, n, dtype=np.uint64) << np.uint64(56)
    k2 = (k1 & np.uint64((1 << 56) - 1)) | top
    run_all(rr, k2, 64)


def test_device_count_and_big_bucket(rr):
    n_max, n = 250000, 190001
    k = big_bucket_keys(n_max, 64, 20, 0.5, 3)
    run_all(rr, k, 64, count=n)
    run_all(rr, k, 64, count=0)


def test_fused_call_with_a_bucket_larger_than_a_batch(rr):
    """Half the rays start at one point (origin-direction keys then share
    their origin bits, so one bucket holds them all and the sort's large-
    bucket path also gathers the rays): with RR_SORT_MSD the fused call's
    permutation equals the oracle's and its hits match under the closest-hit
    rule; without the flag (the LSD sort at this size) it gives the same."""
    w = W.soup(seed=9, n_rays=120000, n_tris=2048)
    rays = w.rays.copy()
    rays[::2, 0:3] = np.array([0.31, 0.62, 0.47], np.float32)
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
        for kind in (O.KIND_OD, O.KIND_OT):
            p = rr.key_params(kind, 64, lo, hi, 0.25)
            ref = O.reorder_and_trace(bvh, rays, kind, 64, lo, hi, 0.25)
            for flags in (rr.RR_SORT_MSD, 0, rr.RR_SORT_MSD | rr.RR_HITS_ORIGINAL_ORDER):
                hits, perm, _ = rr.rr_reorder_and_trace(sc, to_dev(rays), p, flags=flags)
                assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref["idx"]), (kind, flags)
                h = rr.hits_to_numpy(hits)
                if flags & rr.RR_HITS_ORIGINAL_ORDER:
                    back = np.empty_like(h)
                    back[ref["idx"]] = ref["hits"]
                    assert_hits_match(h, back, rays, w.tris, f"{kind}/{flags}")
                else:
                    assert_hits_match(h, ref["hits"], ref["rays"], w.tris, f"{kind}/{flags}")


def test_fused_call_with_buckets_of_a_wave(rr):
    """Distinct rays in a soup scene: the 64-bit keys fill buckets of a few
    keys each, so the wave kernel sorts them and also gathers the rays; the
    permutation equals the oracle's and the hits match under the closest-hit
    rule."""
    w = W.soup(seed=11, n_rays=120000, n_tris=2048)
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
        for kind in (O.KIND_OD, O.KIND_OT):
            ref = O.reorder_and_trace(bvh, w.rays, kind, 64, lo, hi, 0.25)
            assert bucket_max(O.keys(w.rays, kind, 64, lo, hi, 0.25)) <= WAVE_CAP
            p = rr.key_params(kind, 64, lo, hi, 0.25)
            hits, perm, _ = rr.rr_reorder_and_trace(sc, to_dev(w.rays), p, flags=rr.RR_SORT_MSD)
            assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref["idx"]), kind
            assert_hits_match(rr.hits_to_numpy(hits), ref["hits"], ref["rays"], w.tris, str(kind))


def test_fused_call_msd_flag_checks(rr):
    """RR_SORT_MSD needs 64-bit keys and refuses the local sorts."""
    w = W.soup(seed=10, n_rays=4096, n_tris=256)
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
        rays = to_dev(w.rays)
        with pytest.raises(rr.RRError) as e:
            rr.rr_reorder_and_trace(sc, rays, rr.key_params(O.KIND_OD, 32, lo, hi, 0.25), flags=rr.RR_SORT_MSD)
        assert e.value.status == -4
        with pytest.raises(rr.RRError) as e:
            rr.rr_reorder_and_trace(sc, rays, rr.key_params(O.KIND_OD, 64, lo, hi, 0.25),
                                    flags=rr.RR_SORT_MSD | rr.RR_LOCAL_SORT_2048)
        assert e.value.status == -1
        # no sort, no effect
        h0, _, _ = rr.rr_reorder_and_trace(sc, rays, rr.key_params(O.KIND_NONE, 32, lo, hi), flags=rr.RR_SORT_MSD)
        h1 = rr.rr_trace(sc, rays)
        assert torch.equal(h0.view(torch.int32), h1.view(torch.int32))
