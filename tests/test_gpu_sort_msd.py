"""GPU parity of the most-significant-digit sort that rr_sort and the fused
call use for 64-bit keys from 1,572,864 up to 2^27 keys (the sizes here are
in that range unless stated): two stable scatter passes on the two highest
digits in which the keys differ, then every bucket of equal top digits
sorted on its other digits in LDS, or, when it holds more keys than fit, by
one block in chunks through global memory.  Its result must be the stable
order of the oracle (Section 3.2), and the LSD sort's (rr_sort_ex) bit for
bit, whatever the key distribution: buckets that straddle the kernel's
windows, buckets too large for LDS with an odd or even number of differing
digits below the top two, keys differing in one digit only, input indices
that do not ascend, a device count below the capacity."""
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


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def keys_np(t, bits):
    a = t.cpu().numpy()
    return a.view(np.uint32) if bits == 32 else a.view(np.uint64)


def run_both(rr, k, bits, idx_in=None, count=None):
    """rr_sort (most-significant-digit sort) and rr_sort_ex (LSD) of the same
    pairs; both must give the oracle's stable order by input position."""
    n = k.shape[0]
    idx_in = np.arange(n, dtype=np.uint32) if idx_in is None else idx_in
    m = n if count is None else count
    _, perm = O.sort_pairs(k[:m])
    outs = []
    for ex in (None, 8):
        kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
        idx = to_dev(idx_in.view(np.int32))
        cnt = None if count is None else torch.tensor([count], dtype=torch.int32, device=DEV)
        rr.rr_sort(kd, idx, count=cnt, keys_per_thread=ex)
        gk, gi = keys_np(kd, bits), idx.cpu().numpy().view(np.uint32)
        assert np.array_equal(gk[:m], k[:m][perm]), ("keys", ex)
        assert np.array_equal(gi[:m], idx_in[:m][perm]), ("idx", ex)
        assert np.array_equal(gk[m:], k[m:]) and np.array_equal(gi[m:], idx_in[m:]), ("tail", ex)
        outs.append(gi.copy())
    assert np.array_equal(outs[0], outs[1])


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


@pytest.mark.parametrize("bits,low_bits", [(64, 24), (64, 16), (64, 40), (32, 16)])
def test_buckets_larger_than_a_batch(rr, bits, low_bits):
    """One bucket of ~960K keys (an odd and an even number of differing
    digits below the top two), with reversed input indices (32-bit keys: the
    LSD sort on the same pattern)."""
    n = 1_600_007
    k = big_bucket_keys(n, bits, low_bits, 0.6, 7 + low_bits)
    run_both(rr, k, bits, idx_in=np.arange(n, dtype=np.uint32)[::-1].copy())


@pytest.mark.parametrize("bits", [32, 64])
def test_bucket_sizes_around_the_batch(rr, bits):
    """Buckets of 1 to ~12K keys (sizes spread over the whole range, some
    just above and below a batch of 8192 and straddling the kernel's 8192-key
    windows), keys differing in every digit inside a bucket, shuffled input
    indices."""
    rng = np.random.default_rng(bits)
    sizes = np.concatenate([rng.integers(1, 12000, 280), [8191, 8192, 8193, 1, 2, 4095, 4097]])
    rng.shuffle(sizes)
    n = int(sizes.sum())
    prefixes = np.sort(rng.choice(1 << 16, sizes.shape[0], replace=False)).astype(np.uint64)
    sh = np.uint64(bits - 16)
    k = np.repeat(prefixes << sh, sizes)
    k |= rng.integers(0, 1 << (bits - 16), n, dtype=np.uint64)
    k = k[rng.permutation(n)].astype(np.uint32 if bits == 32 else np.uint64)
    run_both(rr, k, bits, idx_in=rng.permutation(n).astype(np.uint32))


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("n", [1, 2, 3, 100, 8193, 65537, (3 << 19) - 1, 3 << 19, (3 << 19) + 8191, (1 << 21) + 1])
def test_sizes_around_the_windows_and_the_threshold(rr, bits, n):
    """Sizes on both sides of the size from which 64-bit keys take the MSD
    sort, and ragged against its 8,192-key windows."""
    rng = np.random.default_rng(n + bits)
    k = rng.integers(0, (1 << bits) - 1, n, dtype=np.uint64, endpoint=True)
    k = (k >> np.uint64(rng.integers(0, bits - 1))).astype(np.uint32 if bits == 32 else np.uint64)
    run_both(rr, k, bits)


@pytest.mark.parametrize("bits", [32, 64])
@pytest.mark.parametrize("digit", [0, 1, 3])
def test_one_or_two_differing_digits(rr, bits, digit):
    """Keys that differ in one digit only, or in that digit and the top one:
    the two scatter passes alone order them."""
    n = 1_600_003
    rng = np.random.default_rng(digit * 3 + bits)
    base = np.uint64(0x0123456789ABCDEF & ((1 << bits) - 1))
    d = rng.integers(0, 256, n, dtype=np.uint64)
    k1 = (base & ~np.uint64(255 << (8 * digit))) | (d << np.uint64(8 * digit))
    run_both(rr, k1.astype(np.uint32 if bits == 32 else np.uint64), bits)
    top = rng.integers(0, 4, n, dtype=np.uint64) << np.uint64(bits - 8)
    k2 = (k1 & np.uint64((1 << (bits - 8)) - 1)) | top
    run_both(rr, k2.astype(np.uint32 if bits == 32 else np.uint64), bits)


def test_device_count_and_big_bucket(rr):
    n_max, n = 1_700_000, 1_600_001
    k = big_bucket_keys(n_max, 64, 20, 0.5, 3)
    run_both(rr, k, 64, count=n)
    run_both(rr, k, 64, count=0)


def test_fused_call_with_a_bucket_larger_than_a_batch(rr):
    """Half the rays start at one point (origin-direction keys then share
    their origin bits, so one bucket holds them all and the sort's large-
    bucket path also gathers the rays): the fused call's permutation equals
    the oracle's and its hits match under the closest-hit rule."""
    w = W.soup(seed=9, n_rays=1_600_000, n_tris=2048)
    rays = w.rays.copy()
    rays[::2, 0:3] = np.array([0.31, 0.62, 0.47], np.float32)
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        lo, hi = sc.bounds()
        for kind, bits in ((O.KIND_OD, 32), (O.KIND_OD, 64), (O.KIND_OT, 64)):
            p = rr.key_params(kind, bits, lo, hi, 0.25)
            hits, perm, _ = rr.rr_reorder_and_trace(sc, to_dev(rays), p, flags=0)
            ref = O.reorder_and_trace(bvh, rays, kind, bits, lo, hi, 0.25)
            assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref["idx"]), (kind, bits)
            assert_hits_match(rr.hits_to_numpy(hits), ref["hits"], ref["rays"], w.tris, f"{kind}/{bits}")
