"""GPU parity of the block-wise (local) sort of Section 3.2 against the
oracle: permutation and keys bit for bit, alone and inside the fused call."""
import numpy as np
import pytest

import oracle as O

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


def rand_keys(n, bits, seed, dup):
    rng = np.random.default_rng(seed)
    if bits == 32:
        k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        k &= np.uint32(~((1 << dup) - 1) & 0xFFFFFFFF)
        k[::97] = 0xFFFFFFFF                      # real all-ones keys tie with the padding
    else:
        k = rng.integers(0, 1 << 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
        k &= ~np.uint64((1 << dup) - 1)
        k[::97] = np.uint64(0xFFFFFFFFFFFFFFFF)
    return k


@pytest.mark.parametrize("block", [1024, 2048, 4096])
@pytest.mark.parametrize("bits", [32, 64])
def test_local_sort_matches_oracle(rr, block, bits):
    for n, dup in ((1, 0), (1000, 20), (block, 0), (block + 1, 28), (5000, 0), (65553, 12), (300007, 0)):
        k = rand_keys(n, bits, n + block, dup)
        idx = (np.arange(n, dtype=np.uint32) * 2 + 5)     # ascending, not positions
        kd = to_dev(k.view(np.int32 if bits == 32 else np.int64))
        idd = to_dev(idx.view(np.int32))
        rr.rr_local_sort(kd, idd, block=block, key_bits=bits)
        ko, io = O.local_sort_pairs(k, idx, block)
        assert np.array_equal(kd.cpu().numpy().view(k.dtype), ko), (n, block, bits)
        assert np.array_equal(idd.cpu().numpy().view(np.uint32), io), (n, block, bits)


def test_local_sort_device_count_and_errors(rr):
    k = rand_keys(10000, 32, 3, 4)
    kd = to_dev(k.view(np.int32))
    idd = to_dev(np.arange(10000, dtype=np.int32))
    cnt = to_dev(np.array([6000], np.int32))
    rr.rr_local_sort(kd, idd, block=2048, count=cnt)
    ko, io = O.local_sort_pairs(k[:6000], block=2048)
    assert np.array_equal(kd.cpu().numpy().view(np.uint32)[:6000], ko)
    assert np.array_equal(idd.cpu().numpy().view(np.uint32)[:6000], io)
    assert np.array_equal(kd.cpu().numpy().view(np.uint32)[6000:], k[6000:])   # untouched past the count
    with pytest.raises(rr.RRError) as e:
        rr.rr_local_sort(kd, idd, block=512)
    assert e.value.status == -4


def test_fused_local_sort(rr, soup65k):
    w = soup65k
    lo, hi = O.scene_box(w.tris)
    bvh = O.BVH(w.tris)
    with rr.Scene(w.tris) as sc:
        rays = to_dev(w.rays)
        for kind, bits in ((O.KIND_OT, 32), (O.KIND_OD, 64), (O.KIND_AILA_COMPACT, 32)):
            p = rr.key_params(kind, bits, lo, hi)
            k = O.keys(w.rays, kind, bits, lo, hi)
            for flag, block in ((rr.RR_LOCAL_SORT_1024, 1024), (rr.RR_LOCAL_SORT_2048, 2048),
                                (rr.RR_LOCAL_SORT_4096, 4096)):
                _, want = O.local_sort_pairs(k, block=block)
                hits, perm, cnt = rr.rr_reorder_and_trace(sc, rays, p, flags=flag)
                assert np.array_equal(perm.cpu().numpy().view(np.uint32), want), (kind, bits, block)
                h = rr.hits_to_numpy(hits)
                assert h.tobytes() == bvh.trace(w.rays[want]).tobytes()
        with pytest.raises(rr.RRError) as e:
            rr.rr_reorder_and_trace(sc, rays, p, flags=rr.RR_LOCAL_SORT_1024 | rr.RR_LOCAL_SORT_2048)
        assert e.value.status == -1
