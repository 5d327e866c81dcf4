"""GPU checks at the largest sizes: the sort at the largest pair count a call
accepts (2^30 - 1, the tile status words' 30-bit counts) and the fused call
on 134M rays.  The oracle cannot sort a billion pairs in a test's time, so the
result is checked through properties that together define the stable sort:
output keys ascend, the index output is a permutation of the input
positions, each output key is the input key at its index, and equal keys keep
ascending indices."""
import sys

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


def assert_stable_sort(keys_in, keys, idx):
    """keys_in: the input keys (int64 holding uint64 bits); keys / idx: the
    sort's outputs for identity input indices."""
    n = keys.shape[0]
    flip = torch.tensor(-(1 << 63), dtype=torch.int64, device=DEV)
    u = torch.bitwise_xor(keys, flip)  # unsigned order as signed order
    assert bool((u[1:] >= u[:-1]).all()), "keys do not ascend"
    del u
    il = idx.long()
    assert bool(((il >= 0) & (il < n)).all()), "index out of range"
    seen = torch.zeros(n, dtype=torch.bool, device=DEV)
    seen[il] = True
    assert bool(seen.all()), "indices are not a permutation"
    del seen
    assert bool((keys_in.index_select(0, il) == keys).all()), "output key is not the input key at its index"
    del il
    eq = keys[1:] == keys[:-1]
    assert bool(((idx[1:] > idx[:-1]) | ~eq).all()), "equal keys out of input order"


def test_sort_at_the_largest_accepted_count(rr):
    n = (1 << 30) - 1
    print(f"sort n={n} 64-bit", flush=True)
    g = torch.Generator(device=DEV)
    g.manual_seed(30)
    # 2^24 distinct values over the whole unsigned range (top 24 bits, low 40
    # zero): every digit pass meets many equal keys
    v = torch.randint(0, 1 << 24, (n,), dtype=torch.int64, device=DEV, generator=g)
    keys = (v - (1 << 23)) * (1 << 40)
    del v
    keys_in = keys.clone()
    idx = torch.arange(n, dtype=torch.int32, device=DEV)
    rr.rr_sort(keys, idx)
    torch.cuda.synchronize()
    assert_stable_sort(keys_in, keys, idx)


def test_fused_call_on_134m_rays(rr):
    """The 1080p bounce-2 wavefront repeated 64.7 times (2^27 + 5 rays, so
    every key occurs in many copies): keys against the oracle's keys of the
    wavefront, the permutation through the sort properties, hits scattered
    back against the unsorted trace, and 2,048 sorted hits against the
    oracle's trace."""
    w = W.bounce2_1080p()
    B = w.rays.shape[0]
    N = (1 << 27) + 5
    print(f"fused call N={N}", flush=True)
    base = torch.from_numpy(w.rays).to(DEV)
    rays = base.repeat((N + B - 1) // B, 1)[:N].contiguous()
    with rr.Scene(w.tris) as scene:
        lo, hi = scene.bounds()
        p = rr.key_params(O.KIND_OT, 64, lo, hi, 0.25)
        want_base = torch.from_numpy(O.keys(w.rays, O.KIND_OT, 64, lo, hi, 0.25).view(np.int64)).to(DEV)
        k, _, _ = rr.rr_compute_keys(rays, p)
        want = want_base.repeat((N + B - 1) // B)[:N]
        assert bool((k == want).all())
        hits, perm, cnt = rr.rr_reorder_and_trace(scene, rays, p, flags=0)
        torch.cuda.synchronize()
        assert int(cnt.cpu()[0]) == N
        assert_stable_sort(want, want.index_select(0, perm.long()), perm)
        del k
        plain = rr.rr_trace(scene, rays)
        back = torch.empty_like(plain)
        back[perm.long()] = hits
        assert bool((back.view(torch.int32) == plain.view(torch.int32)).all())
        s = np.random.default_rng(27).choice(N, 2048, replace=False)
        sd = torch.from_numpy(s).to(DEV)
        got = rr.hits_to_numpy(hits.index_select(0, sd))
        src = perm.index_select(0, sd).cpu().numpy().view(np.uint32) % B
        assert got.tobytes() == O.BVH(w.tris).trace(w.rays[src]).tobytes()
