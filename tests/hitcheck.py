"""The hit-parity rule shared by the GPU tests (BASELINE tolerance for
closest hits): the primitive must match exactly, t, u and v bit for bit when
it does; a differing primitive is accepted only as a near-tie, where the
oracle's own test of the GPU's primitive passes with t within 1e-5 relative
of the oracle's t (and the GPU's t is within 1e-5 relative too).  A hit
against a miss is always a failure."""
import numpy as np

import oracle as O


def assert_hits_match(gpu, ref, rays, tris, what="", max_ties=None):
    same = gpu["prim"] == ref["prim"]
    bad = np.nonzero(~same)[0]
    for i in bad[:1000]:
        gp, op = int(gpu["prim"][i]), int(ref["prim"][i])
        assert gp >= 0 and op >= 0, f"{what}: hit/miss mismatch at ray {i}: gpu {gp} oracle {op}"
        ok, t, _, _ = O.mt(rays[i], tris[gp])
        assert ok and abs(t - ref["t"][i]) <= 1e-5 * abs(ref["t"][i]), f"{what}: ray {i}"
        assert abs(gpu["t"][i] - ref["t"][i]) <= 1e-5 * abs(ref["t"][i]), f"{what}: ray {i}"
    limit = max(2, len(ref) // 10000) if max_ties is None else max_ties
    assert len(bad) <= limit, f"{what}: {len(bad)} near-tie differences"
    m = same
    assert np.array_equal(gpu["t"][m].view(np.uint32), ref["t"][m].view(np.uint32)), what
    assert np.array_equal(gpu["u"][m].view(np.uint32), ref["u"][m].view(np.uint32)), what
    assert np.array_equal(gpu["v"][m].view(np.uint32), ref["v"][m].view(np.uint32)), what
    return int(len(bad))
