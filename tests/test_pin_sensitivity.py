"""Are the closest-hit pins strong enough?  Plausible mistakes are planted in
a small test-local copy of the Moller-Trumbore test (numpy, float64), and
each planted copy must fail at least one of the pin checks that the oracle's
own test passes (hand cases with closed-form answers; agreement with a
float64 linear solve of o + t d = v0 + u e1 + v e2).  The unplanted copy
passes them all, so each failure comes from its mistake."""
import numpy as np
import pytest

import oracle as O

MISTAKES = ["none", "det_sign", "cross_term_dropped", "u_v_swapped", "edges_swapped", "uv_bound_1_5",
            "one_sided", "origin_vector_reversed", "det_term_dropped"]


def mt_planted(ray, tri, mistake):
    o, d = ray[0:3].astype(np.float64), ray[4:7].astype(np.float64)
    v = tri.astype(np.float64).reshape(3, 3)
    e1, e2 = v[1] - v[0], v[2] - v[0]
    if mistake == "edges_swapped":
        e1, e2 = e2, e1
    p = np.cross(d, e2)
    if mistake == "cross_term_dropped":
        p[0] = d[1] * e2[2]
    det = e1 @ p
    if mistake == "det_term_dropped":
        det = e1[0] * p[0] + e1[1] * p[1]
    if det == 0 or (mistake == "one_sided" and det < 0):
        return False, 0.0, 0.0, 0.0
    inv = 1.0 / det
    if mistake == "det_sign":
        inv = -inv
    s = o - v[0] if mistake != "origin_vector_reversed" else v[0] - o
    u = (s @ p) * inv
    q = np.cross(s, e1)
    w = (d @ q) * inv
    bound = 1.5 if mistake == "uv_bound_1_5" else 1.0
    if u < 0 or w < 0 or u + w > bound:
        return False, 0.0, 0.0, 0.0
    t = (e2 @ q) * inv
    if mistake == "u_v_swapped":
        u, w = w, u
    return t > ray[3] and t < ray[7], t, u, w


def ray(o, d, tmin=0.0, tmax=np.inf):
    return np.array([*o, tmin, *d, tmax], np.float32)


def closed_form_ok(mt) -> bool:
    tri = np.array([0, 0, 0.5, 1, 0, 0.5, 0, 1, 0.5], np.float32)
    tri2 = tri.reshape(3, 3)[[0, 2, 1]].ravel()
    cases = [(ray((0.25, 0.25, 0), (0, 0, 1)), tri, (True, 0.5, 0.25, 0.25)),
             (ray((0.5, 0.125, 2), (0, 0, -1)), tri, (True, 1.5, 0.5, 0.125)),
             (ray((0.75, 0.5, 0), (0, 0, 1)), tri, (False,)),
             (ray((0.2, 0.2, 0.5), (1, 0, 0)), tri, (False,)),
             (ray((0.25, 0.125, 0), (0, 0, 1)), tri2, (True, 0.5, 0.125, 0.25))]
    for r, t, want in cases:
        got = mt(r, t)
        if bool(got[0]) != want[0]:
            return False
        if want[0] and not np.allclose(got[1:], want[1:], rtol=0, atol=1e-6):
            return False
    return True


def solve_ok(mt) -> bool:
    rng = np.random.default_rng(3)
    for _ in range(400):
        v = rng.uniform(-1, 1, (3, 3))
        o = rng.uniform(-2, 2, 3)
        d = v[0] + rng.uniform(-0.2, 1.2) * (v[1] - v[0]) + rng.uniform(-0.2, 1.2) * (v[2] - v[0]) - o
        d /= np.linalg.norm(d)
        r, tri = ray(o, d), v.astype(np.float32).ravel()
        tf = tri.astype(np.float64).reshape(3, 3)
        A = np.stack([-r[4:7].astype(np.float64), tf[1] - tf[0], tf[2] - tf[0]], axis=1)
        if abs(np.linalg.det(A)) < 1e-3:
            continue
        t, uu, vv = np.linalg.solve(A, r[0:3].astype(np.float64) - tf[0])
        margin = min(uu, vv, 1 - uu - vv)
        if abs(margin) < 1e-4:
            continue
        hit, t2, u2, v2 = mt(r, tri)
        if bool(hit) != bool(margin > 0 and t > 0):
            return False
        if hit and (abs(t2 - t) > 1e-4 * max(1.0, abs(t)) or abs(u2 - uu) > 1e-4 or abs(v2 - vv) > 1e-4):
            return False
    return True


def test_the_oracle_passes_the_pins():
    assert closed_form_ok(O.mt) and solve_ok(O.mt)


@pytest.mark.parametrize("mistake", MISTAKES)
def test_each_planted_mistake_fails_a_pin(mistake):
    def mt(r, t):
        return mt_planted(r, t, mistake)
    passes = closed_form_ok(mt) and solve_ok(mt)
    assert passes == (mistake == "none"), mistake


# ------------------------------------------------------------------ sort
# The same for the sort pins: plausible mistakes in a (key, index) pair sort
# (numpy, test-local) must fail the checks the oracle's sort passes (Python's
# sorted() on tuples for 32-bit keys; order, permutation, stability and key
# consistency for 64-bit keys with the top bit in use).

SORT_MISTAKES = ["none", "unstable", "descending", "index_first", "signed_view", "low_32_bits_only",
                 "index_not_moved"]


def sort_planted(k, idx, mistake):
    k = np.asarray(k)
    idx = np.arange(k.shape[0], dtype=np.uint32) if idx is None else np.asarray(idx, np.uint32)
    if mistake == "unstable":
        order = np.argsort(k, kind="quicksort")[::-1]
        order = order[np.argsort(k[order], kind="stable")]  # equal keys in reversed input order
    elif mistake == "descending":
        order = np.lexsort((idx, k))[::-1]
    elif mistake == "index_first":
        order = np.lexsort((k, idx))
    elif mistake == "signed_view":
        order = np.lexsort((idx, k.view(np.int64 if k.dtype == np.uint64 else np.int32)))
    elif mistake == "low_32_bits_only":
        order = np.lexsort((idx, k & np.array(0xFFFFFFFF, k.dtype)))
    else:
        order = np.lexsort((idx, k))
    if mistake == "index_not_moved":
        return k[order], idx
    return k[order], idx[order]


def sort_pins_ok(sort_pairs) -> bool:
    rng = np.random.default_rng(0)
    for n, hi in ((7, 3), (300, 16), (1000, 1 << 32)):
        k = rng.integers(0, hi, n, dtype=np.uint64).astype(np.uint32)
        idx = np.arange(n, dtype=np.uint32)
        ks, ix = sort_pairs(k, idx)
        ref = sorted(zip(k.tolist(), idx.tolist()))
        if ks.tolist() != [a for a, _ in ref] or ix.tolist() != [b for _, b in ref]:
            return False
    n = 20000
    k = rng.integers(0, 1 << 12, n, dtype=np.uint64) << np.uint64(52)  # top bit used, many equal keys
    ks, ix = sort_pairs(k, None)
    eq = ks[1:] == ks[:-1]
    return bool(np.all(ks[1:] >= ks[:-1]) and np.array_equal(np.sort(ix), np.arange(n, dtype=np.uint32))
                and np.all(ix[1:][eq] > ix[:-1][eq]) and np.array_equal(k[ix], ks))


def test_the_oracle_sort_passes_the_pins():
    assert sort_pins_ok(O.sort_pairs)


@pytest.mark.parametrize("mistake", SORT_MISTAKES)
def test_each_planted_sort_mistake_fails_a_pin(mistake):
    assert sort_pins_ok(lambda k, i: sort_planted(k, i, mistake)) == (mistake == "none"), mistake
