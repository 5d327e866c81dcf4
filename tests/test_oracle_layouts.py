"""Pins for the oracle's other key layouts (Figure "codes": Origin, Costa,
Aila, Aila Compact, Octahedron) and for the Two Point termination estimates
of Section 3.1.6 (adaptive length table, real termination point).

Pins: hand-worked keys (tests/golden/keys_worked_layouts.txt); the figure's
rows transcribed; identities between layouts (Origin is origin-direction
with all 32 slots on the origin, Costa is the 24/8 origin-direction key
rotated, the length-table cell is the top of the Aila Compact key); the
octahedral map against its inverse and its special directions; the table's
mean against closed forms and its independence of accumulation order.
"""
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
BOX = (np.zeros(3, np.float32), np.ones(3, np.float32))
KINDS = {"ORIG": O.KIND_ORIGIN, "COSTA": O.KIND_COSTA, "AILA": O.KIND_AILA, "AILAC": O.KIND_AILA_COMPACT,
         "OCTA": O.KIND_OCTAHEDRON, "CELL": None}


def ray(o, d, tmax=np.inf):
    return np.array([*o, 0.0, *d, tmax], np.float32)


def golden():
    rows = []
    with open(os.path.join(HERE, "golden", "keys_worked_layouts.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                p = line.split()
                rows.append((p[0], p[1], [float(x) for x in p[2:5]], [float(x) for x in p[5:8]], int(p[8], 16)))
    return rows


@pytest.mark.parametrize("row", golden(), ids=lambda r: r[0])
def test_worked_values(row):
    name, kind, o, d, expected = row
    if kind == "CELL":
        got = int(O.cell_code(ray(o, d)[None], *BOX)[0])
    else:
        got = int(O.keys(ray(o, d)[None], KINDS[kind], 32, *BOX)[0])
    assert got == expected, f"{name}: {got:#x} != {expected:#x}"


# Figure "codes", the owner of each bit, MSB first (z = a zero bit, q = an
# octahedral direction bit).
FIGURE = {
    O.KIND_ORIGIN: "o" * 32,
    O.KIND_COSTA: "d" * 8 + "o" * 24,
    O.KIND_AILA: ("ooo" + "zzz") * 3 + ("ooo" + "ddd") * 2 + "oo",
    O.KIND_AILA_COMPACT: "o" * 12 + ("ddd" + "ooo") * 3 + "dd",
    O.KIND_OCTAHEDRON: "o" * 15 + ("qq" + "ooo") * 3 + "qq",
}
CH = {-1: "z", 0: "o", 1: "d", 2: "t", 3: "q"}


@pytest.mark.parametrize("kind", list(FIGURE))
def test_layouts_match_figure(kind):
    src, comp = O.key_layout(kind, 32)
    assert "".join(CH[int(s)] for s in src) == FIGURE[kind]
    # within a run, components cycle x, y, z (u, v for the octahedral bits)
    runs = []
    for s, c in zip(src, comp):
        if runs and runs[-1][0] == int(s):
            runs[-1][1].append(int(c))
        else:
            runs.append((int(s), [int(c)]))
    for s, cs in runs:
        period = 2 if s == 3 else 3
        if s != -1:
            assert cs == [i % period for i in range(len(cs))]


def test_other_layouts_are_32_bit_only():
    for kind in FIGURE:
        with pytest.raises(ValueError):
            O.keys(ray((0.5,) * 3, (0, 0, 1))[None], kind, 64, *BOX)


def _random_rays(n, seed=11):
    rng = np.random.default_rng(seed)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = rng.uniform(-0.2, 1.2, (n, 3))
    d = rng.normal(size=(n, 3))
    r[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r[:, 7] = np.where(rng.uniform(size=n) < 0.2, rng.uniform(0, 0.5, n), np.inf)
    # exact axis directions and box faces
    r[:8, 4:7] = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1], [0, 0, 1], [0, 0, -1]]
    r[8:12, 0:3] = [[0, 0, 0], [1, 1, 1], [0, 1, 0], [1, 0, 1]]
    return r


def test_origin_is_origin_direction_with_32_origin_slots():
    r = _random_rays(20000)
    assert np.array_equal(O.keys(r, O.KIND_ORIGIN, 32, *BOX), O.keys(r, O.KIND_OD, 32, *BOX, origin_bits=32))


def test_costa_is_rotated_origin_direction():
    # Costa (d8 o24) is the origin-direction key with 24 origin slots (o24 d8)
    # rotated by 8 bits
    r = _random_rays(20000)
    od = O.keys(r, O.KIND_OD, 32, *BOX, origin_bits=24).astype(np.uint64)
    costa = O.keys(r, O.KIND_COSTA, 32, *BOX).astype(np.uint64)
    assert np.array_equal(costa, ((od & np.uint64(0xFF)) << np.uint64(24)) | (od >> np.uint64(8)))


def test_aila_zero_slots_and_fields():
    r = _random_rays(20000)
    k = O.keys(r, O.KIND_AILA, 32, *BOX).astype(np.uint64)
    src, _ = O.key_layout(O.KIND_AILA, 32)
    zmask = sum(1 << (31 - i) for i, s in enumerate(src) if s == -1)
    assert not np.any(k & np.uint64(zmask))
    # its origin bits are those of the Origin layout's 6/6/5-bit quantisation:
    # the 17 origin slots read back give the top bits of the 11/11/10 origin key
    orig = O.keys(r, O.KIND_ORIGIN, 32, *BOX).astype(np.uint64)
    opos = [31 - i for i, s in enumerate(src) if s == 0]
    got = np.zeros_like(k)
    for j, p in enumerate(opos):
        got |= ((k >> np.uint64(p)) & np.uint64(1)) << np.uint64(16 - j)
    assert np.array_equal(got, orig >> np.uint64(15))


def test_cell_code_is_top_of_aila_compact():
    r = _random_rays(20000)
    ac = O.keys(r, O.KIND_AILA_COMPACT, 32, *BOX)
    assert np.array_equal(O.cell_code(r, *BOX), ac >> np.uint32(12))


def test_octahedral_special_directions():
    d = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0.6, 0, -0.8]], np.float32)
    uv = O.octahedral(d)
    np.testing.assert_array_equal(uv[:6], [[0, 0], [1, 1], [1, 0], [-1, 0], [0, 1], [0, -1]])
    # folded lower half: (1 - |py|) sign(px), (1 - |px|) sign(py) with px = 0.6 / 1.4, py = 0
    assert uv[6, 0] == 1.0 and abs(uv[6, 1] - (1 - 0.6 / 1.4)) < 1e-6


def test_octahedral_inverse_and_hemispheres():
    rng = np.random.default_rng(2)
    d = rng.normal(size=(3000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    uv = O.octahedral(d.astype(np.float32)).astype(np.float64)
    u, v = uv[:, 0], uv[:, 1]
    a = np.abs(u) + np.abs(v)
    assert np.all(a[d[:, 2] > 1e-6] <= 1 + 1e-6) and np.all(a[d[:, 2] < -1e-6] >= 1 - 1e-6)
    # decode: z = 1 - |u| - |v|; below the equator unfold the diagonals
    z = 1 - a
    x = np.where(z < 0, (1 - np.abs(v)) * np.where(u >= 0, 1, -1), u)
    y = np.where(z < 0, (1 - np.abs(u)) * np.where(v >= 0, 1, -1), v)
    back = np.stack([x, y, z], 1)
    back /= np.linalg.norm(back, axis=1, keepdims=True)
    assert np.max(np.abs(back - d)) < 1e-5


# ------------------------------------------------------ termination estimates

def test_real_termination_equals_fixed_length_of_the_same_distance():
    # Two Point Real with every hit at distance 0.125 = the fixed estimate
    # with ratio 0.125 in the unit box; a miss falls back to the fixed estimate
    r = _random_rays(5000)
    r[:, 7] = np.inf
    hits = np.zeros(r.shape[0], O.HIT_DTYPE)
    hits["t"] = 0.125
    hits["prim"] = 3
    hits["prim"][::7] = -1
    hits["t"][::7] = np.inf
    for bits in (32, 64):
        real = O.keys(r, O.KIND_TP_REAL, bits, *BOX, ratio=0.125, aux=hits)
        fixed = O.keys(r, O.KIND_OT, bits, *BOX, ratio=0.125)
        assert np.array_equal(real, fixed)
    # and a real distance differing from the fixed one moves the key
    hits["t"] = 0.6
    assert np.mean(O.keys(r, O.KIND_TP_REAL, 32, *BOX, aux=hits) != O.keys(r, O.KIND_OT, 32, *BOX)) > 0.5


@pytest.mark.parametrize("ratio", [0.25, 0.125, 0.375])
def test_fresh_length_table_gives_the_fixed_estimate(ratio):
    lo = np.array([-3, 0, 2], np.float32)
    hi = np.array([7, 4, 5], np.float32)
    r = _random_rays(5000)
    r[:, 0:3] = r[:, 0:3] * (hi - lo) + lo
    t = O.LengthTable(lo, hi, ratio)
    # each cell holds one dummy ray of length ratio x 10 (the largest extent)
    assert np.all(t.cells["count"] == 1)
    est = t.lookup(r[:200])
    assert np.all(est == np.float32(np.float32(ratio) * np.float32(10)))
    for bits in (32, 64):
        assert np.array_equal(O.keys(r, O.KIND_TP_ADAPTIVE, bits, lo, hi, ratio=ratio, aux=t),
                              O.keys(r, O.KIND_OT, bits, lo, hi, ratio=ratio))


def test_non_dyadic_dummy_truncates_to_a_unit():
    # the dummy length is held in units of E / 2^24: ratio 0.1 loses less than one unit
    lo, hi = BOX
    t = O.LengthTable(lo, hi, 0.1)
    est = float(t.lookup(_random_rays(16)[:1])[0])
    assert 0.1 - 2.0 ** -24 < est <= 0.1


def test_length_table_mean_and_order_independence():
    lo, hi = BOX
    rng = np.random.default_rng(4)
    r = _random_rays(6000)
    # three cells' worth of rays: copy three rays many times
    picks = r[[20, 40, 60]]
    rays = np.repeat(picks, [5, 9, 1], axis=0)
    hits = np.zeros(rays.shape[0], O.HIT_DTYPE)
    # lengths that are whole units of E / 2^24: sums are exact
    units = rng.integers(1, 1 << 24, rays.shape[0])
    hits["t"] = (units / float(1 << 24)).astype(np.float32)
    hits["prim"] = 1
    t1 = O.LengthTable(lo, hi)
    t1.accumulate(rays, hits)
    perm = rng.permutation(rays.shape[0])
    t2 = O.LengthTable(lo, hi)
    t2.accumulate(rays[perm[:7]], hits[perm[:7]])
    t2.accumulate(rays[perm[7:]], hits[perm[7:]])
    assert t1.cells.tobytes() == t2.cells.tobytes()
    cells = O.cell_code(picks, lo, hi)
    for j, c in enumerate(cells):
        sel = np.all(rays == picks[j], axis=1)
        lens = [0.25] + list(hits["t"][sel].astype(np.float64))
        want = np.float32(np.mean(lens))     # the mean of the dummy and the traced lengths
        got = t1.lookup(picks[j][None])[0]
        assert t1.cells["count"][c] == len(lens)
        assert got == want, (got, want)


def test_length_table_ignores_misses_and_truncates_to_units():
    lo, hi = BOX
    r = _random_rays(16)[:2]
    t = O.LengthTable(lo, hi)
    before = t.cells.copy()
    miss = np.zeros(2, O.HIT_DTYPE)
    miss["t"] = np.inf
    miss["prim"] = -1
    t.accumulate(r, miss)
    assert t.cells.tobytes() == before.tobytes()
    h = np.zeros(1, O.HIT_DTYPE)
    h["t"] = np.float32((1000 + 0.75) / float(1 << 24))  # 1000.75 units -> 1000
    h["prim"] = 0
    t.accumulate(r[:1], h)
    c = O.cell_code(r[:1], lo, hi)[0]
    assert int(t.cells["sum"][c]) == (1 << 22) + 1000 and t.cells["count"][c] == 2
