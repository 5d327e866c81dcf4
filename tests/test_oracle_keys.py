"""Pins for the oracle's sort keys (Section 3.1, Figure "codes").

The paper prints no key values, so the oracle is pinned by
  * hand-worked keys (tests/golden/keys_worked.txt),
  * the bit layouts transcribed from the figure (which vector owns each bit),
  * single-bit moves: raising one quantised coordinate by its least (or most)
    significant unit flips exactly the bit the layout assigns to it,
  * prefix invariants between the 32- and 64-bit layouts,
  * quantiser edge cases.
"""
import os

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
BOX = (np.zeros(3, np.float32), np.ones(3, np.float32))


def ray(o, d, tmax=np.inf):
    return np.array([*o, 0.0, *d, tmax], np.float32)


def load_golden():
    rows = []
    with open(os.path.join(HERE, "golden", "keys_worked.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            p = line.split()
            rows.append((p[0], {"OD": O.KIND_OD, "OT": O.KIND_OT}[p[1]], int(p[2]),
                         [float(x) for x in p[3:6]], [float(x) for x in p[6:9]], float(p[9]), int(p[10], 16)))
    return rows


@pytest.mark.parametrize("row", load_golden(), ids=lambda r: r[0])
def test_worked_values(row):
    name, kind, bits, o, d, ratio, expected = row
    got = int(O.keys(ray(o, d)[None], kind, bits, *BOX, ratio=ratio)[0])
    assert got == expected, f"{name}: {got:#x} != {expected:#x}"


# Figure "codes": the owner of each of the 32 bits, MSB first.
FIGURE_ROWS = {
    (O.KIND_OD, 32): "o" * 22 + "d" * 10,              # Reis
    (O.KIND_OT, 32): ("ooo" + "ttt") * 5 + "oo",       # Two Point
}
SRC_CHAR = {0: "o", 1: "d", 2: "t"}


@pytest.mark.parametrize("kind_bits", list(FIGURE_ROWS))
def test_layout_matches_figure(kind_bits):
    kind, bits = kind_bits
    src, comp = O.key_layout(kind, bits)
    assert "".join(SRC_CHAR[int(s)] for s in src) == FIGURE_ROWS[kind_bits]
    # consecutive triples run x, y, z: within each vector, components cycle
    for v in (0, 1, 2):
        c = [int(x) for x, s in zip(comp, src) if s == v]
        assert c == [i % 3 for i in range(len(c))]


def test_64bit_layouts_extend_32bit():
    src, comp = O.key_layout(O.KIND_OD, 64)
    assert "".join(SRC_CHAR[int(s)] for s in src) == "o" * 44 + "d" * 20
    src, comp = O.key_layout(O.KIND_OT, 64)
    assert "".join(SRC_CHAR[int(s)] for s in src) == ("ooottt" * 11)[:64]


def _bits_per_component(kind, bits):
    src, comp = O.key_layout(kind, bits)
    out = {}
    for pos, (s, c) in enumerate(zip(src, comp)):
        out.setdefault((int(s), int(c)), []).append(bits - 1 - pos)  # bit index, MSB first
    return out


def _origin_for(q, b):
    """A coordinate in [0,1] that quantises to q with b bits."""
    return (q + 0.5) / (1 << b)


@pytest.mark.parametrize("kind,bits", [(O.KIND_OD, 32), (O.KIND_OD, 64), (O.KIND_OT, 32), (O.KIND_OT, 64)])
def test_single_bit_moves_origin(kind, bits):
    owners = _bits_per_component(kind, bits)
    d = (0.0, 0.0, 1.0)
    for comp in range(3):
        positions = owners[(0, comp)]
        b = len(positions)
        for which, pos in (("lsb", positions[-1]), ("msb", positions[0])):
            q0 = 0 if which == "lsb" else 0
            q1 = 1 if which == "lsb" else (1 << (b - 1))
            base = [0.5 / (1 << 20)] * 3
            o0 = list(base)
            o1 = list(base)
            o0[comp] = _origin_for(q0, b)
            o1[comp] = _origin_for(q1, b)
            # ratio 0: the termination point sits on the origin, so for Two
            # Point keys its bits move too; isolate the origin with ratio 0
            # and compare against the t-slot positions as well.
            k0 = int(O.keys(ray(o0, d)[None], kind, bits, *BOX, ratio=0.0)[0])
            k1 = int(O.keys(ray(o1, d)[None], kind, bits, *BOX, ratio=0.0)[0])
            flipped = k0 ^ k1
            expect = 1 << pos
            if kind == O.KIND_OT:
                tpos = owners[(2, comp)]
                bt = len(tpos)
                # the termination coordinate is the same value quantised with bt bits
                qt0 = int(min(np.floor(_origin_for(q0, b) * (1 << bt)), (1 << bt) - 1))
                qt1 = int(min(np.floor(_origin_for(q1, b) * (1 << bt)), (1 << bt) - 1))
                for i in range(bt):
                    if ((qt0 ^ qt1) >> (bt - 1 - i)) & 1:
                        expect |= 1 << tpos[i]
            assert flipped == expect, (kind, bits, comp, which, hex(flipped), hex(expect))


@pytest.mark.parametrize("bits", [32, 64])
def test_single_bit_moves_direction(bits):
    owners = _bits_per_component(O.KIND_OD, bits)
    o = (0.3, 0.3, 0.3)
    for comp in range(3):
        positions = owners[(1, comp)]
        b = len(positions)
        # direction component d quantises u = (d + 1) / 2; pick u on cell centres
        def dval(q):
            return 2.0 * (q + 0.5) / (1 << b) - 1.0
        for q0, q1, pos in ((0, 1, positions[-1]), (0, 1 << (b - 1), positions[0])):
            d0 = [dval(0)] * 3
            d1 = list(d0)
            d1[comp] = dval(q1)
            d0[comp] = dval(q0)
            k0 = int(O.keys(ray(o, d0)[None], O.KIND_OD, bits, *BOX)[0])
            k1 = int(O.keys(ray(o, d1)[None], O.KIND_OD, bits, *BOX)[0])
            assert k0 ^ k1 == 1 << pos


def test_termination_bits_follow_direction_and_length():
    # Two Point: only the t-slots move when the direction changes
    owners = _bits_per_component(O.KIND_OT, 32)
    tmask = 0
    for c in range(3):
        for p in owners[(2, c)]:
            tmask |= 1 << p
    rng = np.random.default_rng(5)
    for _ in range(200):
        o = rng.uniform(0.1, 0.9, 3)
        d1 = rng.normal(size=3); d1 /= np.linalg.norm(d1)
        d2 = rng.normal(size=3); d2 /= np.linalg.norm(d2)
        k1 = int(O.keys(ray(o, d1)[None], O.KIND_OT, 32, *BOX)[0])
        k2 = int(O.keys(ray(o, d2)[None], O.KIND_OT, 32, *BOX)[0])
        assert (k1 ^ k2) & ~tmask == 0


def _random_rays(n, seed=3):
    rng = np.random.default_rng(seed)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = rng.uniform(-0.2, 1.2, (n, 3))
    d = rng.normal(size=(n, 3))
    r[:, 4:7] = d / np.linalg.norm(d, axis=1, keepdims=True)
    r[:, 7] = np.where(rng.uniform(size=n) < 0.2, rng.uniform(0, 0.5, n), np.inf)
    return r


def test_prefix_invariant_two_point():
    # I1: the 64-bit Two Point key starts with the 32-bit one
    r = _random_rays(20000)
    k32 = O.keys(r, O.KIND_OT, 32, *BOX)
    k64 = O.keys(r, O.KIND_OT, 64, *BOX)
    assert np.array_equal((k64 >> np.uint64(32)).astype(np.uint32), k32)


def test_prefix_invariant_origin_direction():
    # I2: the 64-bit origin field starts with the 32-bit origin field, and
    # likewise the direction field
    r = _random_rays(20000)
    k32 = O.keys(r, O.KIND_OD, 32, *BOX).astype(np.uint64)
    k64 = O.keys(r, O.KIND_OD, 64, *BOX)
    assert np.array_equal(k64 >> np.uint64(42), k32 >> np.uint64(10))
    assert np.array_equal((k64 >> np.uint64(10)) & np.uint64(0x3FF), k32 & np.uint64(0x3FF))


def test_ratio_zero_is_origin_only():
    # I3: with ratio 0 the Two Point key does not depend on the direction
    r = _random_rays(5000)
    r2 = r.copy()
    r2[:, 4:7] = -r2[:, 4:7]
    for bits in (32, 64):
        assert np.array_equal(O.keys(r, O.KIND_OT, bits, *BOX, ratio=0.0),
                              O.keys(r2, O.KIND_OT, bits, *BOX, ratio=0.0))


def test_finite_tmax_shortens_estimate():
    # the estimate never runs past tmax: a ray with tmax 0 has t = o
    o = (0.3, 0.6, 0.2)
    a = O.keys(ray(o, (1, 0, 0), tmax=0.0)[None], O.KIND_OT, 32, *BOX)[0]
    b = O.keys(ray(o, (0, 1, 0), tmax=np.inf)[None], O.KIND_OT, 32, *BOX, ratio=0.0)[0]
    assert a == b


def test_quantiser_edges():
    lo, hi = BOX
    # below / above the box clamp to 0 / all ones; NaN maps to 0
    below = O.keys(ray((-5, -5, -5), (-1, -1, -1))[None], O.KIND_OD, 32, lo, hi)[0]
    above = O.keys(ray((5, 5, 5), (1, 1, 1))[None], O.KIND_OD, 32, lo, hi)[0]
    nan = O.keys(ray((np.nan,) * 3, (np.nan,) * 3)[None], O.KIND_OD, 32, lo, hi)[0]
    assert below == 0 and nan == 0 and above == 0xFFFFFFFF
    # exactly on the upper face: u = 1 clamps to 2^b - 1
    on_hi = O.keys(ray((1, 1, 1), (1, 1, 1))[None], O.KIND_OD, 64, lo, hi)[0]
    assert on_hi == np.uint64(0xFFFFFFFFFFFFFFFF)
    # a flat box axis quantises that axis to 0
    flat_hi = np.array([1, 0, 1], np.float32)
    k = O.keys(ray((0.99, 0.0, 0.0), (0, 0, 1))[None], O.KIND_OD, 32, lo, flat_hi)[0]
    owners = _bits_per_component(O.KIND_OD, 32)
    ymask = sum(1 << p for p in owners[(0, 1)])
    assert int(k) & ymask == 0


def test_box_scaling_is_affine_invariant():
    # keys depend on the origin only through its position relative to the box
    r = _random_rays(4000)
    lo2 = np.array([10, -20, 3], np.float32)
    scale = np.float32(4.0)
    r2 = r.copy()
    r2[:, 0:3] = r[:, 0:3] * scale + lo2
    r2[:, 7] = r[:, 7] * scale
    for kind in (O.KIND_OD, O.KIND_OT):
        a = O.keys(r, kind, 32, *BOX)
        b = O.keys(r2, kind, 32, lo2, lo2 + scale)
        # power-of-two scale and exactly representable offsets keep most
        # quantisations identical; allow rare off-by-one cells from the
        # rounding of the shifted coordinates
        assert np.mean(a == b) > 0.99
