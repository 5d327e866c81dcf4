"""Pins for the oracle's coherence measure M^64_CPS (Section 4.3): a capsule
fitted to each group of 64 consecutive rays (axis through the centroids of
origins and termination points, radii the mean distances from it).

Closed forms: rays on a cylinder give a sphere of radius R plus the
cylinder's side (4 pi R^2 + 2 pi R H); rays on a cone frustum give the two
hemispheres plus the frustum's side; coincident rays give 0; coincident
centroids give a sphere.  Invariants: translation, rotation, scale (area
scales by s^2), order within a group.  The miss rule (o + min(tmax, E) d)
and the partial last group are checked directly.
"""
import numpy as np
import pytest

import oracle as O

BOX = (np.zeros(3, np.float32), np.full(3, 10, np.float32))  # E = 10


def rays_between(p0, p1):
    """Rays from p0[i] to p1[i], with hits at the far point."""
    p0 = np.asarray(p0, np.float64)
    p1 = np.asarray(p1, np.float64)
    d = p1 - p0
    t = np.linalg.norm(d, axis=1)
    r = np.zeros((len(p0), 8), np.float32)
    r[:, 0:3] = p0
    r[:, 4:7] = d / t[:, None]
    r[:, 7] = np.inf
    h = np.zeros(len(p0), O.HIT_DTYPE)
    h["t"] = t
    h["prim"] = 0
    return r, h


def ring(R, z, n=64, phase=0.0):
    a = 2 * np.pi * (np.arange(n) + phase) / n
    return np.stack([R * np.cos(a) + 5, R * np.sin(a) + 5, np.full(n, z)], 1)


def test_cylinder():
    R, H = 0.5, 2.0
    r, h = rays_between(ring(R, 1.0), ring(R, 1.0 + H))
    g, m = O.coherence_m64(r, h, *BOX)
    want = 4 * np.pi * R * R + 2 * np.pi * R * H
    assert len(g) == 1 and abs(m - want) < 1e-5 * want


@pytest.mark.parametrize("R1,R2,H", [(0.25, 1.0, 3.0), (1.5, 0.5, 0.5)])
def test_cone_frustum(R1, R2, H):
    r, h = rays_between(ring(R1, 2.0), ring(R2, 2.0 + H))
    _, m = O.coherence_m64(r, h, *BOX)
    want = 2 * np.pi * R1 ** 2 + 2 * np.pi * R2 ** 2 + np.pi * (R1 + R2) * np.hypot(H, R1 - R2)
    assert abs(m - want) < 1e-5 * want


def test_coincident_rays_have_zero_area():
    p0 = np.tile([[1.0, 2.0, 3.0]], (64, 1))
    r, h = rays_between(p0, p0 + [0.0, 0.0, 1.5])
    _, m = O.coherence_m64(r, h, *BOX)
    assert abs(m) < 1e-9


def test_coincident_centroids_give_a_sphere():
    # every ray crosses the sphere's centre: origins and ends are antipodes
    rng = np.random.default_rng(0)
    u = rng.normal(size=(64, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    u = np.concatenate([u[:32], -u[:32]])      # centroid exactly at the centre
    c = np.array([5.0, 5.0, 5.0])
    r, h = rays_between(c + 0.75 * u, c - 0.75 * u)
    _, m = O.coherence_m64(r, h, *BOX)
    assert abs(m - 4 * np.pi * 0.75 ** 2) < 1e-4


def _random_set(n, seed):
    rng = np.random.default_rng(seed)
    p0 = rng.uniform(2, 8, (n, 3))
    p1 = p0 + rng.normal(size=(n, 3))
    return rays_between(p0, p1)


def test_invariances():
    r, h = _random_set(64, 1)
    _, m = O.coherence_m64(r, h, *BOX)
    perm = np.random.default_rng(2).permutation(64)
    _, mp = O.coherence_m64(r[perm], h[perm], *BOX)
    assert abs(mp - m) < 1e-9 * m
    # translation by a dyadic offset
    r2 = r.copy()
    r2[:, 0:3] += np.float32(0.5)
    _, mt = O.coherence_m64(r2, h, *BOX)
    assert abs(mt - m) < 1e-5 * m
    # scaling by 2: area x 4 (rays and hit distances scale together)
    r3, h3 = r.copy(), h.copy()
    r3[:, 0:3] *= 2
    h3["t"] *= 2
    _, ms = O.coherence_m64(r3, h3, (0, 0, 0), (20, 20, 20))
    assert abs(ms - 4 * m) < 1e-5 * m
    # rotation about z by 90 degrees
    r4 = r.copy()
    r4[:, [0, 1]] = np.stack([10 - r[:, 1], r[:, 0]], 1)
    r4[:, [4, 5]] = np.stack([-r[:, 5], r[:, 4]], 1)
    _, mr = O.coherence_m64(r4, h, *BOX)
    assert abs(mr - m) < 1e-5 * m


def test_misses_end_at_tmax_or_the_extent():
    R = 0.5
    p0 = ring(R, 1.0)
    r, h = rays_between(p0, p0 + [0.0, 0.0, 4.0])
    h["prim"] = -1
    h["t"] = np.inf
    r[:, 7] = 3.0                      # ends at tmax = 3
    _, m = O.coherence_m64(r, h, *BOX)
    assert abs(m - (4 * np.pi * R * R + 2 * np.pi * R * 3.0)) < 1e-5 * m
    r[:, 7] = np.inf                   # ends at E = 10
    _, m = O.coherence_m64(r, h, *BOX)
    assert abs(m - (4 * np.pi * R * R + 2 * np.pi * R * 10.0)) < 1e-5 * m


def test_groups_and_partial_tail():
    r, h = _random_set(100, 3)
    g, m = O.coherence_m64(r, h, *BOX)
    g0, _ = O.coherence_m64(r[:64], h[:64], *BOX)
    g1, _ = O.coherence_m64(r[64:], h[64:], *BOX)
    assert len(g) == 2 and g[0] == g0[0] and g[1] == g1[0] and m == (g[0] + g[1]) / 2
    assert O.coherence_m64(r[:0], h[:0], *BOX)[1] == 0.0
