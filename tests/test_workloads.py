"""The seeded generators: determinism and the shape of each workload."""
import numpy as np

import workloads as W


def test_deterministic():
    a = W.soup(seed=1, n_rays=1000, n_tris=100)
    b = W.soup(seed=1, n_rays=1000, n_tris=100)
    c = W.soup(seed=2, n_rays=1000, n_tris=100)
    assert a.rays.tobytes() == b.rays.tobytes() and a.tris.tobytes() == b.tris.tobytes()
    assert a.rays.tobytes() != c.rays.tobytes()


def test_soup_shape():
    w = W.soup()
    assert w.rays.shape == (65536, 8) and w.tris.shape == (4096, 9)
    n = np.linalg.norm(w.rays[:, 4:7].astype(np.float64), axis=1)
    assert np.allclose(n, 1, atol=1e-6)
    assert (w.rays[:, 0:3] >= 0).all() and (w.rays[:, 0:3] < 1).all()
    assert np.all(w.rays[:, 3] == 0) and np.all(np.isinf(w.rays[:, 7]))
    e = np.linalg.norm(w.tris[:, 3:6] - w.tris[:, 0:3], axis=1)
    assert e.min() > 0.0049 and e.max() < 0.0501


def test_city_counts_and_bounce():
    w = W.city_small(seed=3, width=64, height=36, depth=2, n=12, n_clutter=1000)
    assert w.tris.shape[0] == 12 * 144 + 1000 + 2
    assert w.rays.shape == (64 * 36, 8)
    assert w.alive is not None and 0 < w.alive.mean() < 1
    n = np.linalg.norm(w.rays[:, 4:7].astype(np.float64), axis=1)
    assert np.allclose(n[w.alive == 1], 1, atol=1e-6)


def test_thread_count_does_not_change_output():
    c = W.city(5, 12, 12, 0)
    rays = W.camera_rays(5, 80, 45, (6.0, 7.2, 6.0))
    a, al = W.bounce(c, 5, 100, rays, threads=1)
    b, bl = W.bounce(c, 5, 100, rays, threads=7)
    assert a.tobytes() == b.tobytes() and al.tobytes() == bl.tobytes()


def test_segment_sizes_range():
    s = W.segment_sizes(4)
    assert s.shape == (64,) and s.min() >= 4096 and s.max() < (1 << 21)


def test_shadow_rays_end_on_the_light():
    w = W.city_small(seed=5, width=48, height=27, depth=1)
    c = w.city
    lc = (c.nx / 2.0, 30.0, c.nz / 2.0)
    size = 0.05 * c.extent
    s = W.shadow_rays(5, 400, w.rays, lc, size, spp=2)
    assert s.shape == (2 * w.rays.shape[0], 8)
    assert np.array_equal(s[0::2, 0:3], w.rays[:, 0:3]) and np.array_equal(s[1::2, 0:3], w.rays[:, 0:3])
    assert np.allclose(np.linalg.norm(s[:, 4:7], axis=1), 1.0, atol=1e-6)
    end = s[:, 0:3].astype(np.float64) + s[:, 7:8].astype(np.float64) * s[:, 4:7].astype(np.float64)
    assert np.allclose(end[:, 1], 30.0, atol=1e-3)
    assert np.all(np.abs(end[:, 0] - lc[0]) <= size / 2 + 1e-3) and np.all(np.abs(end[:, 2] - lc[2]) <= size / 2 + 1e-3)
    assert np.all(s[:, 3] == 0)
    # the same seed and stream give the same rays; another stream other ones
    assert np.array_equal(s, W.shadow_rays(5, 400, w.rays, lc, size, spp=2))
    assert not np.array_equal(s, W.shadow_rays(5, 401, w.rays, lc, size, spp=2))
