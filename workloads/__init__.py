"""Seeded synthetic workloads shared by the CPU oracle and the HIP path.

The paper measures on seven public scenes with a wavefront path tracer
(Section 4, Results).  Neither is available here, so these generators stand
in for them: a random triangle soup with uniform rays, and a procedural
"grid city" (boxes on a ground plane plus thin clutter triangles) seen by a
pinhole camera, whose diffuse bounces give incoherent secondary-ray
wavefronts like the ones the paper reorders (Section 1, Section 4.1).

Nothing here computes sort keys, sorts, builds a BVH or intersects a ray with
a triangle: the bounce rays are placed with an analytic box/plane
intersection in double precision (the thin clutter is ignored for that).
Arrays are float32: rays as (N, 8) = {org.xyz, tmin, dir.xyz, tmax},
triangles as (M, 9) = {v0.xyz, v1.xyz, v2.xyz}.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libwl.so")
_lib = None

DEFAULT_THREADS = min(16, os.cpu_count() or 1)


def build(force: bool = True) -> str:
    """Compile the generator with gcc into workloads/libwl.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u64, i64, i32, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        vp = ctypes.c_void_p
        L.wl_rng64.argtypes = [u64, u64, u64]; L.wl_rng64.restype = u64
        L.wl_rngu.argtypes = [u64, u64, u64]; L.wl_rngu.restype = dbl
        L.wl_random_tris.argtypes = [u64, i64, dbl, dbl, vp]; L.wl_random_tris.restype = None
        L.wl_random_rays.argtypes = [u64, i64, vp]; L.wl_random_rays.restype = None
        L.wl_city_heights.argtypes = [u64, i32, i32, vp]; L.wl_city_heights.restype = None
        L.wl_city_tris.argtypes = [u64, i32, i32, i64, vp, vp]; L.wl_city_tris.restype = i64
        L.wl_camera_rays.argtypes = [u64, i32, i32, vp, dbl, vp]; L.wl_camera_rays.restype = None
        L.wl_city_bounce.argtypes = [u64, u64, i32, i32, vp, vp, i64, dbl, vp, vp, i32]
        L.wl_city_bounce.restype = i64
        L.wl_city_hit_t.argtypes = [i32, i32, vp, vp, i64, vp, i32]; L.wl_city_hit_t.restype = None
        L.wl_sample.argtypes = [u64, u64, i64, i64, vp]; L.wl_sample.restype = None
        L.wl_shadow_rays.argtypes = [u64, u64, vp, i64, vp, dbl, i32, vp]; L.wl_shadow_rays.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


def rng64(seed: int, stream: int, ctr: int) -> int:
    return int(_get().wl_rng64(seed, stream, ctr))


def rngu(seed: int, stream: int, ctr: int) -> float:
    return float(_get().wl_rngu(seed, stream, ctr))


# ------------------------------------------------------------------ soup

def random_tris(seed: int, n: int, edge_lo: float = 0.005, edge_hi: float = 0.05) -> np.ndarray:
    out = np.empty((n, 9), np.float32)
    _get().wl_random_tris(seed, n, edge_lo, edge_hi, _p(out))
    return out


def random_rays(seed: int, n: int) -> np.ndarray:
    out = np.empty((n, 8), np.float32)
    _get().wl_random_rays(seed, n, _p(out))
    return out


# ------------------------------------------------------------------ city

@dataclass
class City:
    nx: int
    nz: int
    heights: np.ndarray   # (nz*nx,) float64, row-major over z then x
    tris: np.ndarray      # (M, 9) float32

    @property
    def extent(self) -> float:
        """Largest extent of the scene bounding box."""
        hi = float(self.tris[:, 1::3].max())
        return max(float(self.nx), float(self.nz), hi)


def city(seed: int, nx: int, nz: int, n_clutter: int) -> City:
    L = _get()
    h = np.empty(nx * nz, np.float64)
    L.wl_city_heights(seed, nx, nz, _p(h))
    m = 12 * nx * nz + n_clutter + 2
    tris = np.empty((m, 9), np.float32)
    got = L.wl_city_tris(seed, nx, nz, n_clutter, _p(h), _p(tris))
    assert got == m
    return City(nx, nz, h, tris)


def camera_rays(seed: int, w: int, h: int, eye, vfov_deg: float = 45.0) -> np.ndarray:
    out = np.empty((w * h, 8), np.float32)
    e = np.asarray(eye, np.float64)
    _get().wl_camera_rays(seed, w, h, _p(e), vfov_deg, _p(out))
    return out


def bounce(c: City, seed: int, stream: int, rays: np.ndarray, alive: np.ndarray | None = None,
           threads: int = DEFAULT_THREADS):
    """One diffuse bounce: returns (new_rays, alive) with alive[i] = 1 where
    the input ray hit the analytic city (and was itself alive)."""
    n = rays.shape[0]
    out = np.empty_like(rays)
    al = np.ones(n, np.uint8) if alive is None else np.ascontiguousarray(alive, dtype=np.uint8).copy()
    off = 1e-4 * c.extent
    _get().wl_city_bounce(seed, stream, c.nx, c.nz, _p(c.heights), _p(np.ascontiguousarray(rays)), n, off,
                          _p(out), _p(al), threads)
    return out, al


def city_hit_t(c: City, rays: np.ndarray, threads: int = DEFAULT_THREADS) -> np.ndarray:
    t = np.empty(rays.shape[0], np.float64)
    _get().wl_city_hit_t(c.nx, c.nz, _p(c.heights), _p(np.ascontiguousarray(rays)), rays.shape[0], _p(t), threads)
    return t


# ------------------------------------------------------------- workloads

@dataclass
class Workload:
    name: str
    tris: np.ndarray
    rays: np.ndarray
    alive: np.ndarray | None = None
    city: City | None = None


def soup(seed: int = 1, n_rays: int = 65536, n_tris: int = 4096) -> Workload:
    """Uniform rays in a random triangle soup: 65,536 rays against 4,096
    triangles by default (the small plain-method case)."""
    return Workload(f"soup{n_rays}x{n_tris}", random_tris(seed, n_tris), random_rays(seed, n_rays))


def _city_eye(c: City):
    return (c.nx / 2.0, 0.6 * max(c.nx, c.nz), c.nz / 2.0)


def city_bounce(seed: int, width: int, height: int, depth: int, nx: int = 100, nz: int = 100,
                n_clutter: int = 880_000, scene_seed: int | None = None, c: City | None = None) -> Workload:
    """Diffuse wavefront of a pinhole camera looking down on the grid city.

    depth 0 = primary rays; depth k >= 1 = rays leaving the hit points of
    depth k-1.  For depth >= 2 some slots are terminated (the depth k-1 ray
    escaped); `alive` marks the live ones.
    """
    if c is None:
        c = city(seed if scene_seed is None else scene_seed, nx, nz, n_clutter)
    rays = camera_rays(seed, width, height, _city_eye(c))
    alive = np.ones(rays.shape[0], np.uint8)
    for k in range(depth):
        rays, alive = bounce(c, seed, 100 + k, rays, alive)
        if k == 0:
            assert alive.all(), "a primary ray missed the ground quad"
    name = f"city{c.nx}x{c.nz}_{width}x{height}_d{depth}"
    return Workload(name, c.tris, rays, None if depth <= 1 else alive, c)


def bounce2_1080p(seed: int = 2) -> Workload:
    """1920x1080 bounce-2 diffuse wavefront on the ~1M-triangle grid city."""
    return city_bounce(seed, 1920, 1080, 1)


def shadow_rays(seed: int, stream: int, origins: np.ndarray, light_center, light_size: float, spp: int = 2):
    """spp shadow rays per origin (rows of a ray array) toward points uniform
    on a horizontal square light; tmax is the distance to the light point."""
    o = np.ascontiguousarray(origins, dtype=np.float32)
    out = np.empty((o.shape[0] * spp, 8), np.float32)
    lc = np.asarray(light_center, np.float64)
    _get().wl_shadow_rays(seed, stream, _p(o), o.shape[0], _p(lc), float(light_size), spp, _p(out))
    return out


def shadow_1080p(seed: int = 2) -> Workload:
    """Two shadow rays per primary hit point of the 1920x1080 view of the
    grid city (4,147,200 rays) toward a square light of side 5% of the
    largest scene extent, 30 units above the middle of the city (the paper's
    path tracer traces two shadow rays per bounce toward an area light of
    that size)."""
    w = bounce2_1080p(seed)
    c = w.city
    light = (c.nx / 2.0, 30.0, c.nz / 2.0)
    return Workload("city_shadow_1920x1080x2", w.tris, shadow_rays(seed, 400, w.rays, light, 0.05 * c.extent), None, c)


def bounce3_2160p(seed: int = 3, scene_seed: int = 2) -> Workload:
    """3840x2160 bounce-3 wavefront (8,294,400 slots) on the same city."""
    return city_bounce(seed, 3840, 2160, 2, scene_seed=scene_seed)


def city_small(seed: int = 7, width: int = 160, height: int = 90, depth: int = 1, n: int = 12,
               n_clutter: int = 4000) -> Workload:
    """A small city for tests: n x n boxes, a few thousand clutter triangles."""
    return city_bounce(seed, width, height, depth, nx=n, nz=n, n_clutter=n_clutter)


def segment_sizes(seed: int, count: int = 64, lo: int = 4096, hi: int = 1 << 21) -> np.ndarray:
    """Segment ray counts, floor(exp(U(ln lo, ln hi)))."""
    u = np.array([rngu(seed, 40, i) for i in range(count)])
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)



def _degenerate_scene(rng, n: int) -> np.ndarray:
    """n triangles in the unit cube: a tenth with two equal vertices, a tenth
    with collinear vertices, a tenth exact copies of earlier ones, a tenth
    axis-aligned in the plane z = 0.5, the rest random."""
    T = rng.random((n, 9)).astype(np.float32)
    k = n // 10
    T[0:k, 3:6] = T[0:k, 0:3]                                   # repeated vertex
    mid = rng.random((k, 1)).astype(np.float32)
    T[k:2 * k, 6:9] = T[k:2 * k, 0:3] + mid * (T[k:2 * k, 3:6] - T[k:2 * k, 0:3])  # collinear
    T[2 * k:3 * k] = T[rng.integers(3 * k, n, k)]               # duplicates (later ids)
    T[3 * k:4 * k, 2::3] = np.float32(0.5)                      # in the plane z = 0.5
    return T


def _degenerate_rays(rng, n: int) -> np.ndarray:
    """Rays with axis-aligned directions (zero and negative-zero components),
    rays in the plane z = 0.5 (parallel to the axis-aligned triangles), empty
    and inverted intervals, origins on that plane, and negative tmin."""
    o = rng.random((n, 3)).astype(np.float32) * np.float32(1.4) - np.float32(0.2)
    d = rng.normal(size=(n, 3)).astype(np.float32)
    q = n // 8
    axis = rng.integers(0, 3, q)
    d[:q] = 0.0
    d[np.arange(q), axis] = np.where(rng.random(q) < 0.5, -1.0, 1.0)
    d[:q:2][d[:q:2] == 0] = -0.0                                # negative zeros
    o[q:2 * q, 2] = np.float32(0.5)
    d[q:2 * q, 2] = 0.0                                         # in the plane z = 0.5
    o[2 * q:3 * q, 2] = np.float32(0.5)                         # starting on the plane
    d /= np.linalg.norm(d, axis=1, keepdims=True).astype(np.float32)
    tmin = np.zeros(n, np.float32)
    tmax = np.full(n, np.inf, np.float32)
    tmin[3 * q:3 * q + q // 2] = np.float32(0.3)
    tmax[3 * q:3 * q + q // 2] = np.float32(0.3)                # empty interval
    tmin[3 * q + q // 2:4 * q] = np.float32(2.0)
    tmax[3 * q + q // 2:4 * q] = np.float32(1.0)                # inverted interval
    tmin[4 * q:5 * q] = np.float32(-1.0)                        # hits behind the origin count
    return np.ascontiguousarray(np.concatenate([o, tmin[:, None], d, tmax[:, None]], axis=1), np.float32)


def degenerate(seed: int, n_tris: int, n_rays: int, scale: float = 1.0):
    """Triangles and rays at the degenerate ends of the closest-hit test,
    scaled by `scale` (a power of two keeps every scaled value exact)."""
    rng = np.random.default_rng(seed)
    T = _degenerate_scene(rng, n_tris)
    rays = _degenerate_rays(rng, n_rays)
    s = np.float32(scale)
    T = T * s
    rays[:, 0:3] *= s
    rays[:, 3] *= s
    rays[:, 7] *= s
    return T, rays


def sample_indices(seed: int, stream: int, n: int, pool: int) -> np.ndarray:
    """n indices drawn with replacement from range(pool)."""
    out = np.empty(n, np.int64)
    _get().wl_sample(seed, stream, n, pool, _p(out))
    return out
