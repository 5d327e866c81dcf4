"""CPU oracle for the ray-reordering hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It
shares no code with the HIP library (different language, different build,
different data layout) and follows the paper (Meister et al., "On Ray
Reordering Techniques for Faster GPU Ray Tracing", I3D 2020) directly:

* keys            -- Section 3.1 and Figure "codes": origin-direction
                     (Reis) and Two Point (origin-termination) keys with the
                     fixed-length termination estimate (Section 3.1.6), the
                     figure's other layouts (Origin, Costa, Aila, Aila
                     Compact, Octahedron), and Two Point with the adaptive
                     (length table) or real (traced) termination point.
* LengthTable     -- Section 3.1.6: the 2^20-cell table of mean traced
                     lengths keyed by the 20-bit Aila Compact code.
* coherence_m64   -- Section 4.3: the capsule surface-area coherence measure
                     of groups of 64 consecutive rays and its mean.
* sort_pairs      -- Section 3.2: key/index pairs sorted by key; the
                     stable order is the lexicographic order of (key, index).
* local_sort_pairs -- Section 3.2: sorting within segments of consecutive
                     keys (block-wise) instead of globally.
* gather          -- Section 3.2: "an additional pass" moving the ray data.
* BVH.trace       -- closest-hit trace (Section 4.1), brute_force its
                     definition.
* compact         -- the live slots of a wavefront, ascending.

Every function here is pinned by the CPU tests against hand-derived values,
closed forms, invariants or brute force; see the tests for each pin.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

KIND_NONE, KIND_OD, KIND_OT = 0, 1, 2
KIND_ORIGIN, KIND_COSTA, KIND_AILA, KIND_AILA_COMPACT, KIND_OCTAHEDRON = 3, 4, 5, 6, 7
KIND_TP_ADAPTIVE, KIND_TP_REAL = 8, 9
KIND_CODE20 = 100
CELL_DTYPE = np.dtype([("sum", np.uint64), ("count", np.uint32), ("unused", np.uint32)])
N_CELLS = 1 << 20
HIT_DTYPE = np.dtype([("t", np.float32), ("prim", np.int32), ("u", np.float32), ("v", np.float32)])
DEFAULT_THREADS = min(16, os.cpu_count() or 1)


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc: binary32 arithmetic in source order, no
    contraction into fused multiply-adds, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _get():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        vp, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float
        L.orc_keys.argtypes = [vp, i64, i32, i32, vp, vp, f32, i32, vp, vp]; L.orc_keys.restype = ctypes.c_int
        L.orc_octahedral.argtypes = [vp, vp, vp]; L.orc_octahedral.restype = None
        L.orc_cell_code.argtypes = [vp, vp, vp]; L.orc_cell_code.restype = ctypes.c_uint32
        L.orc_len_init.argtypes = [vp, f32]; L.orc_len_init.restype = None
        L.orc_len_accumulate.argtypes = [vp, vp, vp, i64, vp, vp]; L.orc_len_accumulate.restype = None
        L.orc_len_lookup.argtypes = [vp, vp, vp, vp]; L.orc_len_lookup.restype = f32
        L.orc_cps.argtypes = [vp, vp, i64, vp, vp, vp, vp]; L.orc_cps.restype = None
        L.orc_key_layout.argtypes = [i32, i32, i32, vp, vp]; L.orc_key_layout.restype = ctypes.c_int
        L.orc_mt.argtypes = [vp, vp, vp, vp, vp, vp]; L.orc_mt.restype = ctypes.c_int
        L.orc_brute_force.argtypes = [vp, i64, vp, i64, vp, i32]; L.orc_brute_force.restype = None
        L.orc_bvh_build.argtypes = [vp, i64]; L.orc_bvh_build.restype = vp
        L.orc_bvh_free.argtypes = [vp]; L.orc_bvh_free.restype = None
        L.orc_bvh_depth.argtypes = [vp]; L.orc_bvh_depth.restype = i32
        L.orc_bvh_nodes.argtypes = [vp]; L.orc_bvh_nodes.restype = i32
        L.orc_bvh_trace.argtypes = [vp, vp, vp, i64, vp, i32]; L.orc_bvh_trace.restype = None
        L.orc_compact.argtypes = [vp, i64, vp]; L.orc_compact.restype = i64
        _lib = L
    return _lib


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


# ------------------------------------------------------------------ keys

def key_layout(kind: int, key_bits: int, origin_bits: int = 0):
    """(src, comp) per key bit, MSB first; src 0 = origin, 1 = direction,
    2 = termination point, 3 = octahedral direction (u, v), -1 = zero."""
    src = np.zeros(key_bits, np.int8)
    comp = np.zeros(key_bits, np.int8)
    rc = _get().orc_key_layout(kind, key_bits, origin_bits, _p(src), _p(comp))
    if rc != 0:
        raise ValueError("bad layout")
    return src, comp


def keys(rays, kind: int, key_bits: int, box_lo, box_hi, ratio: float = 0.25, origin_bits: int = 0,
         aux=None) -> np.ndarray:
    """Sort keys of rays (N, 8) float32; uint32 for 32-bit keys, uint64 for
    64-bit keys.  aux: a LengthTable (Two Point Adaptive) or the rays' hits,
    HIT_DTYPE (Two Point Real)."""
    r = _c(rays, np.float32).reshape(-1, 8)
    lo = _c(box_lo, np.float32)
    hi = _c(box_hi, np.float32)
    out = np.empty(r.shape[0], np.uint64)
    a = None
    if kind == KIND_TP_ADAPTIVE:
        a = aux.cells
    elif kind == KIND_TP_REAL:
        a = np.ascontiguousarray(aux, dtype=HIT_DTYPE)
        if a.shape[0] != r.shape[0]:
            raise ValueError("one hit per ray")
    rc = _get().orc_keys(_p(r), r.shape[0], kind, key_bits, _p(lo), _p(hi), float(np.float32(ratio)), origin_bits,
                         _p(a) if a is not None else None, _p(out))
    if rc != 0:
        raise ValueError("bad key parameters")
    return out.astype(np.uint32) if key_bits == 32 else out


def octahedral(dirs) -> np.ndarray:
    """Octahedral coordinates (u, v) in [-1, 1]^2 of directions (N, 3)."""
    d = _c(dirs, np.float32).reshape(-1, 3)
    out = np.empty((d.shape[0], 2), np.float32)
    u = ctypes.c_float()
    v = ctypes.c_float()
    L = _get()
    for i in range(d.shape[0]):
        L.orc_octahedral(_p(d[i]), ctypes.byref(u), ctypes.byref(v))
        out[i] = (u.value, v.value)
    return out


def cell_code(rays, box_lo, box_hi) -> np.ndarray:
    """20-bit length-table cell of each ray (the Aila Compact prefix)."""
    r = _c(rays, np.float32).reshape(-1, 8)
    lo = _c(box_lo, np.float32)
    hi = _c(box_hi, np.float32)
    L = _get()
    return np.array([L.orc_cell_code(_p(r[i]), _p(lo), _p(hi)) for i in range(r.shape[0])], np.uint32)


class LengthTable:
    """Two Point Adaptive length table (Section 3.1.6): 2^20 cells of
    {sum of fixed-point lengths, count}, each starting with one dummy ray
    of length ratio x the largest box extent."""

    def __init__(self, box_lo, box_hi, ratio: float = 0.25):
        self.lo = _c(box_lo, np.float32)
        self.hi = _c(box_hi, np.float32)
        self.cells = np.zeros(N_CELLS, CELL_DTYPE)
        _get().orc_len_init(_p(self.cells), float(np.float32(ratio)))

    def accumulate(self, rays, hits):
        r = _c(rays, np.float32).reshape(-1, 8)
        h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
        if h.shape[0] != r.shape[0]:
            raise ValueError("one hit per ray")
        _get().orc_len_accumulate(_p(self.cells), _p(r), _p(h), r.shape[0], _p(self.lo), _p(self.hi))

    def lookup(self, rays) -> np.ndarray:
        r = _c(rays, np.float32).reshape(-1, 8)
        L = _get()
        return np.array([L.orc_len_lookup(_p(self.cells), _p(r[i]), _p(self.lo), _p(self.hi))
                         for i in range(r.shape[0])], np.float32)


def coherence_m64(rays, hits, box_lo, box_hi):
    """(per-group measures, mean) of M^64_CPS over consecutive groups of 64."""
    r = _c(rays, np.float32).reshape(-1, 8)
    h = np.ascontiguousarray(hits, dtype=HIT_DTYPE)
    if h.shape[0] != r.shape[0]:
        raise ValueError("one hit per ray")
    lo = _c(box_lo, np.float32)
    hi = _c(box_hi, np.float32)
    g = np.zeros((r.shape[0] + 63) // 64, np.float64)
    m = ctypes.c_double()
    _get().orc_cps(_p(r), _p(h), r.shape[0], _p(lo), _p(hi), _p(g), ctypes.byref(m))
    return g, m.value


def scene_box(tris):
    """Axis-aligned bounds of a triangle array (M, 9), float32."""
    t = _c(tris, np.float32).reshape(-1, 3)
    return t.min(axis=0), t.max(axis=0)


# ------------------------------------------------------- compact / sort

def compact(alive) -> np.ndarray:
    a = _c(alive, np.uint8)
    out = np.empty(a.shape[0], np.uint32)
    m = _get().orc_compact(_p(a), a.shape[0], _p(out))
    return out[:m].copy()


def sort_pairs(k, idx=None):
    """Pairs (key, index) in ascending key order; equal keys keep ascending
    index order, so the result is the lexicographic order of (key, index)."""
    k = np.asarray(k)
    if idx is None:
        idx = np.arange(k.shape[0], dtype=np.uint32)
    idx = np.asarray(idx, dtype=np.uint32)
    order = np.lexsort((idx, k))
    return k[order], idx[order]


def local_sort_pairs(k, idx=None, block: int = 1024):
    """Section 3.2's local sorting: each run of `block` consecutive pairs
    (the last may be shorter) sorted on its own, stably, by key."""
    k = np.asarray(k)
    if idx is None:
        idx = np.arange(k.shape[0], dtype=np.uint32)
    idx = np.asarray(idx, dtype=np.uint32)
    ko = np.empty_like(k)
    io = np.empty_like(idx)
    for b in range(0, k.shape[0], block):
        ko[b:b + block], io[b:b + block] = sort_pairs(k[b:b + block], idx[b:b + block])
    return ko, io


def gather(rays, idx) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(rays)[np.asarray(idx, dtype=np.int64)])


def scatter(values, idx, n: int | None = None, fill=None):
    """out[idx[i]] = values[i]; the inverse of gather for a permutation."""
    v = np.asarray(values)
    n = v.shape[0] if n is None else n
    out = np.empty((n,) + v.shape[1:], v.dtype)
    if fill is not None:
        out[...] = fill
    out[np.asarray(idx, dtype=np.int64)] = v
    return out


# ----------------------------------------------------------------- trace

def miss_hit():
    return np.array((np.inf, -1, 0.0, 0.0), dtype=HIT_DTYPE)


def mt(ray, tri):
    """Moller-Trumbore test of one ray (8 floats) and one triangle (9
    floats): (hit, t, u, v)."""
    r = _c(ray, np.float32)
    tr = _c(tri, np.float32)
    t = ctypes.c_float(); u = ctypes.c_float(); v = ctypes.c_float()
    ok = _get().orc_mt(_p(r), _p(r[4:]), _p(tr), ctypes.byref(t), ctypes.byref(u), ctypes.byref(v))
    return bool(ok), t.value, u.value, v.value


def brute_force(tris, rays, threads: int = DEFAULT_THREADS) -> np.ndarray:
    t = _c(tris, np.float32)
    r = _c(rays, np.float32)
    out = np.empty(r.shape[0], HIT_DTYPE)
    _get().orc_brute_force(_p(t), t.shape[0], _p(r), r.shape[0], _p(out), threads)
    return out


class BVH:
    """Median-split binary BVH over a triangle array (kept alive here)."""

    def __init__(self, tris):
        self.tris = _c(tris, np.float32)
        self.h = _get().orc_bvh_build(_p(self.tris), self.tris.shape[0])
        if not self.h:
            raise ValueError("oracle BVH build failed")

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_bvh_free(self.h)
            self.h = None

    @property
    def depth(self) -> int:
        return int(_get().orc_bvh_depth(self.h))

    @property
    def nodes(self) -> int:
        return int(_get().orc_bvh_nodes(self.h))

    def trace(self, rays, idx=None, threads: int = DEFAULT_THREADS) -> np.ndarray:
        r = _c(rays, np.float32)
        n = r.shape[0] if idx is None else len(idx)
        ix = None if idx is None else _c(idx, np.uint32)
        out = np.empty(n, HIT_DTYPE)
        _get().orc_bvh_trace(self.h, _p(r), None if ix is None else _p(ix), n, _p(out), threads)
        return out


# --------------------------------------------------------------- pipeline

def reorder_and_trace(bvh: BVH, rays, kind: int, key_bits: int, box_lo, box_hi, ratio: float = 0.25,
                      origin_bits: int = 0, alive=None, threads: int = DEFAULT_THREADS):
    """The whole path on the CPU: (compaction), keys, sort, gather, trace.
    Returns dict(keys, idx, rays, hits) in sorted order."""
    r = _c(rays, np.float32)
    idx = np.arange(r.shape[0], dtype=np.uint32) if alive is None else compact(alive)
    if kind == KIND_NONE:
        k = None
        sidx = idx
    else:
        k = keys(r[idx], kind, key_bits, box_lo, box_hi, ratio, origin_bits)
        k, sidx = sort_pairs(k, idx)
    sr = gather(r, sidx)
    hits = bvh.trace(sr, threads=threads)
    return {"keys": k, "idx": sidx, "rays": sr, "hits": hits}
