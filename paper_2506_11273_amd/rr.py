"""ctypes binding of librr (include/rr.h), with the same function names.

Argument marshalling only: every step runs in the HIP library.  Device
memory comes from PyTorch tensors on a ROCm device and work goes on the
current torch stream unless a stream is given.  A missing library is a hard
error; there is no CPU fallback.

Tensor conventions:
  rays   (N, 8) float32  {org.xyz, tmin, dir.xyz, tmax}
  hits   (N, 4) float32  {t, prim (int32 bits), u, v}
  keys   (N,)  int32 / int64 holding the uint32 / uint64 key bits
  idx    (N,)  int32 holding uint32 indices
  alive  (N,)  uint8
  count  (1,)  int32 holding a uint32 count
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

RR_OK = 0
RR_ERR_INVALID_ARGUMENT = -1
RR_ERR_OUT_OF_MEMORY = -2
RR_ERR_DEVICE = -3
RR_ERR_UNSUPPORTED = -4
RR_ERR_WORKSPACE_TOO_SMALL = -5
RR_ERR_BUDGET = -6

RR_KEY_NONE = 0
RR_KEY_ORIGIN_DIRECTION = 1
RR_KEY_ORIGIN_TERMINATION = 2
RR_KEY_ORIGIN = 3
RR_KEY_DIRECTION_ORIGIN = 4
RR_KEY_AILA = 5
RR_KEY_AILA_COMPACT = 6
RR_KEY_OCTAHEDRON = 7
RR_KEY_TWO_POINT_ADAPTIVE = 8
RR_KEY_TWO_POINT_REAL = 9
RR_LENGTH_CELLS = 1 << 20

RR_HITS_ORIGINAL_ORDER = 1
RR_INDIRECT = 2
RR_LOCAL_SORT_1024 = 4
RR_LOCAL_SORT_2048 = 8
RR_LOCAL_SORT_4096 = 16
RR_ANY_HIT = 32
RR_SORT_MSD = 64

# every symbol include/rr.h declares
EXPORTS = (
    "rr_status_string", "rr_device_count",
    "rr_scene_create", "rr_scene_create_ex", "rr_scene_bounds", "rr_scene_info", "rr_scene_destroy",
    "rr_keys_workspace_size", "rr_compute_keys", "rr_length_table_init", "rr_length_table_accumulate",
    "rr_coherence_m64",
    "rr_sort_workspace_size", "rr_sort", "rr_sort_ex", "rr_sort_msd", "rr_local_sort",
    "rr_gather", "rr_scatter_hits", "rr_trace", "rr_trace_ex", "rr_trace_any", "rr_trace_profile",
    "rr_reorder_workspace_size", "rr_reorder_and_trace", "rr_reorder_and_trace_noalloc",
)


class RRError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = status_string(status) if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


class KeyParams(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("key_bits", ctypes.c_uint32),
                ("box_lo", ctypes.c_float * 3), ("box_hi", ctypes.c_float * 3),
                ("term_ratio", ctypes.c_float), ("origin_bits", ctypes.c_uint32), ("aux", ctypes.c_void_p)]


_lib = None


def load():
    """Load librr.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    st = ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "rr_status_string": ([st], ctypes.c_char_p),
        "rr_device_count": ([P(i32)], st),
        "rr_scene_create": ([vp, i64, P(vp)], st),
        "rr_scene_create_ex": ([vp, i64, i32, P(vp)], st),
        "rr_scene_bounds": ([vp, vp, vp], st),
        "rr_scene_info": ([vp, P(i64), P(i32), P(i64)], st),
        "rr_scene_destroy": ([vp], st),
        "rr_keys_workspace_size": ([i64, P(sz)], st),
        "rr_compute_keys": ([vp, i64, vp, P(KeyParams), vp, vp, vp, vp, sz, vp], st),
        "rr_length_table_init": ([vp, P(KeyParams), vp], st),
        "rr_coherence_m64": ([vp, vp, i64, P(KeyParams), vp, vp, vp], st),
        "rr_length_table_accumulate": ([vp, vp, vp, vp, i64, vp, P(KeyParams), vp], st),
        "rr_sort_workspace_size": ([i64, u32, P(sz)], st),
        "rr_sort": ([vp, vp, i64, vp, u32, vp, sz, vp], st),
        "rr_sort_ex": ([vp, vp, i64, vp, u32, u32, u32, vp, sz, vp], st),
        "rr_sort_msd": ([vp, vp, i64, vp, u32, vp, sz, vp], st),
        "rr_local_sort": ([vp, vp, i64, vp, u32, u32, vp], st),
        "rr_gather": ([vp, vp, i64, vp, vp, vp], st),
        "rr_scatter_hits": ([vp, vp, i64, vp, vp, vp], st),
        "rr_trace": ([vp, vp, i64, vp, vp, vp], st),
        "rr_trace_profile": ([vp, vp, i64, vp, vp, vp], st),
        "rr_trace_any": ([vp, vp, i64, vp, vp, vp], st),
        "rr_trace_ex": ([vp, vp, i64, vp, vp, u32, vp], st),
        "rr_reorder_workspace_size": ([i64, P(KeyParams), P(sz)], st),
        "rr_reorder_and_trace": ([vp, vp, i64, vp, P(KeyParams), vp, vp, vp, u32, vp, sz, vp], st),
        "rr_reorder_and_trace_noalloc": ([vp, vp, i64, vp, P(KeyParams), vp, vp, vp, u32, vp], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    _bind_extras(L)
    return L


def _bind_extras(L):
    """Symbols of the batched and serving layers, when present."""
    try:
        from . import batch as _b
        _b._bind(L)
    except (ImportError, AttributeError):
        pass


def status_string(s: int) -> str:
    return load().rr_status_string(s).decode()


def _check(status: int, what: str):
    if status != RR_OK:
        raise RRError(status, what)


# ------------------------------------------------------------ marshalling

def _torch():
    import torch
    return torch


def _ptr(t, name: str, dtype=None, required: bool = True) -> Optional[int]:
    if t is None:
        if required:
            raise ValueError(f"{name} is required")
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on a ROCm device")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live in device memory, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def key_params(kind: int, key_bits: int, box_lo, box_hi, term_ratio: float = 0.25,
               origin_bits: int = 0, aux=None) -> KeyParams:
    """aux: the length table (a LengthTable or its device tensor) for
    RR_KEY_TWO_POINT_ADAPTIVE, the rays' hits (N, 4) float32 device tensor
    for RR_KEY_TWO_POINT_REAL."""
    p = KeyParams()
    p.kind = int(kind)
    p.key_bits = int(key_bits)
    for k in range(3):
        p.box_lo[k] = float(box_lo[k])
        p.box_hi[k] = float(box_hi[k])
    p.term_ratio = float(np.float32(term_ratio))
    p.origin_bits = int(origin_bits)
    if isinstance(aux, LengthTable):
        aux = aux.cells
    p.aux = int(aux.data_ptr()) if aux is not None else None
    # the tensor must outlive every call that uses these parameters
    p._aux_ref = aux
    return p


class LengthTable:
    """Two Point Adaptive length table on the device (RR_LENGTH_CELLS cells
    of 16 bytes), initialised to one dummy ray of term_ratio x the largest
    extent of params' box per cell."""

    def __init__(self, params: KeyParams, device=None, stream=None):
        torch = _torch()
        self.cells = torch.empty((RR_LENGTH_CELLS, 4), dtype=torch.int32, device=device or "cuda")
        self.params = params
        _check(load().rr_length_table_init(self.cells.data_ptr(), ctypes.byref(params), _stream(stream)),
               "rr_length_table_init")

    def accumulate(self, rays, hits, idx=None, count=None, stream=None):
        torch = _torch()
        n = int(hits.shape[0])
        _check(load().rr_length_table_accumulate(self.cells.data_ptr(), _ptr(rays, "rays", torch.float32),
                                                 _ptr(idx, "idx", torch.int32, False),
                                                 _ptr(hits, "hits", torch.float32), n,
                                                 _ptr(count, "count", torch.int32, False),
                                                 ctypes.byref(self.params), _stream(stream)),
               "rr_length_table_accumulate")

    def numpy(self):
        """Cells as a structured array {sum uint64, count uint32, unused uint32}."""
        import numpy as _np
        raw = self.cells.cpu().numpy().view(_np.uint8).reshape(-1)
        return raw.view(_np.dtype([("sum", _np.uint64), ("count", _np.uint32), ("unused", _np.uint32)]))


def _n_rows(rays) -> int:
    if rays.dim() != 2 or rays.shape[1] != 8:
        raise ValueError("rays must be (N, 8) float32")
    return int(rays.shape[0])


# ------------------------------------------------------------------ scene

class Scene:
    """A BVH over a host triangle array (M, 9) float32, resident on the
    current device until close()."""

    def __init__(self, tris, builder: int = 1):
        L = load()
        a = np.ascontiguousarray(tris, dtype=np.float32).reshape(-1, 9)
        h = ctypes.c_void_p()
        _check(L.rr_scene_create_ex(a.ctypes.data, a.shape[0], builder, ctypes.byref(h)), "rr_scene_create")
        self.handle = h
        self.n_tris = a.shape[0]

    def bounds(self):
        lo = np.zeros(3, np.float32)
        hi = np.zeros(3, np.float32)
        _check(load().rr_scene_bounds(self.handle, lo.ctypes.data, hi.ctypes.data), "rr_scene_bounds")
        return lo, hi

    def info(self) -> dict:
        n = ctypes.c_int64(); d = ctypes.c_int32(); b = ctypes.c_int64()
        _check(load().rr_scene_info(self.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(b)), "rr_scene_info")
        return {"nodes": n.value, "depth": d.value, "device_bytes": b.value}

    def close(self):
        if getattr(self, "handle", None):
            if _lib is not None:
                _lib.rr_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ------------------------------------------------------------- allocation

def _empty(n, dtype, device):
    torch = _torch()
    return torch.empty(n, dtype=dtype, device=device)


def workspace(nbytes: int, device):
    """A 256-byte aligned device workspace of at least nbytes."""
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def keys_workspace_size(n: int) -> int:
    b = ctypes.c_size_t()
    _check(load().rr_keys_workspace_size(n, ctypes.byref(b)), "rr_keys_workspace_size")
    return b.value


def sort_workspace_size(n: int, key_bits: int) -> int:
    b = ctypes.c_size_t()
    _check(load().rr_sort_workspace_size(n, key_bits, ctypes.byref(b)), "rr_sort_workspace_size")
    return b.value


def reorder_workspace_size(n: int, params: KeyParams) -> int:
    b = ctypes.c_size_t()
    _check(load().rr_reorder_workspace_size(n, ctypes.byref(params), ctypes.byref(b)), "rr_reorder_workspace_size")
    return b.value


# -------------------------------------------------------------- functions

def rr_compute_keys(rays, params: KeyParams, alive=None, keys=None, idx=None, count=None, ws=None, stream=None):
    """Keys and indices of rays (compacted when alive is given).
    Returns (keys, idx, count)."""
    torch = _torch()
    L = load()
    n = _n_rows(rays)
    kd = torch.int64 if params.key_bits == 64 else torch.int32
    keys = _empty(n, kd, rays.device) if keys is None else keys
    idx = _empty(n, torch.int32, rays.device) if idx is None else idx
    if alive is not None and count is None:
        count = _empty(1, torch.int32, rays.device)
    if alive is not None and ws is None:
        ws = workspace(keys_workspace_size(n), rays.device)
    _check(L.rr_compute_keys(_ptr(rays, "rays", torch.float32), n, _ptr(alive, "alive", torch.uint8, False),
                             ctypes.byref(params), _ptr(keys, "keys", kd), _ptr(idx, "idx", torch.int32),
                             _ptr(count, "count", torch.int32, False), _ptr(ws, "workspace", None, False),
                             0 if ws is None else ws.numel() * ws.element_size(), _stream(stream)),
           "rr_compute_keys")
    return keys, idx, count


def rr_sort(keys, idx, count=None, key_bits: Optional[int] = None, digit_bits: int = 8,
            keys_per_thread: Optional[int] = None, ws=None, stream=None, msd: bool = False):
    """Stable in-place sort of (keys, idx); keys_per_thread None takes the
    library's choice for the size (rr_sort), a value calls rr_sort_ex (the
    LSD sort), msd=True calls rr_sort_msd."""
    torch = _torch()
    L = load()
    n = int(keys.shape[0])
    kb = key_bits or (64 if keys.dtype == torch.int64 else 32)
    if ws is None:
        ws = workspace(sort_workspace_size(n, kb), keys.device)
    kp = _ptr(keys, "keys", (torch.int32, torch.int64))
    ip = _ptr(idx, "idx", torch.int32)
    cp = _ptr(count, "count", torch.int32, False)
    wp, wb = _ptr(ws, "workspace"), ws.numel() * ws.element_size()
    if msd:
        _check(L.rr_sort_msd(kp, ip, n, cp, kb, wp, wb, _stream(stream)), "rr_sort_msd")
    elif keys_per_thread is None and digit_bits == 8:
        _check(L.rr_sort(kp, ip, n, cp, kb, wp, wb, _stream(stream)), "rr_sort")
    else:
        _check(L.rr_sort_ex(kp, ip, n, cp, kb, digit_bits, keys_per_thread or 8, wp, wb, _stream(stream)),
               "rr_sort")
    return keys, idx


def rr_local_sort(keys, idx, block: int = 1024, count=None, key_bits: Optional[int] = None, stream=None):
    """Stable in-place sort of every run of `block` consecutive (key, idx)
    pairs (Section 3.2's local sorting)."""
    torch = _torch()
    kb = key_bits or (64 if keys.dtype == torch.int64 else 32)
    _check(load().rr_local_sort(_ptr(keys, "keys", (torch.int32, torch.int64)), _ptr(idx, "idx", torch.int32),
                                int(keys.shape[0]), _ptr(count, "count", torch.int32, False), kb, int(block),
                                _stream(stream)), "rr_local_sort")
    return keys, idx


def rr_gather(rays, idx, count=None, out=None, stream=None):
    torch = _torch()
    n = int(idx.shape[0])
    out = torch.empty((n, 8), dtype=torch.float32, device=rays.device) if out is None else out
    _check(load().rr_gather(_ptr(rays, "rays", torch.float32), _ptr(idx, "idx", torch.int32), n,
                            _ptr(count, "count", torch.int32, False), _ptr(out, "out", torch.float32),
                            _stream(stream)), "rr_gather")
    return out


def rr_scatter_hits(hits, idx, count=None, out=None, stream=None):
    torch = _torch()
    n = int(idx.shape[0])
    out = torch.empty((n, 4), dtype=torch.float32, device=hits.device) if out is None else out
    _check(load().rr_scatter_hits(_ptr(hits, "hits", torch.float32), _ptr(idx, "idx", torch.int32), n,
                                  _ptr(count, "count", torch.int32, False), _ptr(out, "out", torch.float32),
                                  _stream(stream)), "rr_scatter_hits")
    return out


def rr_trace(scene: Scene, rays, count=None, hits=None, refill: Optional[int] = None, stream=None):
    torch = _torch()
    n = _n_rows(rays)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device) if hits is None else hits
    if refill is None:
        _check(load().rr_trace(scene.handle, _ptr(rays, "rays", torch.float32), n,
                               _ptr(count, "count", torch.int32, False), _ptr(hits, "hits", torch.float32),
                               _stream(stream)), "rr_trace")
    else:
        _check(load().rr_trace_ex(scene.handle, _ptr(rays, "rays", torch.float32), n,
                                  _ptr(count, "count", torch.int32, False), _ptr(hits, "hits", torch.float32),
                                  int(refill), _stream(stream)), "rr_trace_ex")
    return hits


def rr_trace_any(scene: Scene, rays, count=None, hits=None, stream=None):
    """Any-hit (occlusion) trace: prim >= 0 where some triangle meets the
    ray in (tmin, tmax)."""
    torch = _torch()
    n = _n_rows(rays)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device) if hits is None else hits
    _check(load().rr_trace_any(scene.handle, _ptr(rays, "rays", torch.float32), n,
                               _ptr(count, "count", torch.int32, False), _ptr(hits, "hits", torch.float32),
                               _stream(stream)), "rr_trace_any")
    return hits


def rr_trace_profile(scene: Scene, rays, hits=None, stream=None) -> dict:
    """Trace with the profiling counters; synchronises and returns them."""
    torch = _torch()
    n = _n_rows(rays)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device) if hits is None else hits
    st = torch.zeros(8, dtype=torch.int64, device=rays.device)
    _check(load().rr_trace_profile(scene.handle, _ptr(rays, "rays", torch.float32), n,
                                   _ptr(hits, "hits", torch.float32), _ptr(st, "stats", torch.int64),
                                   _stream(stream)), "rr_trace_profile")
    v = [int(x) for x in st.cpu().tolist()]
    keys = ("lane_trips", "wave_trips64", "inner_visits", "leaf_visits", "tri_tests", "rays", "max_stack",
            "spill_pushes")
    out = dict(zip(keys, v))
    out["simd_efficiency"] = v[0] / v[1] if v[1] else 0.0
    return out


def rr_reorder_and_trace(scene: Scene, rays, params: KeyParams, alive=None, flags: int = RR_HITS_ORIGINAL_ORDER,
                         hits=None, perm=None, count=None, ws=None, want_perm: bool = True, want_count: bool = True,
                         stream=None):
    """Keys, sort, gather and trace in one call.  Returns (hits, perm, count);
    perm and count are None when not given and not wanted."""
    torch = _torch()
    L = load()
    n = _n_rows(rays)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device) if hits is None else hits
    if perm is None and want_perm:
        perm = _empty(n, torch.int32, rays.device)
    if count is None and want_count:
        count = _empty(1, torch.int32, rays.device)
    if ws is None:
        ws = workspace(reorder_workspace_size(n, params), rays.device)
    _check(L.rr_reorder_and_trace(scene.handle, _ptr(rays, "rays", torch.float32), n,
                                  _ptr(alive, "alive", torch.uint8, False), ctypes.byref(params),
                                  _ptr(hits, "hits", torch.float32), _ptr(perm, "perm", torch.int32, False),
                                  _ptr(count, "count", torch.int32, False), flags, _ptr(ws, "workspace"),
                                  ws.numel() * ws.element_size(), _stream(stream)), "rr_reorder_and_trace")
    return hits, perm, count


def rr_reorder_and_trace_noalloc(scene: Scene, rays, params: KeyParams, alive=None,
                                 flags: int = RR_HITS_ORIGINAL_ORDER, hits=None, perm=None, count=None,
                                 stream=None):
    """rr_reorder_and_trace with the library's static device workspace (no
    device allocation inside the call); outputs the caller did not pass are
    allocated here, before the call.  Returns (hits, perm, count)."""
    torch = _torch()
    n = _n_rows(rays)
    hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device) if hits is None else hits
    _check(load().rr_reorder_and_trace_noalloc(scene.handle, _ptr(rays, "rays", torch.float32), n,
                                               _ptr(alive, "alive", torch.uint8, False), ctypes.byref(params),
                                               _ptr(hits, "hits", torch.float32),
                                               _ptr(perm, "perm", torch.int32, False),
                                               _ptr(count, "count", torch.int32, False), flags, _stream(stream)),
           "rr_reorder_and_trace_noalloc")
    return hits, perm, count


def coherence_m64(rays, hits, params: KeyParams, stream=None):
    """M^64_CPS of rays in their order (Section 4.3): (per-group areas,
    mean), float64 device tensors."""
    torch = _torch()
    n = _n_rows(rays)
    groups = torch.empty(max(1, (n + 63) // 64), dtype=torch.float64, device=rays.device)
    mean = torch.empty(1, dtype=torch.float64, device=rays.device)
    _check(load().rr_coherence_m64(_ptr(rays, "rays", torch.float32), _ptr(hits, "hits", torch.float32), n,
                                   ctypes.byref(params), groups.data_ptr(), mean.data_ptr(), _stream(stream)),
           "rr_coherence_m64")
    return groups[:(n + 63) // 64], mean


def hits_to_numpy(hits) -> np.ndarray:
    """(N, 4) float32 device tensor -> structured array (t, prim, u, v)."""
    a = np.ascontiguousarray(hits.detach().cpu().numpy(), dtype=np.float32)
    dt = np.dtype([("t", np.float32), ("prim", np.int32), ("u", np.float32), ("v", np.float32)])
    return a.view(dt).reshape(-1)
