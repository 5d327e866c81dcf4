"""ctypes binding of the batched and serving layers (include/rr_batch.h).

Argument marshalling only; the work runs in librr.  A Batch reorders and
traces many wavefronts in one captured graph launch; a Server runs a
continuous-batching request loop over several slots.  The autotuner's
choices can be kept in a small JSON tuning database keyed by device
architecture, key width and batch size bucket.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from typing import Optional, Sequence

from . import rr as _rr
from .rr import KeyParams, _check, _ptr, _stream, load

RR_BATCH_EAGER = 0x100

EXTRA_EXPORTS = (
    "rr_batch_create", "rr_batch_info", "rr_batch_set_config", "rr_batch_run", "rr_batch_autotune",
    "rr_batch_destroy", "rr_server_create", "rr_server_start", "rr_server_submit", "rr_server_wait",
    "rr_server_drain", "rr_server_stats_get", "rr_server_destroy",
)


class Segment(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_void_p), ("hits", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("key", KeyParams)]


RR_TILES_COUNTER = 0
RR_TILES_FIXED = 1


class BatchConfig(ctypes.Structure):
    _fields_ = [("digit_bits", ctypes.c_uint32), ("keys_per_thread", ctypes.c_uint32), ("refill", ctypes.c_uint32),
                ("tile_order", ctypes.c_uint32), ("trace_block", ctypes.c_uint32)]

    @classmethod
    def of(cls, config: dict):
        return cls(config["digit_bits"], config["keys_per_thread"], config["refill"],
                   config.get("tile_order", RR_TILES_COUNTER), config.get("trace_block", 256))

    def as_dict(self):
        return {"digit_bits": self.digit_bits, "keys_per_thread": self.keys_per_thread, "refill": self.refill,
                "tile_order": self.tile_order, "trace_block": self.trace_block}


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_int64), ("max_batch_rays", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int32), ("split_rays", ctypes.c_int64)]


class RequestStats(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("n", ctypes.c_int64), ("status", ctypes.c_int32), ("done", ctypes.c_int32),
                ("arrival_s", ctypes.c_double), ("start_s", ctypes.c_double), ("finish_s", ctypes.c_double),
                ("batch_requests", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("rays", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("mrays_per_s", ctypes.c_double), ("batches", ctypes.c_int64),
                ("peak_inflight_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _bind(L):
    vp, i64, i32, u32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    st = ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "rr_batch_create": ([vp, i64, i32, P(BatchConfig), P(vp)], st),
        "rr_batch_info": ([vp, P(i64), P(BatchConfig)], st),
        "rr_batch_set_config": ([vp, P(BatchConfig)], st),
        "rr_batch_run": ([vp, P(Segment), i32, u32, vp], st),
        "rr_batch_autotune": ([vp, P(Segment), i32, i32, P(BatchConfig), P(ctypes.c_float), vp], st),
        "rr_batch_destroy": ([vp], st),
        "rr_server_create": ([vp, P(ServerConfig), P(vp)], st),
        "rr_server_start": ([vp], st),
        "rr_server_submit": ([vp, vp, i64, P(KeyParams), vp, u32, dbl, P(i64)], st),
        "rr_server_wait": ([vp, i64, dbl, P(RequestStats)], st),
        "rr_server_drain": ([vp, dbl], st),
        "rr_server_stats_get": ([vp, P(ServerStats)], st),
        "rr_server_destroy": ([vp], st),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res


def segment(rays, hits, key: KeyParams, perm=None, n: Optional[int] = None) -> Segment:
    """A segment over device tensors rays (N, 8) and hits (N, 4)."""
    import torch
    s = Segment()
    s.rays = _ptr(rays, "rays", torch.float32)
    s.hits = _ptr(hits, "hits", torch.float32)
    s.perm = _ptr(perm, "perm", torch.int32, False)
    s.n = int(rays.shape[0]) if n is None else int(n)
    s.key = key
    return s


def _segs(segs: Sequence[Segment]):
    arr = (Segment * max(1, len(segs)))(*segs)
    return arr, len(segs)


class Batch:
    def __init__(self, scene, max_rays: int, max_segments: int = 64, config: Optional[dict] = None):
        L = load()
        h = ctypes.c_void_p()
        cfg = None
        if config is not None:
            cfg = BatchConfig.of(config)
        _check(L.rr_batch_create(scene.handle, max_rays, max_segments, ctypes.byref(cfg) if cfg else None,
                                 ctypes.byref(h)), "rr_batch_create")
        self.handle = h
        self.scene = scene  # keeps the scene alive

    def info(self) -> dict:
        b = ctypes.c_int64()
        c = BatchConfig()
        _check(load().rr_batch_info(self.handle, ctypes.byref(b), ctypes.byref(c)), "rr_batch_info")
        return {"device_bytes": b.value, "config": c.as_dict()}

    def set_config(self, config: dict):
        c = BatchConfig.of(config)
        _check(load().rr_batch_set_config(self.handle, ctypes.byref(c)), "rr_batch_set_config")

    def run(self, segs: Sequence[Segment], flags: int = _rr.RR_HITS_ORIGINAL_ORDER, stream=None):
        arr, n = _segs(segs)
        _check(load().rr_batch_run(self.handle, arr, n, flags, _stream(stream)), "rr_batch_run")

    def autotune(self, segs: Sequence[Segment], reps: int = 3, stream=None):
        arr, n = _segs(segs)
        best = BatchConfig()
        ms = ctypes.c_float()
        _check(load().rr_batch_autotune(self.handle, arr, n, reps, ctypes.byref(best), ctypes.byref(ms),
                                        _stream(stream)), "rr_batch_autotune")
        return best.as_dict(), float(ms.value)

    def close(self):
        if getattr(self, "handle", None):
            if _rr._lib is not None:
                _rr._lib.rr_batch_destroy(self.handle)
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


class Server:
    def __init__(self, scene, slots: int = 2, hbm_budget_bytes: int = 32 << 30, max_batch_rays: int = 1 << 23,
                 max_batch_requests: int = 64, split_rays: int = 0):
        L = load()
        h = ctypes.c_void_p()
        cfg = ServerConfig(slots, hbm_budget_bytes, max_batch_rays, max_batch_requests, split_rays)
        _check(L.rr_server_create(scene.handle, ctypes.byref(cfg), ctypes.byref(h)), "rr_server_create")
        self.handle = h
        self.scene = scene
        self._keep = {}

    def start(self):
        _check(load().rr_server_start(self.handle), "rr_server_start")

    def submit(self, rays, hits, key: KeyParams, arrival_s: float = -1.0,
               flags: int = _rr.RR_HITS_ORIGINAL_ORDER, sync: bool = True) -> int:
        """Queues a request.  The server's streams read the rays without
        waiting for the stream that wrote them, so by default the current
        stream is synchronised first (pass sync=False when the rays are
        known to be complete)."""
        import torch
        if sync:
            torch.cuda.current_stream().synchronize()
        rid = ctypes.c_int64()
        _check(load().rr_server_submit(self.handle, _ptr(rays, "rays", torch.float32), int(rays.shape[0]),
                                       ctypes.byref(key), _ptr(hits, "hits", torch.float32),
                                       int(flags), float(arrival_s), ctypes.byref(rid)),
               "rr_server_submit")
        self._keep[rid.value] = (rays, hits)
        return rid.value

    def wait(self, rid: int, timeout_s: float = 60.0) -> dict:
        st = RequestStats()
        _check(load().rr_server_wait(self.handle, rid, timeout_s, ctypes.byref(st)), "rr_server_wait")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def drain(self, timeout_s: float = 120.0):
        _check(load().rr_server_drain(self.handle, timeout_s), "rr_server_drain")

    def stats(self) -> dict:
        s = ServerStats()
        _check(load().rr_server_stats_get(self.handle, ctypes.byref(s)), "rr_server_stats_get")
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            if _rr._lib is not None:
                _rr._lib.rr_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ------------------------------------------------------------ tuning DB

def tuning_db_path() -> str:
    return os.environ.get("RR_TUNING_DB", os.path.join(os.path.expanduser("~"), ".cache", "rr_tuning.json"))


def _bucket(total_rays: int, key_bits: int, arch: str) -> str:
    return f"{arch}/k{key_bits}/n2^{int(round(math.log2(max(total_rays, 1))))}"


def load_tuned(total_rays: int, key_bits: int, arch: str = "gfx950", path: Optional[str] = None) -> Optional[dict]:
    p = path or tuning_db_path()
    try:
        with open(p) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return None
    return db.get(_bucket(total_rays, key_bits, arch))


def save_tuned(total_rays: int, key_bits: int, config: dict, ms: float, arch: str = "gfx950",
               path: Optional[str] = None):
    p = path or tuning_db_path()
    try:
        with open(p) as f:
            db = json.load(f)
    except (OSError, ValueError):
        db = {}
    db[_bucket(total_rays, key_bits, arch)] = dict(config, ms=ms)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, p)
