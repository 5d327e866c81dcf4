"""The C-ABI library loads and exports every symbol include/rr.h declares;
host-only argument checks (no device needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for h in ("rr.h", "rr_batch.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        syms |= set(re.findall(r"\b(rr_[a-z_0-9]+)\s*\(", text))
    return sorted(syms)


@pytest.fixture(scope="module")
def lib():
    import paper_2506_11273_amd as rr
    return rr.load()


def test_header_declares_the_path():
    syms = declared_symbols()
    for s in ("rr_compute_keys", "rr_sort", "rr_gather", "rr_trace", "rr_reorder_and_trace", "rr_batch_run",
              "rr_server_submit"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    import paper_2506_11273_amd as rr
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared_symbols()) <= set(rr.EXPORTS) | set(getattr(rr, "EXTRA_EXPORTS", ()))


def test_status_strings(lib):
    assert lib.rr_status_string(0) == b"ok"
    assert lib.rr_status_string(-5) == b"workspace too small"


def test_workspace_queries_are_host_only(lib):
    import paper_2506_11273_amd as rr
    b = ctypes.c_size_t()
    assert lib.rr_sort_workspace_size(1000, 32, ctypes.byref(b)) == 0 and b.value > 1000 * 8
    big = ctypes.c_size_t()
    assert lib.rr_sort_workspace_size(1000, 64, ctypes.byref(big)) == 0 and big.value > b.value
    assert lib.rr_sort_workspace_size(1000, 48, ctypes.byref(b)) == rr.rr.RR_ERR_INVALID_ARGUMENT
    assert lib.rr_sort_workspace_size(-1, 32, ctypes.byref(b)) == rr.rr.RR_ERR_INVALID_ARGUMENT
    assert lib.rr_sort_workspace_size(1 << 30, 32, ctypes.byref(b)) == rr.rr.RR_ERR_INVALID_ARGUMENT
    assert lib.rr_keys_workspace_size(0, ctypes.byref(b)) == 0
    p = rr.key_params(rr.RR_KEY_ORIGIN_TERMINATION, 64, (0, 0, 0), (1, 1, 1))
    assert lib.rr_reorder_workspace_size(5000, ctypes.byref(p), ctypes.byref(b)) == 0
    assert b.value > 5000 * (8 + 4 + 32 + 16)
    bad = rr.key_params(7, 64, (0, 0, 0), (1, 1, 1))
    assert lib.rr_reorder_workspace_size(5000, ctypes.byref(bad), ctypes.byref(b)) == 0  # kind checked at call


def test_rejects_bad_arguments_before_touching_the_device(lib):
    import paper_2506_11273_amd as rr
    p = rr.key_params(rr.RR_KEY_ORIGIN_DIRECTION, 32, (0, 0, 0), (1, 1, 1))
    # negative n, bad key width, unsupported origin split: all rejected on the host
    assert lib.rr_compute_keys(None, -1, None, ctypes.byref(p), None, None, None, None, 0, None) == -1
    q = rr.key_params(rr.RR_KEY_ORIGIN_DIRECTION, 48, (0, 0, 0), (1, 1, 1))
    assert lib.rr_compute_keys(None, 10, None, ctypes.byref(q), None, None, None, None, 0, None) == -1
    q = rr.key_params(rr.RR_KEY_ORIGIN_DIRECTION, 64, (0, 0, 0), (1, 1, 1), origin_bits=64)
    assert lib.rr_compute_keys(None, 10, None, ctypes.byref(q), None, None, None, None, 0, None) == -4
    q = rr.key_params(rr.RR_KEY_NONE, 32, (0, 0, 0), (1, 1, 1))
    assert lib.rr_compute_keys(None, 10, None, ctypes.byref(q), None, None, None, None, 0, None) == -1
    # unsupported sort configuration
    assert lib.rr_sort_ex(None, None, 10, None, 32, 6, 16, None, 0, None) == -4
    assert lib.rr_sort_ex(None, None, 10, None, 32, 8, 12, None, 0, None) == -4
    # empty sort is a no-op
    assert lib.rr_sort(None, None, 0, None, 32, None, 0, None) == 0
    # the most-significant-digit sort: 64-bit keys below 2^27 only
    assert lib.rr_sort_msd(None, None, 0, None, 64, None, 0, None) == 0
    assert lib.rr_sort_msd(None, None, 10, None, 32, None, 0, None) == -4
    assert lib.rr_sort_msd(None, None, 1 << 27, None, 64, None, 0, None) == -4
    assert lib.rr_sort_msd(None, None, 10, None, 48, None, 0, None) == -1
    # scene from no triangles / non-finite vertices
    h = ctypes.c_void_p()
    assert lib.rr_scene_create(None, 0, ctypes.byref(h)) == -1
    import numpy as np
    t = np.zeros((1, 9), np.float32)
    t[0, 4] = np.nan
    assert lib.rr_scene_create(t.ctypes.data, 1, ctypes.byref(h)) == -1
