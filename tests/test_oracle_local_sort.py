"""Pins for the oracle's block-wise (local) sort of Section 3.2: every run of
`block` consecutive pairs is sorted on its own.

Pins: brute force (Python's sorted() on (key, position) tuples) per block;
one block covering everything equals the global sort; equal keys leave every
block in input order; each block keeps its own multiset of pairs."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("n,block", [(1, 1024), (1000, 1024), (5000, 1024), (5000, 2048), (9000, 4096)])
def test_blocks_match_brute_force(n, block):
    rng = np.random.default_rng(n + block)
    k = rng.integers(0, 64, n).astype(np.uint32)          # many ties
    idx = np.arange(n, dtype=np.uint32) * 3 + 7            # ascending, not positions
    ko, io = O.local_sort_pairs(k, idx, block)
    for b in range(0, n, block):
        want = sorted(zip(k[b:b + block].tolist(), range(b, min(n, b + block))))
        assert ko[b:b + block].tolist() == [x for x, _ in want]
        assert io[b:b + block].tolist() == [int(idx[p]) for _, p in want]


def test_one_block_is_the_global_sort_and_ties_keep_order():
    rng = np.random.default_rng(1)
    k = rng.integers(0, 1 << 63, 3000, dtype=np.uint64)
    assert all(np.array_equal(a, b) for a, b in zip(O.local_sort_pairs(k, block=4096), O.sort_pairs(k)))
    ko, io = O.local_sort_pairs(np.zeros(5000, np.uint32), block=1024)
    assert np.array_equal(io, np.arange(5000, dtype=np.uint32))


def test_blocks_keep_their_pairs():
    rng = np.random.default_rng(2)
    k = rng.integers(0, 1 << 32, 10000, dtype=np.uint64).astype(np.uint32)
    ko, io = O.local_sort_pairs(k, block=2048)
    for b in range(0, 10000, 2048):
        assert np.all(np.diff(ko[b:b + 2048].astype(np.int64)) >= 0)
        assert sorted(io[b:b + 2048].tolist()) == list(range(b, min(10000, b + 2048)))
        assert np.array_equal(k[io[b:b + 2048]], ko[b:b + 2048])
