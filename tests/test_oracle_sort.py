"""Pins of the oracle's ray sort (Sec. 3.3.3-3.3.5).

Compression into chunks of equal keys, a radix sort of the chunks and
decompression yield the ray ids stably ordered by key.  The oracle's result
is checked against numpy's stable argsort and against an explicit
compress / sort-chunks / decompress sequence written here from the paper's
description.
"""
import numpy as np
import pytest

from oracle import oracle as O


def _compress_sort_decompress(keys, ids):
    # head flag where a key differs from its predecessor, chunks from the scan
    n = len(keys)
    head = np.ones(n, bool)
    head[1:] = keys[1:] != keys[:-1]
    base = np.nonzero(head)[0]
    size = np.diff(np.r_[base, n])
    ckey = keys[base]
    order = np.argsort(ckey, kind="stable")      # chunk sort (stable)
    skel = size[order]
    start = np.r_[0, np.cumsum(skel)[:-1]]       # exclusive scan of the skeleton
    out_k = np.empty(n, keys.dtype)
    out_i = np.empty(n, ids.dtype)
    for c, s0 in zip(order, start):
        b, sz = base[c], size[c]
        out_k[s0:s0 + sz] = keys[b:b + sz]
        out_i[s0:s0 + sz] = ids[b:b + sz]
    return out_k, out_i


@pytest.mark.parametrize("n,span", [(0, 1), (1, 1), (1000, 3), (5000, 1 << 32), (20000, 97)])
def test_sort_is_stable_permutation(rng, n, span):
    keys = rng.integers(0, span, size=n, dtype=np.uint64).astype(np.uint32)
    # runs of equal keys, as coherent rays produce
    keys = np.repeat(keys, rng.integers(1, 4, size=n))[:n] if n else keys
    ids = np.arange(len(keys), dtype=np.uint32)
    ks, ix = O.sort_rays(keys, ids)
    ref = np.argsort(keys, kind="stable")
    assert np.array_equal(ix, ref.astype(np.uint32))
    assert np.array_equal(ks, keys[ref])
    assert np.all(np.diff(ks.astype(np.int64)) >= 0)
    ck, ci = _compress_sort_decompress(keys, ids)
    assert np.array_equal(ix, ci) and np.array_equal(ks, ck)


def test_sort_with_arbitrary_values(rng):
    keys = rng.integers(0, 50, size=3000).astype(np.uint32)
    ids = rng.permutation(3000).astype(np.uint32)
    ks, ix = O.sort_rays(keys, ids)
    # equal keys keep their input order, whatever the values are
    o = np.argsort(keys, kind="stable")
    assert np.array_equal(ix, ids[o]) and np.array_equal(ks, keys[o])
    ck, ci = _compress_sort_decompress(keys, ids)
    assert np.array_equal(ix, ci)
