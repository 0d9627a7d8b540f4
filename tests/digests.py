"""Per-pair and per-image digests of matching outputs and hash codes.

Used by tests/golden/make_fullsize_digests.py (which writes the oracle's
digests of the full-size workloads) and by the full-size GPU tests (which
digest the GPU's outputs the same way and compare every pair).  A digest is
the first 8 bytes of BLAKE2b over the raw little-endian bytes, read as a
little-endian uint64; it holds none of the matching method's arithmetic.
"""
from __future__ import annotations

import hashlib
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _h(*arrs) -> int:
    h = hashlib.blake2b(digest_size=8)
    for a in arrs:
        h.update(np.ascontiguousarray(a).tobytes())
    return int.from_bytes(h.digest(), "little")


def pair_offsets(n_feat, pairs) -> np.ndarray:
    """First output slot of every pair (flat layout over pairs) and the end."""
    nq = np.asarray(n_feat, np.int64)[np.asarray(pairs)[:, 0]] if len(pairs) else np.zeros(0, np.int64)
    return np.concatenate([[0], np.cumsum(nq)]).astype(np.int64)


def pair_digests(match_idx, d1sq, d2sq, offsets, threads: int = 8) -> np.ndarray:
    """uint64 digest of (match_idx, d1sq, d2sq) of every pair's slots."""
    a = [np.asarray(x, np.int32) for x in (match_idx, d1sq, d2sq)]
    n = len(offsets) - 1

    def one(p):
        lo, hi = offsets[p], offsets[p + 1]
        return _h(a[0][lo:hi], a[1][lo:hi], a[2][lo:hi])

    with ThreadPoolExecutor(threads) as ex:
        return np.fromiter(ex.map(one, range(n), chunksize=256), np.uint64, n)


def code_digests(codes, keys) -> np.ndarray:
    """uint64 digest of (codes uint64 [n, 2], keys uint8 [n, 6]) per image."""
    return np.fromiter((_h(np.asarray(c, np.uint64), np.asarray(k, np.uint8)) for c, k in zip(codes, keys)),
                       np.uint64, len(codes))
