"""Oracle for the first stage of geometry-aware matching (Sec. 3.1) -- TEST
INFRASTRUCTURE ONLY.

ctypes wrapper over geometry_oracle.c (compiled into the same library as the
matching oracle), plus the two-stage pipeline written out with the plain
matching oracle:

  1. subset    top-scale fifth of every image (top_scale)
  2. stage 1   CasHash matching of the subsets over the given pairs; the
               subsets' codes and keys are rows of the full set's (the
               projection is centred on the whole set, Sec. 2.1)
  3. geometry  RANSAC fundamental matrix from each pair's stage-1 matches
  4. stage 2   epipolar-guided matching (Eq. 1-2) of all features of the
               accepted pairs with the estimated matrix

Parity status: pinned (see tests/test_geometry_oracle.py).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _c, _ptr, lib as _base_lib, match_pairs

ACCEPT, FEW_MATCHES, DEGENERATE, FEW_INLIERS = 0, 1, 2, 3
MIN_MATCHES = 16

_ready = False


def _lib():
    global _ready
    L = _base_lib()
    if not _ready:
        P, I32, D = C.c_void_p, C.c_int32, C.c_double
        L.oracle_subset_size.argtypes = [I32, I32, I32]
        L.oracle_subset_size.restype = I32
        L.oracle_top_scale.argtypes = [P, I32, I32, P]
        L.oracle_top_scale.restype = None
        L.oracle_floyd8.argtypes = [P, I32, P]
        L.oracle_floyd8.restype = None
        L.oracle_jacobi.argtypes = [I32, P, P, I32]
        L.oracle_jacobi.restype = None
        L.oracle_null8.argtypes = [P, P]
        L.oracle_null8.restype = I32
        L.oracle_rank2.argtypes = [P]
        L.oracle_rank2.restype = None
        L.oracle_is_inlier.argtypes = [P, P, P, D]
        L.oracle_is_inlier.restype = I32
        L.oracle_fundamental.argtypes = [P, P, I32, P, I32, D, I32, P, P, P]
        L.oracle_fundamental.restype = I32
        L.oracle_fundamental_batch.argtypes = [I32, P, P, P, P, I32, D, I32, P, P, P, P]
        L.oracle_fundamental_batch.restype = None
        _ready = True
    return L


def subset_size(n: int, frac=(1, 5)) -> int:
    return int(_lib().oracle_subset_size(int(n), int(frac[0]), int(frac[1])))


def top_scale(scale, frac=(1, 5)) -> np.ndarray:
    """Indices of the ceil(n * frac) largest scales, ascending."""
    s = _c(scale, np.float32).reshape(-1)
    m = subset_size(len(s), frac)
    rows = np.zeros(m, np.int32)
    _lib().oracle_top_scale(_ptr(s), len(s), m, _ptr(rows))
    return rows


def floyd8(r, n: int) -> np.ndarray:
    r = _c(r, np.uint32).reshape(8)
    if n < 8:
        raise ValueError("need n >= 8")
    out = np.zeros(8, np.int32)
    _lib().oracle_floyd8(_ptr(r), int(n), _ptr(out))
    return out


def jacobi(A, sweeps: int):
    """Cyclic Jacobi on a symmetric matrix: (rotated A, accumulated V)."""
    A = np.array(A, np.float64, order="C")
    n = A.shape[0]
    V = np.eye(n)
    _lib().oracle_jacobi(n, _ptr(A), _ptr(V), int(sweeps))
    return A, V


def null8(A):
    """Null vector (f[8] = 1) of an 8 x 9 matrix, or None if a pivot is 0."""
    A = np.array(A, np.float64, order="C").reshape(8, 9)
    f = np.zeros(9)
    ok = _lib().oracle_null8(_ptr(A), _ptr(f))
    return f if ok else None


def rank2(F):
    F = np.array(F, np.float64, order="C").reshape(9)
    _lib().oracle_rank2(_ptr(F))
    return F


def is_inlier(F, q, t, thr: float) -> bool:
    F = _c(F, np.float64).reshape(9)
    q, t = _c(q, np.float32).reshape(2), _c(t, np.float32).reshape(2)
    return bool(_lib().oracle_is_inlier(_ptr(F), _ptr(q), _ptr(t), float(thr)))


def fundamental(q_pts, t_pts, rand, thr=2.0, min_matches=MIN_MATCHES):
    """One pair.  Returns (status, F[9], n_inliers, best_hypothesis)."""
    q, t = _c(q_pts, np.float32).reshape(-1, 2), _c(t_pts, np.float32).reshape(-1, 2)
    assert q.shape == t.shape
    r = _c(rand, np.uint32).reshape(-1, 8)
    F = np.zeros(9)
    ni, bh = C.c_int32(0), C.c_int32(0)
    st = _lib().oracle_fundamental(_ptr(q), _ptr(t), len(q), _ptr(r), len(r), float(thr), int(min_matches),
                                   _ptr(F), C.byref(ni), C.byref(bh))
    return int(st), F, int(ni.value), int(bh.value)


def fundamental_batch(q_list, t_list, rand, thr=2.0, min_matches=MIN_MATCHES):
    """Many pairs (OpenMP).  Returns (status, F[P, 9], n_inliers, best_h)."""
    n = np.array([len(a) for a in q_list], np.int64)
    off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    q = _c(np.concatenate([np.asarray(a, np.float32).reshape(-1, 2) for a in q_list]) if len(q_list)
           else np.zeros((0, 2)), np.float32)
    t = _c(np.concatenate([np.asarray(a, np.float32).reshape(-1, 2) for a in t_list]) if len(t_list)
           else np.zeros((0, 2)), np.float32)
    r = _c(rand, np.uint32).reshape(-1, 8)
    P = len(q_list)
    F = np.zeros((P, 9))
    ni = np.zeros(P, np.int32)
    bh = np.zeros(P, np.int32)
    st = np.zeros(P, np.int32)
    _lib().oracle_fundamental_batch(P, _ptr(q), _ptr(t), _ptr(off), _ptr(r), len(r), float(thr),
                                    int(min_matches), _ptr(F), _ptr(ni), _ptr(bh), _ptr(st))
    return st, F, ni, bh


def stage1_points(kp_q, kp_t, match_idx):
    """Matched keypoints of one pair in ascending query order."""
    m = np.asarray(match_idx)
    q = np.flatnonzero(m >= 0)
    return np.asarray(kp_q)[q], np.asarray(kp_t)[m[q]]


def geometric_match(images, codes, keys, kp, scales, pairs, rand, k=10, ratio=(4, 5), frac=(1, 5),
                    thr=2.0, min_matches=MIN_MATCHES, max_px=4.0):
    """The two-stage pipeline.  Returns a dict with the subsets' rows, the
    stage-1 outputs, per-pair status / F / inlier counts, and the stage-2
    outputs of the accepted pairs (in pair order)."""
    pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
    rows = [top_scale(s, frac) for s in scales]
    sub = lambda arrs: [np.ascontiguousarray(np.asarray(a)[r]) for a, r in zip(arrs, rows)]
    s_img, s_codes, s_keys, s_kp = sub(images), sub(codes), sub(keys), sub(kp)
    m1 = match_pairs(s_img, s_codes, s_keys, pairs, k=k, ratio=ratio)
    nq = np.array([len(r) for r in rows], np.int64)[pairs[:, 0]]
    off = np.concatenate([[0], np.cumsum(nq)])
    ql, tl = [], []
    for p, (qi, ti) in enumerate(pairs):
        a, b = stage1_points(s_kp[qi], s_kp[ti], m1[0][off[p]:off[p + 1]])
        ql.append(a)
        tl.append(b)
    st, F, ni, bh = fundamental_batch(ql, tl, rand, thr, min_matches)
    acc = np.flatnonzero(st == ACCEPT)
    if len(acc):
        m2 = match_pairs(images, codes, keys, pairs[acc], k=k, ratio=ratio, kp=kp, F=F[acc], max_px=max_px)
    else:
        m2 = tuple(np.zeros(0, np.int32) for _ in range(3))
    return dict(rows=rows, stage1=m1, n_matches=np.array([len(a) for a in ql], np.int32), status=st, F=F,
                n_inliers=ni, best_h=bh, accepted=acc, stage2=m2)
