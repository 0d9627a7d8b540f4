"""CPU oracle for CasHash pairwise matching -- TEST INFRASTRUCTURE ONLY.

A plain C statement of the method (cashash_oracle.c) with a ctypes wrapper.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
it; the GPU library never imports, links or calls anything here.

Parity status per function (what pins each one is in tests/test_oracle_pins.py):
  column_sums, project, build_codes  -- pinned (closed forms, numpy float64
                                        signs, power-of-two scaling, hand codes)
  match_pair, match_pairs            -- pinned (exhaustive brute force when k
                                        covers every candidate, self-matching,
                                        ratio boundary, hand-built Hamming
                                        order, golden worked example)
  epipolar band                      -- pinned (rectified-stereo closed form,
                                        huge band equals plain matching)
  geometry (oracle.geometry)         -- pinned (see geometry_oracle.c)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cashash_oracle.c")
_SRC_GEO = os.path.join(_HERE, "geometry_oracle.c")
LIB_PATH = os.path.join(_HERE, "libcashash_oracle.so")
DIM, TABLES = 128, 6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no fp contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp",
                        "-shared", "-fPIC", "-o", tmp, _SRC, _SRC_GEO, "-lm"], check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("ratio_num", C.c_int32), ("ratio_den", C.c_int32),
                ("tau", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
                os.path.getmtime(_SRC), os.path.getmtime(_SRC_GEO)):
            build()
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.oracle_column_sums.argtypes = [I32, P, P, P, P]
        L.oracle_project.argtypes = [P, I64, P, I64, P, P, P, P]
        L.oracle_build_codes.argtypes = [I32, P, P, P, P, P, P]
        L.oracle_match_pair.argtypes = [P, P, P, I32, P, P, P, I32, P, P, P, P, D, P, I32, P, P, P]
        L.oracle_match_pairs.argtypes = [I32, P, P, P, P, I64, P, P, P, P, D, P, P, P]
        L.oracle_num_threads.restype = I32
        for f in ("oracle_column_sums", "oracle_project", "oracle_build_codes",
                  "oracle_match_pair", "oracle_match_pairs"):
            getattr(L, f).restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _ptr_array(arrs):
    return (C.c_void_p * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def column_sums(images):
    images = [_c(im, np.uint8) for im in images]
    nf = np.array([im.shape[0] for im in images], np.int32)
    S = np.zeros(DIM, np.int64)
    n = np.zeros(1, np.int64)
    lib().oracle_column_sums(len(images), _ptr_array(images), _ptr(nf), _ptr(S), _ptr(n))
    return S, int(n[0])


def project(x, S, n_tot, r_code, r_bucket):
    x = _c(x, np.uint8).reshape(-1, DIM)
    S = _c(S, np.int64)
    r_code, r_bucket = _c(r_code, np.float64), _c(r_bucket, np.float64)
    assert r_code.shape == (128, DIM) and r_bucket.shape == (TABLES, 8, DIM)
    codes = np.zeros((x.shape[0], 2), np.uint64)
    keys = np.zeros((x.shape[0], TABLES), np.uint8)
    lib().oracle_project(_ptr(x), x.shape[0], _ptr(S), int(n_tot), _ptr(r_code), _ptr(r_bucket),
                         _ptr(codes), _ptr(keys))
    return codes, keys


def build_codes(images, r_code, r_bucket):
    images = [_c(im, np.uint8).reshape(-1, DIM) for im in images]
    nf = np.array([im.shape[0] for im in images], np.int32)
    r_code, r_bucket = _c(r_code, np.float64), _c(r_bucket, np.float64)
    codes = [np.zeros((n, 2), np.uint64) for n in nf]
    keys = [np.zeros((n, TABLES), np.uint8) for n in nf]
    lib().oracle_build_codes(len(images), _ptr_array(images), _ptr(nf), _ptr(r_code), _ptr(r_bucket),
                             _ptr_array(codes), _ptr_array(keys))
    return codes, keys


def _params(k, ratio, tau):
    if not 1 <= k <= 64:
        raise ValueError("k must be in 1..64")
    return _Params(int(k), int(ratio[0]), int(ratio[1]), int(tau))


def match_pair(desc_q, codes_q, keys_q, desc_t, codes_t, keys_t, k=10, ratio=(4, 5), tau=128,
               kp_q=None, kp_t=None, F=None, max_px=4.0, q_idx=None):
    """Match queries of Q against T.  Returns (match_idx, d1sq, d2sq), int32."""
    dq, dt = _c(desc_q, np.uint8).reshape(-1, DIM), _c(desc_t, np.uint8).reshape(-1, DIM)
    cq, ct = _c(codes_q, np.uint64).reshape(-1, 2), _c(codes_t, np.uint64).reshape(-1, 2)
    kq, kt = _c(keys_q, np.uint8).reshape(-1, TABLES), _c(keys_t, np.uint8).reshape(-1, TABLES)
    prm = _params(k, ratio, tau)
    qi = None if q_idx is None else _c(q_idx, np.int32)
    if qi is not None and len(qi) and (qi.min() < 0 or qi.max() >= dq.shape[0]):
        raise ValueError("query index out of range")
    n = dq.shape[0] if qi is None else len(qi)
    out = [np.zeros(n, np.int32) for _ in range(3)]
    epi = kp_q is not None
    if epi:
        kp_q, kp_t, F = _c(kp_q, np.float32), _c(kp_t, np.float32), _c(F, np.float64).reshape(9)
    lib().oracle_match_pair(
        _ptr(dq), _ptr(cq), _ptr(kq), dq.shape[0], _ptr(dt), _ptr(ct), _ptr(kt), dt.shape[0],
        C.byref(prm), _ptr(kp_q) if epi else None, _ptr(kp_t) if epi else None,
        _ptr(F) if epi else None, float(max_px),
        _ptr(qi) if qi is not None else None, n, _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
    return tuple(out)


def match_pairs(images, codes, keys, pairs, k=10, ratio=(4, 5), tau=128, kp=None, F=None, max_px=4.0):
    """All queries of every (query, train) pair; flat outputs in pair order."""
    images = [_c(im, np.uint8).reshape(-1, DIM) for im in images]
    codes = [_c(c, np.uint64).reshape(-1, 2) for c in codes]
    keys = [_c(c, np.uint8).reshape(-1, TABLES) for c in keys]
    nf = np.array([im.shape[0] for im in images], np.int32)
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    if len(pairs) and (pairs.min() < 0 or pairs.max() >= len(images)):
        raise ValueError("pair index out of range")
    prm = _params(k, ratio, tau)
    n = int(nf[pairs[:, 0]].sum()) if len(pairs) else 0
    out = [np.zeros(n, np.int32) for _ in range(3)]
    epi = kp is not None
    if epi:
        kp = [_c(a, np.float32).reshape(-1, 2) for a in kp]
        F = _c(F, np.float64).reshape(-1, 9)
    lib().oracle_match_pairs(
        len(images), _ptr_array(images), _ptr_array(codes), _ptr_array(keys), _ptr(nf),
        len(pairs), _ptr(pairs), C.byref(prm), _ptr_array(kp) if epi else None,
        _ptr(F) if epi else None, float(max_px), _ptr(out[0]), _ptr(out[1]), _ptr(out[2]))
    return tuple(out)
