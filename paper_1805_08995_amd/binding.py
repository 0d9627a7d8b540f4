"""ctypes binding of libcashash.so (include/cashash.h), argument marshalling only.

Every step of the matching path runs in the library's HIP kernels.  PyTorch
supplies device memory (tensors whose data pointers are passed through) and
the stream: torch's current stream when the Matcher is made.  For torch's
default stream (handle 0) the library runs on a stream of its own that waits,
at every call, for the work already queued on the default stream.  In
host-memory mode numpy arrays are passed and the library streams them to the
device itself.

The library must have been built (``python -m paper_1805_08995_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcashash.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_UNSAFE_MATRIX, E_LIMIT, E_IO = 0, -1, -2, -3, -4, -5, -6
MODE_BATCHED_BF16X2, MODE_PLAIN_FP32_PER_PAIR = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
MODES = {"batched": MODE_BATCHED_BF16X2, "plain": MODE_PLAIN_FP32_PER_PAIR}
MEMS = {"host": MEM_HOST, "device": MEM_DEVICE}
EXPORTED = ["cashash_default_config", "cashash_create", "cashash_set_config", "cashash_destroy",
            "cashash_build_codes", "cashash_match_pairs", "cashash_match_pairs_epipolar",
            "cashash_last_error", "cashash_plan_schedule", "cashash_last_kernel_ms",
            "cashash_default_geometric_config", "cashash_subset_size", "cashash_select_top_scale",
            "cashash_gather_rows", "cashash_estimate_fundamental", "cashash_match_pairs_geometric",
            "cashash_last_geometric_ms", "cashash_set_write", "cashash_build_codes_disk",
            "cashash_match_pairs_disk", "cashash_match_pairs_noalloc"]
NOALLOC_SCRATCH_BYTES = 32 << 20
GEO_ACCEPT, GEO_FEW_MATCHES, GEO_DEGENERATE, GEO_FEW_INLIERS = 0, 1, 2, 3
GEO_MAX_MATCHES = 8192


class Config(C.Structure):
    _fields_ = [("k", C.c_int32), ("ratio_num", C.c_int32), ("ratio_den", C.c_int32),
                ("max_hamming", C.c_int32), ("margin_coef", C.c_double), ("mode", C.c_int32),
                ("mem", C.c_int32), ("device_budget_bytes", C.c_int64), ("stream", C.c_void_p)]


class Images(C.Structure):
    _fields_ = [("n_images", C.c_int32), ("desc", C.POINTER(C.c_void_p)), ("n_feat", C.POINTER(C.c_int32))]


class Stats(C.Structure):
    _fields_ = [("pairs", C.c_int64), ("queries", C.c_int64), ("bucket_entries", C.c_int64),
                ("union_size", C.c_int64), ("ranked", C.c_int64), ("near_margin_recomputes", C.c_int64),
                ("h2d_bytes", C.c_int64), ("d2h_bytes", C.c_int64), ("image_loads", C.c_int64),
                ("tile_queries", C.c_int64), ("blocks_per_cu", C.c_int64), ("graph_replayed", C.c_int64),
                ("ms_codes", C.c_double), ("ms_match", C.c_double), ("disk_bytes", C.c_int64),
                ("group_loads", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GeoConfig(C.Structure):
    _fields_ = [("frac_num", C.c_int32), ("frac_den", C.c_int32), ("min_matches", C.c_int32),
                ("n_hyp", C.c_int32), ("ransac_px", C.c_double), ("band_px", C.c_double),
                ("rand8", C.c_void_p)]


class CashashError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cashash error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libcashash.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_08995_amd.build` "
                              "(hipcc --offload-arch=gfx950); there is no fallback implementation")
        L = C.CDLL(LIB_PATH)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.cashash_default_config.argtypes = [C.POINTER(Config)]
        L.cashash_default_config.restype = None
        L.cashash_create.argtypes = [C.POINTER(C.c_void_p), P, P, C.POINTER(Config)]
        L.cashash_set_config.argtypes = [P, C.POINTER(Config)]
        L.cashash_destroy.argtypes = [P]
        L.cashash_destroy.restype = None
        L.cashash_build_codes.argtypes = [P, C.POINTER(Images), P, P, C.POINTER(Stats)]
        L.cashash_match_pairs.argtypes = [P, C.POINTER(Images), P, P, I64, P, P, P, P, C.POINTER(Stats)]
        L.cashash_match_pairs_epipolar.argtypes = [P, C.POINTER(Images), P, P, P, I64, P, P, C.c_double,
                                                   P, P, P, C.POINTER(Stats)]
        L.cashash_match_pairs_noalloc.argtypes = [P, C.POINTER(Images), P, P, I64, P, P, P, P, C.POINTER(Stats)]
        L.cashash_last_error.restype = C.c_char_p
        L.cashash_plan_schedule.argtypes = [I32, P, I64, P, I64, P, P, P, P, P, I64, P]
        L.cashash_last_kernel_ms.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.cashash_default_geometric_config.argtypes = [C.POINTER(GeoConfig)]
        L.cashash_default_geometric_config.restype = None
        L.cashash_subset_size.argtypes = [I32, I32, I32]
        L.cashash_subset_size.restype = I64
        L.cashash_select_top_scale.argtypes = [P, I32, P, P, I32, I32, P]
        L.cashash_gather_rows.argtypes = [P, I32, P, P, P, P, P, P, P, P, P, P, P]
        L.cashash_estimate_fundamental.argtypes = [P, I32, P, P, I64, P, P, P, I32, C.c_double, I32,
                                                   P, P, P, P, P]
        L.cashash_match_pairs_geometric.argtypes = [P, C.POINTER(Images), P, P, P, P, I64, P, C.POINTER(GeoConfig),
                                                    P, P, P, P, P, P, P, C.POINTER(Stats)]
        L.cashash_last_geometric_ms.argtypes = [P, P]
        L.cashash_set_write.argtypes = [C.c_char_p, C.POINTER(Images), P]
        L.cashash_build_codes_disk.argtypes = [P, C.c_char_p, C.c_char_p, I64, C.POINTER(Stats)]
        L.cashash_match_pairs_disk.argtypes = [P, C.c_char_p, C.c_char_p, I64, P, C.c_char_p, C.c_char_p, I64, I64,
                                               C.POINTER(C.c_int64), C.POINTER(Stats)]
        for f in ("cashash_create", "cashash_set_config", "cashash_build_codes", "cashash_match_pairs",
                  "cashash_match_pairs_noalloc",
                  "cashash_match_pairs_epipolar", "cashash_plan_schedule", "cashash_last_kernel_ms",
                  "cashash_select_top_scale", "cashash_gather_rows", "cashash_estimate_fundamental",
                  "cashash_match_pairs_geometric", "cashash_last_geometric_ms", "cashash_set_write",
                  "cashash_build_codes_disk", "cashash_match_pairs_disk"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        raise CashashError(rc, lib().cashash_last_error().decode())
    return rc


def default_config() -> Config:
    c = Config()
    lib().cashash_default_config(C.byref(c))
    return c


class Bound:
    """A list of buffers of one kind (images, codes, keys, keypoints, ...)
    marshalled once: the pointer array the library takes and the row counts.
    For repeated calls on the same buffers (Matcher.bind); the buffers are
    held here and must not be resized or moved while it is in use."""

    def __init__(self, arrs, ptrs, n):
        self.arrs, self.ptrs, self.n = arrs, ptrs, n

    def __len__(self):
        return len(self.arrs)

    def __getitem__(self, i):
        return self.arrs[i]

    def __iter__(self):
        return iter(self.arrs)


def _rows(arrs):
    if isinstance(arrs, Bound):
        return arrs.n
    return np.fromiter((int(a.shape[0]) for a in arrs), np.int32, len(arrs))


def _n_queries(images, pairs):
    """Total queries of a pair list (the sum of its query images' sizes).
    Out-of-range indices are clipped here and rejected by the library."""
    if not len(pairs):
        return 0
    nf = _rows(images).astype(np.int64)
    return int(np.take(nf, pairs[:, 0], mode="clip").sum()) if len(nf) else 0


def _ptrs(vals):
    return (C.c_void_p * max(1, len(vals)))(*vals)


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _dptr(t):
    return t.data_ptr() if t.numel() else None


def plan_schedule(img_bytes, pairs, slot_bytes, max_steps=None):
    """Host-side block schedule (no device needed).  Returns a dict with the
    step list [(bi, bk, begin, end)], visiting order and load counts."""
    img_bytes = np.ascontiguousarray(img_bytes, np.int64)
    pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    out = [C.c_int64() for _ in range(4)]
    n_max = max_steps if max_steps is not None else max(1, 2 * len(pairs) + 1)
    steps = np.zeros((n_max, 4), np.int64)
    order = np.zeros(max(1, len(pairs)), np.int64)
    check(lib().cashash_plan_schedule(len(img_bytes), img_bytes.ctypes.data, len(pairs),
                                      pairs.ctypes.data if len(pairs) else None, int(slot_bytes),
                                      *[C.byref(o) for o in out], steps.ctypes.data, n_max,
                                      order.ctypes.data))
    n_steps = out[0].value
    return {"steps": steps[:min(n_steps, n_max)], "n_steps": n_steps, "n_blocks": out[1].value,
            "block_loads": out[2].value, "image_loads": out[3].value, "order": order[:len(pairs)]}


class Matcher:
    """A library context.  mem="device": images/codes/outputs are torch CUDA
    tensors; mem="host": numpy arrays, streamed by the library."""

    def __init__(self, r_code=None, r_bucket=None, *, k=10, ratio=(4, 5), max_hamming=128,
                 margin_coef=1e-3, mode="batched", mem="device", device_budget_bytes=0, stream=None):
        if r_code is None or r_bucket is None:
            r_code, r_bucket = synth.projection_matrices()
        self.r_code = np.ascontiguousarray(r_code, np.float64)
        self.r_bucket = np.ascontiguousarray(r_bucket, np.float64)
        if self.r_code.shape != (128, 128) or self.r_bucket.shape != (6, 8, 128):
            raise ValueError("projection matrices must be [128,128] and [6,8,128]")
        self.cfg = default_config()
        self.cfg.k, self.cfg.ratio_num, self.cfg.ratio_den = int(k), int(ratio[0]), int(ratio[1])
        self.cfg.max_hamming, self.cfg.margin_coef = int(max_hamming), float(margin_coef)
        self.cfg.mode, self.cfg.mem = MODES[mode], MEMS[mem]
        self.cfg.device_budget_bytes = int(device_budget_bytes)
        self.mem = mem
        if mem == "device" and stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self.cfg.stream = stream
        h = C.c_void_p()
        check(lib().cashash_create(C.byref(h), self.r_code.ctypes.data, self.r_bucket.ctypes.data,
                                   C.byref(self.cfg)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().cashash_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, mode):
        self.cfg.mode = MODES[mode]
        check(lib().cashash_set_config(self.h, C.byref(self.cfg)))

    def last_kernel_ms(self):
        ms, n = C.c_double(), C.c_int64()
        check(lib().cashash_last_kernel_ms(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    # ------------------------------------------------------------ marshalling
    def bind(self, arrs, dtype=None):
        """Marshal a list of buffers once for repeated calls (see Bound).  In
        host mode the arrays are made contiguous (dtype if given) first."""
        arrs = list(arrs)
        if self.mem != "device":
            arrs = [np.ascontiguousarray(a, dtype) if dtype is not None else np.ascontiguousarray(a) for a in arrs]
        return Bound(arrs, self._arrays(arrs), _rows(arrs))

    def _images(self, images):
        if isinstance(images, Bound):
            ptrs, nf = images.ptrs, images.n
        else:
            nf = _rows(images)
            if self.mem == "device":
                ptrs = _ptrs([_dptr(im) for im in images])
            else:
                images = [np.ascontiguousarray(im, np.uint8) for im in images]
                ptrs = _ptrs([im.ctypes.data if im.size else None for im in images])
        st = Images(len(images), C.cast(ptrs, C.POINTER(C.c_void_p)), nf.ctypes.data_as(C.POINTER(C.c_int32)))
        return st, (ptrs, nf, images)

    def _arrays(self, arrs):
        if isinstance(arrs, Bound):
            return arrs.ptrs
        if self.mem == "device":
            return _ptrs([_dptr(a) for a in arrs])
        return _ptrs([a.ctypes.data if a.size else None for a in arrs])

    def _alloc(self, n, shape_tail, dtype):
        if self.mem == "device":
            import torch
            tdt = {np.uint64: torch.int64, np.uint8: torch.uint8, np.int32: torch.int32}[dtype]
            return torch.empty((n, *shape_tail), dtype=tdt, device="cuda")
        return np.zeros((n, *shape_tail), dtype)

    def build_codes(self, images, out=None):
        """Codes [n,2] (uint64 bits; int64 tensors on the device) and keys [n,6]
        of every image, centred on the mean of the whole set.  out=(codes,
        keys) reuses caller buffers of those shapes."""
        st, keep = self._images(images)
        if out is not None:
            codes, keys = out
        else:
            codes = [self._alloc(int(im.shape[0]), (2,), np.uint64) for im in images]
            keys = [self._alloc(int(im.shape[0]), (6,), np.uint8) for im in images]
        stats = Stats()
        check(lib().cashash_build_codes(self.h, C.byref(st), self._arrays(codes), self._arrays(keys),
                                        C.byref(stats)))
        return codes, keys, stats.as_dict()

    def _outputs(self, n, out):
        if out is not None:
            return out
        return tuple(self._alloc(n, (), np.int32) for _ in range(3))

    def match_pairs(self, images, codes, keys, pairs, out=None):
        """(match_idx, d1sq, d2sq), flat over pairs in pair order."""
        st, keep = self._images(images)
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        n = _n_queries(images, pairs)
        o = self._outputs(n, out)
        stats = Stats()
        check(lib().cashash_match_pairs(self.h, C.byref(st), self._arrays(codes), self._arrays(keys), len(pairs),
                                        pairs.ctypes.data if len(pairs) else None,
                                        *[(_dptr(a) if self.mem == "device" else (a.ctypes.data if a.size else None))
                                          for a in o], C.byref(stats)))
        return o, stats.as_dict()

    def match_pairs_noalloc(self, images, codes, keys, pairs, out):
        """match_pairs in the library's static device scratch (no device
        allocation in the call); device memory only, out = (match_idx, d1sq,
        d2sq) tensors the caller allocated."""
        st, keep = self._images(images)
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        stats = Stats()
        check(lib().cashash_match_pairs_noalloc(self.h, C.byref(st), self._arrays(codes), self._arrays(keys),
                                                len(pairs), pairs.ctypes.data if len(pairs) else None,
                                                *[_dptr(a) for a in out], C.byref(stats)))
        return out, stats.as_dict()

    def match_pairs_epipolar(self, images, codes, keys, kp, pairs, F, max_px, out=None):
        st, keep = self._images(images)
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        F = np.ascontiguousarray(F, np.float64).reshape(-1, 9)
        if len(F) != len(pairs):
            raise ValueError("one F per pair")
        n = _n_queries(images, pairs)
        o = self._outputs(n, out)
        stats = Stats()
        check(lib().cashash_match_pairs_epipolar(
            self.h, C.byref(st), self._arrays(codes), self._arrays(keys), self._arrays(kp), len(pairs),
            pairs.ctypes.data if len(pairs) else None, F.ctypes.data if len(F) else None, float(max_px),
            *[(_dptr(a) if self.mem == "device" else (a.ctypes.data if a.size else None)) for a in o],
            C.byref(stats)))
        return o, stats.as_dict()

    # ------------------------------------------------------------ disk level (mem="host" only)
    def build_codes_disk(self, set_path, codes_path, host_budget_bytes):
        stats = Stats()
        check(lib().cashash_build_codes_disk(self.h, os.fsencode(set_path), os.fsencode(codes_path),
                                             int(host_budget_bytes), C.byref(stats)))
        return stats.as_dict()

    def match_pairs_disk(self, set_path, codes_path, pairs, out_path, host_budget_bytes, progress_path=None,
                         max_steps=0):
        """Returns (steps_left, stats)."""
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        left = C.c_int64(0)
        stats = Stats()
        check(lib().cashash_match_pairs_disk(
            self.h, os.fsencode(set_path), os.fsencode(codes_path), len(pairs),
            pairs.ctypes.data if len(pairs) else None, os.fsencode(out_path),
            os.fsencode(progress_path) if progress_path else None, int(host_budget_bytes), int(max_steps),
            C.byref(left), C.byref(stats)))
        return left.value, stats.as_dict()

    # ------------------------------------------------------------ geometry-aware two-stage matching
    # (device memory only)

    def _need_device(self):
        if self.mem != "device":
            raise CashashError(E_INVAL, "geometric calls need mem='device'")

    def select_top_scale(self, scales, frac=(1, 5)):
        """Rows of the largest-scale features of each image (int32 tensors)."""
        import torch
        self._need_device()
        nf = np.array([int(s.shape[0]) for s in scales], np.int32)
        rows = [torch.empty(subset_size(n, frac), dtype=torch.int32, device="cuda") for n in nf]
        check(lib().cashash_select_top_scale(self.h, len(scales), self._arrays(scales), nf.ctypes.data,
                                             int(frac[0]), int(frac[1]), self._arrays(rows)))
        return rows

    def gather_rows(self, rows, n_feat, desc=None, codes=None, keys=None, kp=None):
        """Per-image row gathers of the given fields; returns (desc, codes,
        keys, kp) lists (None for fields not given)."""
        import torch
        self._need_device()
        nf = np.ascontiguousarray(n_feat, np.int32)
        nr = np.array([int(r.shape[0]) for r in rows], np.int32)
        outs, args = [], []
        for src, tail, dt in ((desc, (128,), torch.uint8), (codes, (2,), torch.int64), (keys, (6,), torch.uint8),
                              (kp, (2,), torch.float32)):
            if src is None:
                outs.append(None)
                args += [None, None]
                continue
            o = [torch.empty((int(n), *tail), dtype=dt, device="cuda") for n in nr]
            outs.append(o)
            args += [self._arrays(src), self._arrays(o)]
        a = args
        check(lib().cashash_gather_rows(self.h, len(rows), nf.ctypes.data, nr.ctypes.data, self._arrays(rows),
                                        a[0], a[2], a[4], a[6], a[1], a[3], a[5], a[7]))
        return tuple(outs)

    def estimate_fundamental(self, n_feat, kp, pairs, match_idx, rand8, thr=2.0, min_matches=16):
        """Per-pair fundamental matrices from flat stage-1 outputs; returns a
        dict of numpy arrays (F [P,9], n_matches, n_inliers, best_h, status)."""
        self._need_device()
        nf = np.ascontiguousarray(n_feat, np.int32)
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        r = np.ascontiguousarray(rand8, np.uint32).reshape(-1, 8)
        P = len(pairs)
        res = dict(F=np.zeros((P, 9)), n_matches=np.zeros(P, np.int32), n_inliers=np.zeros(P, np.int32),
                   best_h=np.zeros(P, np.int32), status=np.zeros(P, np.int32))
        check(lib().cashash_estimate_fundamental(
            self.h, len(nf), nf.ctypes.data, self._arrays(kp), P, pairs.ctypes.data if P else None,
            _dptr(match_idx), r.ctypes.data, len(r), float(thr), int(min_matches), res["F"].ctypes.data,
            res["n_matches"].ctypes.data, res["n_inliers"].ctypes.data, res["best_h"].ctypes.data,
            res["status"].ctypes.data))
        return res

    def match_pairs_geometric(self, images, codes, keys, kp, scales, pairs, rand8, frac=(1, 5), min_matches=16,
                              ransac_px=2.0, band_px=4.0, out=None):
        """Both stages.  Returns ((match_idx, d1sq, d2sq) over all pairs, per-pair
        dict (F, n_matches, n_inliers, status), stats)."""
        self._need_device()
        st, keep = self._images(images)
        pairs = np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
        r = np.ascontiguousarray(rand8, np.uint32).reshape(-1, 8)
        g = GeoConfig()
        lib().cashash_default_geometric_config(C.byref(g))
        g.frac_num, g.frac_den, g.min_matches = int(frac[0]), int(frac[1]), int(min_matches)
        g.n_hyp, g.ransac_px, g.band_px, g.rand8 = len(r), float(ransac_px), float(band_px), r.ctypes.data
        P = len(pairs)
        n = _n_queries(images, pairs)
        o = self._outputs(n, out)
        res = dict(F=np.zeros((P, 9)), n_matches=np.zeros(P, np.int32), n_inliers=np.zeros(P, np.int32),
                   status=np.zeros(P, np.int32))
        stats = Stats()
        check(lib().cashash_match_pairs_geometric(
            self.h, C.byref(st), self._arrays(codes), self._arrays(keys), self._arrays(kp), self._arrays(scales),
            P, pairs.ctypes.data if P else None, C.byref(g), res["F"].ctypes.data, res["n_matches"].ctypes.data,
            res["n_inliers"].ctypes.data, res["status"].ctypes.data, *[_dptr(a) for a in o], C.byref(stats)))
        return o, res, stats.as_dict()

    def last_geometric_ms(self):
        """Device ms of (subset + gather, stage 1, fundamental, stage 2)."""
        v = (C.c_double * 4)()
        check(lib().cashash_last_geometric_ms(self.h, v))
        return tuple(v)


def set_write(path, images, kp=None):
    """Write the set file of host (numpy) images, with optional keypoints."""
    images = [np.ascontiguousarray(im, np.uint8).reshape(-1, 128) for im in images]
    nf = np.array([im.shape[0] for im in images], np.int32)
    ptrs = _ptrs([im.ctypes.data if im.size else None for im in images])
    st = Images(len(images), C.cast(ptrs, C.POINTER(C.c_void_p)), nf.ctypes.data_as(C.POINTER(C.c_int32)))
    kpp = None
    if kp is not None:
        kp = [np.ascontiguousarray(a, np.float32).reshape(-1, 2) for a in kp]
        kpp = _ptrs([a.ctypes.data if a.size else None for a in kp])
    check(lib().cashash_set_write(os.fsencode(path), C.byref(st), kpp))


def read_codes_file(path):
    """(codes uint64 [N, 2], keys uint8 [N, 6]) of a codes file."""
    hdr = np.fromfile(path, np.int64, count=3, offset=0)
    n = int(hdr[2])
    codes = np.fromfile(path, np.uint64, count=2 * n, offset=64).reshape(n, 2)
    keys = np.fromfile(path, np.uint8, count=6 * n, offset=64 + 16 * n).reshape(n, 6)
    return codes, keys


def read_output_file(path):
    """(match_idx, d1sq, d2sq) int32 arrays of an output file."""
    hdr = np.fromfile(path, np.int64, count=3, offset=0)
    t = int(hdr[2])
    a = np.fromfile(path, np.int32, count=3 * t, offset=64)
    return a[:t], a[t:2 * t], a[2 * t:]


def subset_size(n, frac=(1, 5)) -> int:
    v = int(lib().cashash_subset_size(int(n), int(frac[0]), int(frac[1])))
    if v < 0:
        raise ValueError("need n >= 0 and 0 < frac[0] <= frac[1]")
    return v


def codes_to_numpy(codes):
    """Device int64 [n,2] code tensors -> numpy uint64."""
    return [c.cpu().numpy().view(np.uint64) for c in codes]
