"""CasHash pairwise SIFT matching on one MI355X (gfx950).

The hot path (projection to sign codes and bucket keys, bucket tables,
candidate union, Hamming ranking, exact squared distance and ratio test,
epipolar band) runs in hand-written HIP kernels behind the C ABI declared in
include/cashash.h.  `binding` is a thin ctypes layer over that library; it
raises if the library has not been built.
"""
__all__ = ["binding", "synth"]
