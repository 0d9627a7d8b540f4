"""Write the oracle's digests of the full-size workloads.

For each workload this computes, with the CPU oracle only (inputs from
paper_1805_08995_amd.synth), the codes and keys of every image of the set
and the matches of every pair, and stores per-image code digests and
per-pair output digests (tests/digests.py) in fullsize_<name>.npz:

  scenes   : 100 images x 8000 features, all 4950 pairs i<j (k = 10, ratio 0.8)
  uneven   : 2000 images of 1000-20000 features, 30 partners each (60000 pairs)
  epipolar : 500 images x 12000 features, 15000 neighbour pairs, band 4 px
             around the true fundamental matrix (Eq. 1-2)

Nothing here reads GPU output.  Run from the repository root:
    python tests/golden/make_fullsize_digests.py [scenes uneven epipolar]
It takes about half an hour of oracle time on 8 cores.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from digests import code_digests, pair_digests, pair_offsets  # noqa: E402
from paper_1805_08995_amd import synth  # noqa: E402

WORKLOADS = {"scenes": synth.scene_set, "uneven": synth.uneven_set, "epipolar": synth.epipolar_set}
CHUNK_PAIRS = 600


def path_of(name: str) -> str:
    return os.path.join(HERE, f"fullsize_{name}.npz")


def make(name: str) -> None:
    t0 = time.time()
    w = WORKLOADS[name]()
    mats = synth.projection_matrices()
    print(f"[{name}] generated {len(w.images)} images, {len(w.pairs)} pairs in {time.time() - t0:.0f}s", flush=True)
    codes, keys = oracle.build_codes(w.images, *mats)
    cd = code_digests(codes, keys)
    print(f"[{name}] codes in {time.time() - t0:.0f}s", flush=True)
    nf = w.n_feat
    epi = w.kp is not None
    digests, matches = [], 0
    for lo in range(0, len(w.pairs), CHUNK_PAIRS):
        pr = w.pairs[lo:lo + CHUNK_PAIRS]
        extra = dict(kp=w.kp, F=w.F[lo:lo + CHUNK_PAIRS], max_px=w.max_px) if epi else {}
        out = oracle.match_pairs(w.images, codes, keys, pr, k=10, ratio=(4, 5), **extra)
        digests.append(pair_digests(*out, pair_offsets(nf, pr)))
        matches += int((out[0] >= 0).sum())
        print(f"[{name}] pairs {lo + len(pr)}/{len(w.pairs)} at {time.time() - t0:.0f}s", flush=True)
    np.savez(path_of(name), pair_digest=np.concatenate(digests), code_digest=cd,
             n_matches=np.int64(matches), n_queries=np.int64(w.n_queries), k=np.int64(10),
             ratio=np.array([4, 5], np.int64), max_px=np.float64(w.max_px if epi else 0.0))
    print(f"[{name}] {matches} matches over {w.n_queries} queries; wrote {path_of(name)}", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or list(WORKLOADS):
        make(n)
