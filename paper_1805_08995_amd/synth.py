"""Seeded synthetic inputs for CasHash matching.

This module holds input synthesis only: descriptors, projection matrices,
pair lists, keypoints and fundamental matrices.  It contains none of the
matching method's arithmetic, so both the HIP path and the CPU oracle can
draw their inputs from it.

The paper measures on SfM image collections of roughly 7.4k-8.6k SIFT
features per image (Experiments, Tables 1-2) and on neighbour lists of 30
images per image (Introduction).  Those datasets are not available, so every
workload below is synthetic with the same shapes: 128-d uint8 SIFT-like
descriptors whose norm is about 512, images that share noisy copies of a
common scene pool, and, for the epipolar form, keypoints that are real
projections of 3-D points by pinhole cameras.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

DIM = 128
N_TABLES = 6
KEY_BITS = 8
CODE_BITS = 128
MATRIX_SEED = 0


def projection_matrices(seed: int = MATRIX_SEED):
    """Random projection rows drawn N(0,1) in float64: first the 128x128 code
    matrix, then the 6x8x128 bucket matrices, from one generator."""
    rng = np.random.default_rng(seed)
    r_code = rng.standard_normal((CODE_BITS, DIM))
    r_bucket = rng.standard_normal((N_TABLES, KEY_BITS, DIM))
    return np.ascontiguousarray(r_code), np.ascontiguousarray(r_bucket)


def desc(rng: np.random.Generator, n: int) -> np.ndarray:
    """SIFT-like uint8 descriptors: |N(0,1)| vector, L2-normalised, clipped at
    0.2, renormalised, scaled by 512, rounded half-to-even, clamped to 255."""
    if n == 0:
        return np.zeros((0, DIM), np.uint8)
    z = np.abs(rng.standard_normal((n, DIM), dtype=np.float32))
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    np.minimum(z, np.float32(0.2), out=z)
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    return np.clip(np.rint(z * np.float32(512.0)), 0, 255).astype(np.uint8)


def noisy(rng: np.random.Generator, x: np.ndarray, sigma: float = 8.0) -> np.ndarray:
    """Noisy copy: add N(0, sigma^2) per component, round, clamp to 0..255."""
    noise = rng.standard_normal(x.shape, dtype=np.float32) * np.float32(sigma)
    return np.clip(np.rint(x.astype(np.float32) + noise), 0, 255).astype(np.uint8)


@dataclass
class Workload:
    """A synthetic matching workload.

    images: list of uint8 [n_i, 128] arrays.
    pairs: int32 [P, 2] of (query image, train image).
    truth: optional per-image ground-truth ids (scene pool member or 3-D point
        id, -1 for a fresh descriptor), for statistical sanity checks only.
    kp: optional list of float32 [n_i, 2] keypoints (epipolar form).
    F: optional float64 [P, 9] row-major fundamental matrices; the epipolar
        line of query point (x, y) in the train image is F @ (x, y, 1).
    scales: optional list of float32 [n_i] feature scales.
    """
    name: str
    images: list
    pairs: np.ndarray
    truth: list = field(default_factory=list)
    kp: list | None = None
    F: np.ndarray | None = None
    max_px: float = 4.0
    scales: list | None = None

    @property
    def n_feat(self) -> np.ndarray:
        return np.array([im.shape[0] for im in self.images], np.int32)

    @property
    def n_queries(self) -> int:
        nf = self.n_feat
        return int(nf[self.pairs[:, 0]].sum()) if len(self.pairs) else 0


def single_pair(seed: int = 1, n: int = 2000, n_shared: int = 1200) -> Workload:
    """One pair: A = desc(n); B = noisy copies of A[:n_shared] then fresh
    descriptors, rows permuted by a seeded permutation.  Set = {A, B}."""
    rng = np.random.default_rng(seed)
    a = desc(rng, n)
    b = np.concatenate([noisy(rng, a[:n_shared]), desc(rng, n - n_shared)])
    truth_b = np.concatenate([np.arange(n_shared), -np.ones(n - n_shared, np.int64)])
    perm = rng.permutation(n)
    b = np.ascontiguousarray(b[perm])
    truth_b = truth_b[perm]
    pairs = np.array([[0, 1]], np.int32)
    return Workload("single_pair_2000", [a, b], pairs, [np.arange(n), truth_b])


def exhaustive_pairs(n_images: int) -> np.ndarray:
    """All i<j pairs with query i and train j."""
    ii, jj = np.triu_indices(n_images, k=1)
    return np.stack([ii, jj], axis=1).astype(np.int32)


def scene_set(seed: int = 2, n_images: int = 100, n_feat: int = 8000,
              n_scenes: int = 10, shared_frac: float = 0.5) -> Workload:
    """Images of n_feat descriptors: image i takes shared_frac noisy copies of
    distinct members of scene pool (i mod n_scenes), the rest fresh, shuffled.
    Pairs: exhaustive i<j."""
    rng = np.random.default_rng(seed)
    pool_n = 2 * n_feat
    pools = [desc(rng, pool_n) for _ in range(n_scenes)]
    images, truth = [], []
    n_sh = int(round(shared_frac * n_feat))
    for i in range(n_images):
        s = i % n_scenes
        members = rng.choice(pool_n, size=n_sh, replace=False)
        x = np.concatenate([noisy(rng, pools[s][members]), desc(rng, n_feat - n_sh)])
        t = np.concatenate([s * pool_n + members, -np.ones(n_feat - n_sh, np.int64)])
        perm = rng.permutation(n_feat)
        images.append(np.ascontiguousarray(x[perm]))
        truth.append(t[perm])
    return Workload(f"scenes_{n_images}x{n_feat}", images, exhaustive_pairs(n_images), truth)


def uneven_set(seed: int = 4, n_images: int = 2000, lo: int = 1000, hi: int = 20000,
               n_scenes: int = 200, n_partners: int = 30, shared_frac: float = 0.5) -> Workload:
    """Feature counts floor(exp(U(ln lo, ln hi))); image i shares shared_frac
    noisy copies with scene pool (i mod n_scenes) of `hi` descriptors; each
    image draws n_partners distinct partners (not itself), giving directed
    (query, train) pairs.  Every pool and every image has its own child
    generator, so generation order does not change the bytes."""
    root = np.random.SeedSequence(seed)
    g_counts, g_pairs, g_pools, g_imgs = root.spawn(4)
    rng = np.random.default_rng(g_counts)
    counts = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_images))).astype(np.int64)
    counts = np.clip(counts, lo, hi)
    pool_ss = g_pools.spawn(n_scenes)
    img_ss = g_imgs.spawn(n_images)
    images: list = [None] * n_images
    truth: list = [None] * n_images

    def scene(s):
        members_of = range(s, n_images, n_scenes)
        if not len(members_of):
            return
        pool = desc(np.random.default_rng(pool_ss[s]), hi)
        for i in members_of:
            r = np.random.default_rng(img_ss[i])
            n = int(counts[i])
            n_sh = int(round(shared_frac * n))
            members = r.choice(hi, size=n_sh, replace=False)
            x = np.concatenate([noisy(r, pool[members]), desc(r, n - n_sh)])
            t = np.concatenate([s * hi + members, -np.ones(n - n_sh, np.int64)])
            perm = r.permutation(n)
            images[i] = np.ascontiguousarray(x[perm])
            truth[i] = t[perm]

    # scenes are independent (own generators), so threads do not change the bytes
    with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(scene, range(n_scenes)))
    rp = np.random.default_rng(g_pairs)
    pairs = []
    for i in range(n_images):
        others = rp.choice(n_images - 1, size=n_partners, replace=False)
        others = others + (others >= i)
        pairs.extend((i, int(j)) for j in others)
    return Workload(f"uneven_{n_images}", images, np.array(pairs, np.int32), truth)


def _look_at(center: np.ndarray) -> np.ndarray:
    """World-to-camera rotation for a camera at `center` looking at the
    origin with world +z up (camera y points down in the image)."""
    fwd = -center / np.linalg.norm(center)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return np.stack([right, down, fwd])


def _skew(t: np.ndarray) -> np.ndarray:
    return np.array([[0.0, -t[2], t[1]], [t[2], 0.0, -t[0]], [-t[1], t[0], 0.0]])


def _orbit_images(rng, pts, base, n_images, n_feat, radius, K, width, height, kp_sigma, phase=0.0):
    """Cameras on a horizontal circle of the given radius, looking at the
    origin.  Image i observes n_feat random points that project inside the
    frame: keypoint = projection + N(0, kp_sigma^2) px (float32), descriptor
    = noisy copy of the point's base descriptor.  Returns per-image lists of
    descriptors, point ids, keypoints and depths, and the cameras (R, t)."""
    Rs, ts, images, truth, kps, depths = [], [], [], [], [], []
    for i in range(n_images):
        th = 2.0 * math.pi * i / n_images + phase
        c = np.array([radius * math.cos(th), radius * math.sin(th), 0.0])
        R = _look_at(c)
        t = -R @ c
        Rs.append(R)
        ts.append(t)
        cam = pts @ R.T + t
        uvw = cam @ K.T
        uv = uvw[:, :2] / uvw[:, 2:3]
        vis = np.flatnonzero((cam[:, 2] > 0) & (uv[:, 0] >= 0) & (uv[:, 0] < width)
                             & (uv[:, 1] >= 0) & (uv[:, 1] < height))
        sel = rng.choice(vis, size=min(n_feat, len(vis)), replace=False)
        kp = (uv[sel] + rng.standard_normal((len(sel), 2)) * kp_sigma).astype(np.float32)
        images.append(noisy(rng, base[sel]))
        truth.append(sel.astype(np.int64))
        kps.append(np.ascontiguousarray(kp))
        depths.append(cam[sel, 2])
    return images, truth, kps, depths, Rs, ts


def _intrinsics(focal, width, height):
    return np.array([[focal, 0.0, width / 2], [0.0, focal, height / 2], [0.0, 0.0, 1.0]])


def _true_F(K, Ri, ti, Rj, tj):
    """Fundamental matrix of (query camera i, train camera j):
    F = K^-T [t]x R K^-1 with R = Rj Ri^T, t = tj - R ti."""
    Kinv = np.linalg.inv(K)
    R = Rj @ Ri.T
    t = tj - R @ ti
    return (Kinv.T @ _skew(t) @ R @ Kinv).reshape(9)


def epipolar_set(seed: int = 5, n_images: int = 500, n_feat: int = 12000,
                 n_points: int = 200_000, n_neighbours: int = 30,
                 radius: float = 40.0, half_cube: float = 10.0,
                 focal: float = 1500.0, width: int = 1920, height: int = 1080,
                 kp_sigma: float = 0.5, max_px: float = 4.0) -> Workload:
    """Pinhole cameras on a horizontal circle around a cube of random 3-D
    points.  Each image observes n_feat distinct points that project inside
    the frame; keypoint = projection + N(0, kp_sigma^2) px (float32);
    descriptor = noisy copy of the point's base descriptor.  Each camera is
    paired with its n_neighbours nearest cameras on the orbit; F is the true
    fundamental matrix of the (query, train) pair."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-half_cube, half_cube, (n_points, 3))
    base = desc(rng, n_points)
    K = _intrinsics(focal, width, height)
    images, truth, kps, _, Rs, ts = _orbit_images(rng, pts, base, n_images, n_feat, radius, K, width, height,
                                                  kp_sigma)
    half = n_neighbours // 2
    pairs, Fs = [], []
    for i in range(n_images):
        for off in list(range(-half, 0)) + list(range(1, n_neighbours - half + 1)):
            j = (i + off) % n_images
            pairs.append((i, j))
            Fs.append(_true_F(K, Rs[i], ts[i], Rs[j], ts[j]))
    return Workload(f"epipolar_{n_images}x{n_feat}", images, np.array(pairs, np.int32), truth,
                    kp=kps, F=np.ascontiguousarray(np.array(Fs, np.float64)), max_px=max_px)


def geometric_set(seed: int = 6, n_scenes: int = 2, cams_per_scene: int = 250, n_feat: int = 12000,
                  n_points: int = 200_000, n_near: int = 20, n_far: int = 10,
                  radius: float = 40.0, half_cube: float = 10.0,
                  focal: float = 1500.0, width: int = 1920, height: int = 1080,
                  kp_sigma: float = 0.5, max_px: float = 4.0,
                  size_median: float = 0.04, size_sigma: float = 0.6, scale_jitter: float = 0.1) -> Workload:
    """Inputs of two-stage geometry-aware matching: n_scenes independent
    scenes (own 3-D points, own descriptor pool), each seen by an orbit of
    cams_per_scene cameras as in epipolar_set.  Every 3-D point has a
    physical size (log-normal); a feature's scale is focal * size / depth
    times a log-normal jitter, so the largest-scale features of neighbouring
    views are largely the same points.  Each camera is paired with its n_near
    nearest cameras of its own orbit and n_far random cameras of other scenes
    (pairs with no common point).  F holds the true fundamental matrix of
    same-scene pairs and zeros for the others (not an input of the method)."""
    rng = np.random.default_rng(seed)
    K = _intrinsics(focal, width, height)
    images, truth, kps, scales, cams, scene_of = [], [], [], [], [], []
    for sc in range(n_scenes):
        pts = rng.uniform(-half_cube, half_cube, (n_points, 3))
        base = desc(rng, n_points)
        size = np.exp(rng.standard_normal(n_points) * size_sigma) * size_median
        im, tr, kp, dep, Rs, ts = _orbit_images(rng, pts, base, cams_per_scene, n_feat, radius, K, width, height,
                                                kp_sigma, phase=0.37 * sc)
        for i in range(cams_per_scene):
            jit = np.exp(rng.standard_normal(len(tr[i])) * scale_jitter)
            scales.append(np.ascontiguousarray((focal * size[tr[i]] / dep[i] * jit).astype(np.float32)))
            cams.append((Rs[i], ts[i]))
            scene_of.append(sc)
        images += im
        truth += [t + sc * n_points for t in tr]
        kps += kp
    n_images = len(images)
    scene_of = np.array(scene_of)
    half = n_near // 2
    pairs, Fs = [], []
    for i in range(n_images):
        sc, a = divmod(i, cams_per_scene)
        for off in list(range(-half, 0)) + list(range(1, n_near - half + 1)):
            j = sc * cams_per_scene + (a + off) % cams_per_scene
            pairs.append((i, j))
            Fs.append(_true_F(K, cams[i][0], cams[i][1], cams[j][0], cams[j][1]))
        others = np.flatnonzero(scene_of != sc)
        for j in rng.choice(others, size=min(n_far, len(others)), replace=False):
            pairs.append((i, int(j)))
            Fs.append(np.zeros(9))
    return Workload(f"geometric_{n_images}x{n_feat}", images, np.array(pairs, np.int32), truth,
                    kp=kps, F=np.ascontiguousarray(np.array(Fs, np.float64)), max_px=max_px, scales=scales)
