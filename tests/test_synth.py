"""Seeded generators: determinism and the distribution of the synthetic
SIFT-like descriptors (norm about 512, components clipped at 0.2 * norm)."""
import numpy as np

from paper_1805_08995_amd import synth


def test_same_seed_same_bytes():
    a = synth.single_pair()
    b = synth.single_pair()
    for x, y in zip(a.images, b.images):
        assert np.array_equal(x, y)
    c = synth.scene_set(n_images=3, n_feat=200)
    d = synth.scene_set(n_images=3, n_feat=200)
    assert all(np.array_equal(x, y) for x, y in zip(c.images, d.images))
    assert np.array_equal(c.pairs, d.pairs)


def test_matrices_seed0_shapes():
    rc, rb = synth.projection_matrices()
    assert rc.shape == (128, 128) and rb.shape == (6, 8, 128) and rc.dtype == np.float64
    rc2, _ = synth.projection_matrices()
    assert np.array_equal(rc, rc2)
    norms = np.linalg.norm(np.concatenate([rc, rb.reshape(48, 128)]), axis=1)
    assert norms.max() < 20.0


def test_descriptor_distribution():
    x = synth.desc(np.random.default_rng(0), 5000).astype(np.float64)
    n = np.linalg.norm(x, axis=1)
    assert abs(n.mean() - 512) < 3 and x.max() <= 255
    assert np.all(x.max(1) <= 0.2 * 512 * 1.6)


def test_pair_lists():
    assert len(synth.exhaustive_pairs(100)) == 4950
    w = synth.uneven_set(n_images=40, lo=100, hi=400, n_scenes=4, n_partners=5)
    assert len(w.pairs) == 200 and (w.pairs[:, 0] != w.pairs[:, 1]).all()
    for i in range(40):
        assert len(set(w.pairs[w.pairs[:, 0] == i, 1])) == 5
    nf = w.n_feat
    assert nf.min() >= 100 and nf.max() <= 400
    e = synth.epipolar_set(n_images=6, n_feat=300, n_points=3000, n_neighbours=4)
    assert len(e.pairs) == 24 and e.F.shape == (24, 9)
    assert all(k.dtype == np.float32 and k.shape == (300, 2) for k in e.kp)
