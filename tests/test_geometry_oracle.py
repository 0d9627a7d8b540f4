"""Pins of the geometry-aware first stage oracle (Sec. 3.1: top-scale subset,
fundamental matrix from the subset matches, acceptance rule) against what
the mathematics fixes: numpy sorting, SVD and symmetric eigensolvers as
special cases, closed forms of Floyd's sampler, noise-free correspondences
of known cameras, planted outliers and the rectified-stereo line distance."""
import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_1805_08995_amd import synth


def _rand(h, seed=7):
    return np.random.default_rng(seed).integers(0, 2**32, (h, 8), dtype=np.uint64).astype(np.uint32)


# ---- subset ---------------------------------------------------------------

@pytest.mark.parametrize("n,m", [(0, 0), (1, 1), (5, 1), (6, 2), (12000, 2400), (12001, 2401)])
def test_subset_size_is_ceiling_of_a_fifth(n, m):
    assert G.subset_size(n) == m


def test_top_scale_equals_stable_descending_sort():
    rng = np.random.default_rng(0)
    for n in (1, 7, 100, 3001):
        s = rng.integers(1, 40, n).astype(np.float32) * np.float32(0.25)   # many ties
        m = G.subset_size(n)
        order = np.lexsort((np.arange(n), -s.astype(np.float64)))
        assert np.array_equal(G.top_scale(s), np.sort(order[:m]).astype(np.int32))


def test_top_scale_total_order_of_zeros_and_negatives():
    s = np.array([-0.0, 0.0, -1.0, 3.0, -0.0], np.float32)
    assert list(G.top_scale(s, (2, 5))) == [1, 3]          # 3.0 then +0 (above -0)
    assert list(G.top_scale(s, (3, 5))) == [0, 1, 3]       # then the first -0


# ---- Floyd sampling ---------------------------------------------------------

def test_floyd_closed_forms():
    for n in (8, 9, 20, 1000):
        assert list(G.floyd8(np.zeros(8, np.uint32), n)) == [0] + list(range(n - 7, n))
        assert list(G.floyd8(np.full(8, 0xFFFFFFFF, np.uint32), n)) == list(range(n - 8, n))


def test_floyd_distinct_in_range_and_uniform():
    rng = np.random.default_rng(1)
    n = 10
    counts = np.zeros(n)
    for _ in range(20000):
        s = G.floyd8(rng.integers(0, 2**32, 8, dtype=np.uint64).astype(np.uint32), n)
        assert len(set(s.tolist())) == 8 and s.min() >= 0 and s.max() < n
        counts[s] += 1
    # every index is drawn with probability 8/10
    assert np.all(np.abs(counts / 20000 - 0.8) < 0.02)


# ---- linear algebra ---------------------------------------------------------

@pytest.mark.parametrize("n,sweeps", [(3, 6), (9, 10)])
def test_jacobi_equals_eigh(n, sweeps):
    rng = np.random.default_rng(n)
    for trial in range(20):
        B = rng.standard_normal((n + 3 if trial % 2 else n, n)) * 10.0 ** rng.uniform(-3, 3, n)
        A0 = B.T @ B if trial % 2 else (B + B.T)
        A, V = G.jacobi(A0, sweeps)
        lam = np.diag(A)
        ref = np.linalg.eigvalsh(A0)
        scale = np.abs(ref).max()
        assert np.allclose(np.sort(lam), ref, rtol=0, atol=1e-12 * scale)
        assert np.allclose(V.T @ V, np.eye(n), atol=1e-13)
        assert np.allclose(A0 @ V, V * lam, atol=1e-11 * scale)
        off = A - np.diag(lam)
        assert np.linalg.norm(off) <= 1e-13 * scale


def test_null8_equals_svd_null_vector():
    rng = np.random.default_rng(2)
    for _ in range(50):
        A = rng.standard_normal((8, 9))
        f = G.null8(A)
        assert f[8] == 1.0
        ref = np.linalg.svd(A)[2][-1]
        cos = abs(f @ ref) / np.linalg.norm(f)
        assert cos > 1 - 1e-12
        assert np.linalg.norm(A @ f) < 1e-10 * np.linalg.norm(A) * np.linalg.norm(f)


def test_null8_zero_pivot():
    A = np.random.default_rng(3).standard_normal((8, 9))
    A[:, 0] = 0.0
    assert G.null8(A) is None


def test_rank2_equals_svd_truncation():
    rng = np.random.default_rng(4)
    for _ in range(50):
        F = rng.standard_normal(9) * 10.0 ** rng.uniform(-2, 2)
        U, s, Vt = np.linalg.svd(F.reshape(3, 3))
        ref = (U[:, :2] * s[:2]) @ Vt[:2]
        got = G.rank2(F).reshape(3, 3)
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * s[0])
        assert abs(np.linalg.det(got)) < 1e-12 * s[0] ** 3


def test_inlier_rectified_stereo_is_row_distance():
    # rectified stereo: the epipolar line of (x, y) is y' = y, distance |y - y'|
    F = np.array([0, 0, 0, 0, 0, -1, 0, 1, 0], np.float64)
    q = np.array([300.0, 200.0], np.float32)
    assert G.is_inlier(F, q, [900.0, 202.0], 2.0)             # exactly on the threshold
    assert G.is_inlier(F, q, [10.0, 198.0], 2.0)
    assert not G.is_inlier(F, q, [10.0, 202.125], 2.0)
    assert not G.is_inlier(F, q, [10.0, 197.875], 2.0)


# ---- estimation from known cameras ----------------------------------------

def _cameras(rng):
    """Two cameras 40 m from a 20 m cube, 30 degrees apart, and their F."""
    K = np.array([[1500.0, 0, 960], [0, 1500.0, 540], [0, 0, 1]])

    def cam(th):
        c = np.array([40 * np.cos(th), 40 * np.sin(th), 2.0])
        f = -c / np.linalg.norm(c)
        r = np.cross(f, [0, 0, 1.0])
        r /= np.linalg.norm(r)
        return np.stack([r, np.cross(f, r), f]), c

    (Ri, ci), (Rj, cj) = cam(0.3), cam(0.3 + np.pi / 6)
    ti, tj = -Ri @ ci, -Rj @ cj
    R = Rj @ Ri.T
    t = tj - R @ ti
    tx = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
    Kinv = np.linalg.inv(K)
    F = Kinv.T @ tx @ R @ Kinv

    def project(X, Rc, tc):
        x = (X @ Rc.T + tc) @ K.T
        return x[:, :2] / x[:, 2:3]

    return F, lambda X: project(X, Ri, ti), lambda X: project(X, Rj, tj)


def _unit(F):
    F = np.asarray(F, np.float64).reshape(9)
    F = F / np.linalg.norm(F)
    return F * np.sign(F[np.argmax(np.abs(F))])


def _epi_dist(F, q, t):
    F = F.reshape(3, 3)
    l = np.c_[q, np.ones(len(q))] @ F.T
    return np.abs(np.sum(l * np.c_[t, np.ones(len(t))], 1)) / np.hypot(l[:, 0], l[:, 1])


def test_exact_correspondences_recover_the_true_matrix():
    rng = np.random.default_rng(5)
    Ftrue, Pi, Pj = _cameras(rng)
    X = rng.uniform(-10, 10, (100, 3))
    q, t = Pi(X).astype(np.float32), Pj(X).astype(np.float32)
    st, F, ni, bh = G.fundamental(q, t, _rand(64))
    assert st == G.ACCEPT and ni == 100 and bh >= 0
    assert np.allclose(_unit(F), _unit(Ftrue), atol=1e-5)
    assert _epi_dist(F, q.astype(np.float64), t.astype(np.float64)).max() < 1e-2


def test_planted_outliers_are_rejected():
    rng = np.random.default_rng(6)
    Ftrue, Pi, Pj = _cameras(rng)
    X = rng.uniform(-10, 10, (150, 3))
    q = Pi(X) + rng.standard_normal((150, 2)) * 0.3
    t = Pj(X) + rng.standard_normal((150, 2)) * 0.3
    qo = rng.uniform([0, 0], [1920, 1080], (50, 2))
    to = rng.uniform([0, 0], [1920, 1080], (50, 2))
    perm = rng.permutation(200)
    Q = np.r_[q, qo][perm].astype(np.float32)
    T = np.r_[t, to][perm].astype(np.float32)
    true = perm < 150
    st, F, ni, bh = G.fundamental(Q, T, _rand(256), thr=2.0)
    assert st == G.ACCEPT
    inl = np.array([G.is_inlier(F, Q[i], T[i], 2.0) for i in range(200)])
    assert inl.sum() == ni
    assert inl[true].mean() > 0.97
    assert inl[~true].sum() <= 3
    # the estimate explains the noise-free geometry to within a pixel
    Xt = rng.uniform(-10, 10, (500, 3))
    assert np.median(_epi_dist(F, Pi(Xt), Pj(Xt))) < 0.5


def test_status_rules():
    rng = np.random.default_rng(8)
    few = rng.uniform(0, 1000, (15, 2)).astype(np.float32)
    assert G.fundamental(few, few, _rand(16))[0] == G.FEW_MATCHES
    assert G.fundamental(few, few, _rand(16), min_matches=8)[0] != G.FEW_MATCHES
    same = np.full((40, 2), 100.0, np.float32)
    assert G.fundamental(same, rng.uniform(0, 1000, (40, 2)).astype(np.float32), _rand(16))[0] == G.DEGENERATE
    q = rng.uniform([0, 0], [1920, 1080], (200, 2)).astype(np.float32)
    t = rng.uniform([0, 0], [1920, 1080], (200, 2)).astype(np.float32)
    st, F, ni, bh = G.fundamental(q, t, _rand(256))
    assert st == G.FEW_INLIERS and 3 * ni < 2 * 200


def test_ties_take_the_first_hypothesis():
    rng = np.random.default_rng(9)
    _, Pi, Pj = _cameras(rng)
    X = rng.uniform(-10, 10, (60, 3))
    q, t = Pi(X).astype(np.float32), Pj(X).astype(np.float32)
    r = np.repeat(_rand(1, seed=3), 4, axis=0)        # four identical hypotheses
    assert G.fundamental(q, t, r)[3] == 0


def test_acceptance_boundary_two_thirds():
    # 20 exact correspondences + 10 far outliers: 20 / 30 inliers is accepted,
    # 20 / 31 is not
    rng = np.random.default_rng(10)
    _, Pi, Pj = _cameras(rng)
    X = rng.uniform(-10, 10, (20, 3))
    q, t = Pi(X), Pj(X)
    for n_out, want in ((10, G.ACCEPT), (11, G.FEW_INLIERS)):
        qo = rng.uniform([0, 0], [1920, 1080], (n_out, 2))
        to = rng.uniform([0, 0], [1920, 1080], (n_out, 2))
        Q, T = np.r_[q, qo].astype(np.float32), np.r_[t, to].astype(np.float32)
        st, F, ni, _ = G.fundamental(Q, T, _rand(512), thr=1.0)
        inl = [G.is_inlier(F, Q[i], T[i], 1.0) for i in range(len(Q))]
        assert all(inl[:20]) and ni == 20, (n_out, ni)
        assert st == want


# ---- the two-stage pipeline on a small synthetic set ----------------------

def test_pipeline_accepts_overlapping_pairs_only():
    w = synth.geometric_set(cams_per_scene=12, n_feat=3000, n_points=30000, n_near=4, n_far=2)
    mats = synth.projection_matrices()
    codes, keys = oracle.build_codes(w.images, *mats)
    r = G.geometric_match(w.images, codes, keys, w.kp, w.scales, w.pairs, _rand(256))
    same = np.array([np.any(f != 0) for f in w.F])
    assert np.all(r["status"][same] == G.ACCEPT)
    assert np.all(r["status"][~same] != G.ACCEPT)
    # the estimates explain the true correspondences of each accepted pair
    for p in r["accepted"][:8]:
        qi, ti = w.pairs[p]
        common, a, b = np.intersect1d(w.truth[qi], w.truth[ti], return_indices=True)
        d = _epi_dist(r["F"][p], w.kp[qi][a].astype(np.float64), w.kp[ti][b].astype(np.float64))
        assert np.median(d) < 1.0
    # stage 2 finds far more matches than stage 1
    assert (r["stage2"][0] >= 0).sum() > 3 * r["n_matches"][r["accepted"]].sum()
