"""Pins of the CPU oracle against facts that do not come from the oracle:
closed forms, hand-worked values, textbook exhaustive nearest neighbour,
numpy float64 signs, invariants.  Each test names the part of the method it
pins (paper: Review of Cascade Hashing Steps 1-4; hashing-code and Euclidean
distance sections; ranking section; Eq. 1-2)."""
import json
import os

import numpy as np
import pytest

from paper_1805_08995_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pad(rows):
    x = np.zeros((len(rows), 128), np.uint8)
    for i, r in enumerate(rows):
        x[i, :len(r)] = r
    return x


def _unit_bucket_rows(index_of):
    rb = np.zeros((6, 8, 128))
    for t in range(6):
        for b in range(8):
            rb[t, b, index_of(t, b)] = 1.0
    return rb


# ---------------------------------------------------------------- worked example

def test_golden_worked_example(orc):
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    A, B = _pad(g["A"]), _pad(g["B"])
    rc = np.eye(128)
    rb = _unit_bucket_rows(lambda t, b: 8 * t + b)
    codes, keys = orc.build_codes([A, B], rc, rb)
    assert codes[0][:, 0].tolist() == g["codes_lo"]["A"]
    assert codes[1][:, 0].tolist() == g["codes_lo"]["B"]
    assert not codes[0][:, 1].any() and not codes[1][:, 1].any()
    assert keys[0][:, 0].tolist() == g["keys0"]["A"] and keys[1][:, 0].tolist() == g["keys0"]["B"]
    assert not keys[0][:, 1:].any() and not keys[1][:, 1:].any()
    for k, exp in (("k2", g["k2"]), ("k1", g["k1"])):
        m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=int(k[1]))
        assert m.tolist() == exp["match_idx"], k
        assert d1.tolist() == exp["d1sq"], k
        assert d2.tolist() == exp["d2sq"], k


# ---------------------------------------------------------------- codes

def test_column_sums_match_numpy(orc):
    rng = np.random.default_rng(11)
    ims = [synth.desc(rng, n) for n in (0, 17, 300)]
    S, n = orc.column_sums(ims)
    assert n == 317
    assert np.array_equal(S, np.concatenate(ims).astype(np.int64).sum(0))


def _tiny_integer_set(seed):
    # values in {0, 2, 4, 6}: many components equal the mean exactly
    rng = np.random.default_rng(seed)
    return [rng.choice([0, 2, 4, 6], size=(4, 128)).astype(np.uint8) for _ in range(2)]


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_codes_identity_closed_form(orc, sign):
    """Code rows = +/- identity: bit j = [N x_j > S_j] (resp. <); equality gives 0."""
    ims = _tiny_integer_set(3)
    perm = np.random.default_rng(5).permutation(128)
    rb = _unit_bucket_rows(lambda t, b: int(perm[8 * t + b]))
    codes, keys = orc.build_codes(ims, sign * np.eye(128), rb)
    allx = np.concatenate(ims).astype(np.int64)
    N, S = allx.shape[0], allx.sum(0)
    assert (N * allx == S).any(), "fixture must contain exact ties"
    for m, x in enumerate(ims):
        c = N * x.astype(np.int64) - S
        bits = (sign * c > 0)
        w0 = (bits[:, :64].astype(np.uint64) << np.arange(64, dtype=np.uint64)).sum(1, dtype=np.uint64)
        w1 = (bits[:, 64:].astype(np.uint64) << np.arange(64, dtype=np.uint64)).sum(1, dtype=np.uint64)
        assert np.array_equal(codes[m][:, 0], w0) and np.array_equal(codes[m][:, 1], w1)
        kb = (c[:, perm[:48]] > 0).reshape(-1, 6, 8)
        exp_keys = (kb.astype(np.int64) << np.arange(8)).sum(2)
        assert np.array_equal(keys[m], exp_keys.astype(np.uint8))


def test_codes_exact_zero_projection(orc):
    """r . (N x - S) = 0 exactly gives bit 0; +1 gives bit 1; -1 gives 0."""
    x = _pad([[3, 2], [2, 3]])  # N = 2, N x0 - S = (1, -1)
    rc = np.zeros((128, 128))
    rc[0, :2] = [1, 1]    # 0      -> 0
    rc[1, :2] = [1, 0]    # +1     -> 1
    rc[2, :2] = [0, 1]    # -1     -> 0
    rc[3, :2] = [2, 1]    # +1     -> 1
    rc[4, :2] = [-1, -1]  # -0.0   -> 0
    codes, _ = orc.build_codes([x], rc, np.zeros((6, 8, 128)))
    assert int(codes[0][0, 0]) == 0b01010
    assert int(codes[0][1, 0]) == 0b00100  # second row: N x1 - S = (-1, 1)


@pytest.mark.parametrize("scale", [2.0 ** -7, 2.0 ** 9])
def test_codes_power_of_two_scaling_invariant(orc, scale):
    rc, rb = synth.projection_matrices()
    ims = [synth.desc(np.random.default_rng(7), 64), synth.desc(np.random.default_rng(8), 40)]
    c1, k1 = orc.build_codes(ims, rc, rb)
    c2, k2 = orc.build_codes(ims, rc * scale, rb * scale)
    for m in range(2):
        assert np.array_equal(c1[m], c2[m]) and np.array_equal(k1[m], k2[m])


def test_codes_vs_numpy_float64_signs(orc):
    """Where |r . c| is far above float64 rounding, the oracle's sign must
    equal numpy's BLAS-order float64 product."""
    rc, rb = synth.projection_matrices()
    w = synth.single_pair()
    codes, keys = orc.build_codes(w.images, rc, rb)
    allx = np.concatenate(w.images).astype(np.int64)
    N, S = allx.shape[0], allx.sum(0)
    rows = np.concatenate([rc, rb.reshape(48, 128)])
    for m, x in enumerate(w.images):
        c = (N * x.astype(np.int64) - S).astype(np.float64)
        p = c @ rows.T
        safe = np.abs(p) > 1e-9 * np.linalg.norm(rows, axis=1)[None, :] * np.linalg.norm(c, axis=1)[:, None]
        assert safe.mean() > 0.999
        bits = np.zeros((x.shape[0], 176), bool)
        for j in range(128):
            bits[:, j] = (codes[m][:, j >> 6] >> np.uint64(j & 63)) & np.uint64(1)
        for t in range(6):
            for b in range(8):
                bits[:, 128 + 8 * t + b] = (keys[m][:, t] >> b) & 1
        assert np.array_equal(bits[safe], (p > 0)[safe])
    # the codes are balanced: mean-centred signs are close to fair coins
    assert 0.45 < bits[:, :128].mean() < 0.55


# ---------------------------------------------------------------- matching

def _brute(A, B, cand_sets, k, codes_a=None, codes_b=None):
    """Textbook reference: for each query, rank the candidate set by
    (Hamming, index) with Python ints, keep k, exact int64 squared distances,
    nearest with smallest index, ratio 25 d1 < 16 d2."""
    out = []
    Ai, Bi = A.astype(np.int64), B.astype(np.int64)
    for q, cs in enumerate(cand_sets):
        cs = sorted(cs)
        if codes_a is not None:
            cq = int(codes_a[q, 0]) | (int(codes_a[q, 1]) << 64)
            ham = {j: (cq ^ (int(codes_b[j, 0]) | (int(codes_b[j, 1]) << 64))).bit_count() for j in cs}
            cs = sorted(cs, key=lambda j: (ham[j], j))
        top = cs[:k]
        if not top:
            out.append((-1, -1, -1))
            continue
        d = {j: int(((Ai[q] - Bi[j]) ** 2).sum()) for j in top}
        ds = sorted(d.values())
        d1 = ds[0]
        d2 = ds[1] if len(ds) > 1 else -1
        j1 = min(j for j in top if d[j] == d1)
        ok = len(top) >= 2 and 25 * d1 < 16 * d2
        out.append((j1 if ok else -1, d1, d2))
    return [np.array(c, np.int32) for c in zip(*out)] if out else [np.zeros(0, np.int32)] * 3


def test_exhaustive_nn_when_k_covers_all(orc):
    """Zero bucket rows: every key is 0, so each query's candidates are all of
    B; with k >= |B| the result is exhaustive NN + ratio test (numpy argsort)."""
    rng = np.random.default_rng(21)
    A = synth.desc(rng, 50)
    B = np.concatenate([synth.noisy(rng, A[:30]), synth.desc(rng, 30)])
    rc, _ = synth.projection_matrices()
    codes, keys = orc.build_codes([A, B], rc, np.zeros((6, 8, 128)))
    assert not np.concatenate(keys).any()
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=64)
    D = ((A[:, None, :].astype(np.int64) - B[None, :, :].astype(np.int64)) ** 2).sum(2)
    order = np.argsort(D, axis=1, kind="stable")
    e1 = D[np.arange(50), order[:, 0]]
    e2 = D[np.arange(50), order[:, 1]]
    assert np.array_equal(d1, e1) and np.array_equal(d2, e2)
    exp_m = np.where(25 * e1 < 16 * e2, order[:, 0], -1)
    assert np.array_equal(m, exp_m)
    assert (m[:30] == np.arange(30)).mean() > 0.9  # noisy copies are found


def test_union_bruteforce_when_k_covers_union(orc):
    """Real bucket rows, k >= |U|: NN restricted to the set union of the six
    same-key buckets, computed independently in Python."""
    rc, rb = synth.projection_matrices()
    rng = np.random.default_rng(22)
    A = synth.desc(rng, 40)
    B = np.concatenate([synth.noisy(rng, A[:20]), synth.desc(rng, 40)])
    codes, keys = orc.build_codes([A, B], rc, rb)
    cand = [{j for t in range(6) for j in range(len(B)) if keys[1][j, t] == keys[0][q, t]}
            for q in range(len(A))]
    assert max(len(c) for c in cand) <= 60 and sum(len(c) for c in cand) > 40
    got = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=64)
    exp = _brute(A, B, cand, 64)
    for g, e in zip(got, exp):
        assert np.array_equal(g, e)


@pytest.mark.parametrize("k", [1, 2, 3, 10])
def test_ranking_bruteforce_small_k(orc, k):
    """k below |U|: Hamming ranking by (distance, index) with Python ints."""
    rc, rb = synth.projection_matrices()
    rng = np.random.default_rng(23)
    A = synth.desc(rng, 60)
    B = np.concatenate([synth.noisy(rng, A[:30], sigma=20.0), synth.desc(rng, 50)])
    # fewer bucket bits in play -> large candidate sets: keep only 2 bits per key
    rb2 = rb.copy()
    rb2[:, 2:, :] = 0.0
    codes, keys = orc.build_codes([A, B], rc, rb2)
    cand = [{j for t in range(6) for j in range(len(B)) if keys[1][j, t] == keys[0][q, t]}
            for q in range(len(A))]
    assert np.mean([len(c) for c in cand]) > 3 * k
    got = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=k)
    exp = _brute(A, B, cand, k, codes[0], codes[1])
    for g, e in zip(got, exp):
        assert np.array_equal(g, e)


def test_hamming_ranking_excludes_far_code(orc):
    """The Euclidean-nearest candidate is dropped when its Hamming distance is
    not among the k smallest (Step 3 ranking happens before Step 4).
    Identity code rows, set {q, B0..B3}: means of components 0..7 are
    (44, 38, 38, 30, 18, 10, 10, 10), so the code bits are
    q {1,2,3}, B0 {1,2,4}, B1 {1..7}, B2 {}, B3 {0,1,2,3} and the Hamming
    distances to q are (2, 4, 3, 1); squared distances (3200, 6400, 800, 900)."""
    A = _pad([[40, 40, 40, 40, 0, 0, 0, 0]])
    B = _pad([[40, 40, 40, 0, 40, 0, 0, 0], [40] * 8,
              [30, 30, 30, 30, 10, 10, 10, 10], [70, 40, 40, 40, 0, 0, 0, 0]])
    codes, keys = orc.build_codes([A, B], np.eye(128), np.zeros((6, 8, 128)))
    assert int(codes[0][0, 0]) == 0b1110
    assert [int(c) for c in codes[1][:, 0]] == [0b10110, 0b11111110, 0, 0b1111]
    # k = 2 -> {B3, B0}: d = (900, 3200), 25*900 < 16*3200 -> B3, although B2 is nearer
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=2)
    assert (m[0], d1[0], d2[0]) == (3, 900, 3200)
    # k = 3 -> {B3, B0, B2}: d1 = 800 (B2), d2 = 900, 25*800 >= 16*900 -> no match
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=3)
    assert (m[0], d1[0], d2[0]) == (-1, 800, 900)


def test_self_match(orc):
    rc, rb = synth.projection_matrices()
    A = synth.desc(np.random.default_rng(31), 500)
    assert len(np.unique(A, axis=0)) == 500
    codes, keys = orc.build_codes([A], rc, rb)
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], A, codes[0], keys[0], k=10)
    assert np.array_equal(m, np.arange(500)) and not d1.any() and (d2 > 0).all()
    # planted duplicate rows: d1 = d2 = 0 -> ratio test fails
    A2 = A.copy()
    A2[1] = A2[0]
    codes, keys = orc.build_codes([A2], rc, rb)
    m, d1, d2 = orc.match_pair(A2, codes[0], keys[0], A2, codes[0], keys[0], k=10)
    assert m[0] == -1 and m[1] == -1 and d1[0] == 0 and d2[0] == 0
    assert np.array_equal(m[2:], np.arange(2, 500))


@pytest.mark.parametrize("da,db,expect", [((4,), (5,), False),          # 25*16 == 16*25
                                          ((2, 1, 1, 1), (3, 1, 1), True),  # 25*7 = 175 < 176
                                          ((4,), (5, 1), True)])         # 400 < 416
def test_ratio_boundary(orc, da, db, expect):
    A = np.zeros((1, 128), np.uint8)
    B = _pad([list(da), list(db)])
    codes, keys = orc.build_codes([A, B], np.eye(128), np.zeros((6, 8, 128)))
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=64)
    D1, D2 = sum(v * v for v in da), sum(v * v for v in db)
    assert (d1[0], d2[0]) == (D1, D2)
    assert (m[0] == 0) == expect and (m[0] in (-1, 0))


def test_degenerate_sizes(orc):
    rc, rb = synth.projection_matrices()
    rng = np.random.default_rng(41)
    A, B1 = synth.desc(rng, 20), synth.desc(rng, 1)
    E = np.zeros((0, 128), np.uint8)
    codes, keys = orc.build_codes([A, B1, E], rc, np.zeros((6, 8, 128)))
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], E, codes[2], keys[2])
    assert (m == -1).all() and (d1 == -1).all() and (d2 == -1).all() and len(m) == 20
    m, d1, d2 = orc.match_pair(E, codes[2], keys[2], A, codes[0], keys[0])
    assert len(m) == 0
    m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B1, codes[1], keys[1])
    D = ((A.astype(np.int64) - B1.astype(np.int64)) ** 2).sum(1)
    assert (m == -1).all() and np.array_equal(d1, D) and (d2 == -1).all()


def test_tau_filter(orc):
    rc, rb = synth.projection_matrices()
    w = synth.single_pair()
    codes, keys = orc.build_codes(w.images, rc, rb)
    args = (w.images[0], codes[0], keys[0], w.images[1], codes[1], keys[1])
    full = orc.match_pair(*args, k=10)
    off = orc.match_pair(*args, k=10, tau=128)
    for a, b in zip(full, off):
        assert np.array_equal(a, b)
    zero = orc.match_pair(*args, k=10, tau=0)
    # tau = 0 keeps only identical codes: every survivor has Hamming distance 0
    cq = codes[0][:, 0], codes[0][:, 1]
    for q in np.flatnonzero(zero[1] >= 0)[:50]:
        d = ((w.images[0][q].astype(np.int64) - w.images[1].astype(np.int64)) ** 2).sum(1)
        j = np.flatnonzero(d == zero[1][q])
        assert any(codes[1][jj, 0] == cq[0][q] and codes[1][jj, 1] == cq[1][q] for jj in j)
    assert (zero[1] >= 0).sum() < (full[1] >= 0).sum()


def test_single_pair_statistics(orc):
    """Sanity (not parity): most noisy copies are matched to their source."""
    rc, rb = synth.projection_matrices()
    w = synth.single_pair()
    codes, keys = orc.build_codes(w.images, rc, rb)
    m, d1, d2 = orc.match_pair(w.images[0], codes[0], keys[0], w.images[1], codes[1], keys[1], k=10)
    truth_b = w.truth[1]
    inv = np.full(2000, -1)
    inv[truth_b[truth_b >= 0]] = np.flatnonzero(truth_b >= 0)
    shared = np.arange(1200)
    assert (m[shared] == inv[shared]).mean() > 0.9
    assert (m[1200:] >= 0).mean() < 0.2


# ---------------------------------------------------------------- epipolar

def test_epipolar_rectified_closed_form(orc):
    """F of a rectified pair maps (x, y) to the line y' = y: keep iff
    (y - y')^2 <= d^2 (Eq. 1, inclusive)."""
    F = np.array([0, 0, 0, 0, 0, -1, 0, 1, 0], np.float64)
    A = np.zeros((1, 128), np.uint8)
    B = _pad([[4], [5], [6]])
    codes, keys = orc.build_codes([A, B], np.eye(128), np.zeros((6, 8, 128)))
    kp_q = np.array([[100.0, 0.0]], np.float32)
    on = np.float32(4.0)
    off = np.nextafter(np.float32(4.0), np.float32(5.0))  # 4 + 2^-21
    assert float(off) == 4.0 + 2.0 ** -21
    for y1, y2, y3, exp in [(on, 0.0, 1.0, (-1, 16, 25)),
                            (off, 0.0, 1.0, (-1, 25, 36)),
                            (-on, 9.0, -9.0, (-1, 16, -1))]:
        kp_t = np.array([[7.0, y1], [500.0, y2], [-3.0, y3]], np.float32)
        m, d1, d2 = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=64,
                                   kp_q=kp_q, kp_t=kp_t, F=F, max_px=4.0)
        # 25*16 = 400 == 16*25: the ratio test rejects; the band decides which
        # candidates are compared at all
        assert (m[0], d1[0], d2[0]) == exp


def test_epipolar_huge_band_equals_plain(orc):
    w = synth.epipolar_set(n_images=3, n_feat=400, n_points=2000, n_neighbours=2)
    rc, rb = synth.projection_matrices()
    codes, keys = orc.build_codes(w.images, rc, rb)
    plain = orc.match_pairs(w.images, codes, keys, w.pairs, k=10)
    epi = orc.match_pairs(w.images, codes, keys, w.pairs, k=10, kp=w.kp, F=w.F, max_px=1e7)
    for a, b in zip(plain, epi):
        assert np.array_equal(a, b)
    narrow = orc.match_pairs(w.images, codes, keys, w.pairs, k=10, kp=w.kp, F=w.F, max_px=4.0)
    # true correspondences lie inside the 4 px band: where plain matching found
    # the true partner, it is still among the band's candidates and nearest
    off, kept, total = 0, 0, 0
    for qi, ti in w.pairs:
        n = len(w.images[qi])
        m = plain[0][off:off + n]
        good = np.flatnonzero(m >= 0)
        good = good[w.truth[ti][m[good]] == w.truth[qi][good]]
        total += len(good)
        kept += int((narrow[1][off:off + n][good] == plain[1][off:off + n][good]).sum())
        off += n
    assert total > 300 and kept >= 0.99 * total
    assert (narrow[1] == -1).sum() > (plain[1] == -1).sum()  # the band removes candidates


def test_match_pairs_equals_per_pair(orc):
    rc, rb = synth.projection_matrices()
    w = synth.scene_set(n_images=4, n_feat=300)
    codes, keys = orc.build_codes(w.images, rc, rb)
    flat = orc.match_pairs(w.images, codes, keys, w.pairs, k=10)
    off = 0
    for qi, ti in w.pairs:
        one = orc.match_pair(w.images[qi], codes[qi], keys[qi], w.images[ti], codes[ti], keys[ti], k=10)
        n = len(one[0])
        for a, b in zip(flat, one):
            assert np.array_equal(a[off:off + n], b)
        off += n
    sel = np.array([5, 3, 3, 299], np.int32)
    sub = orc.match_pair(w.images[0], codes[0], keys[0], w.images[1], codes[1], keys[1], k=10, q_idx=sel)
    full = orc.match_pair(w.images[0], codes[0], keys[0], w.images[1], codes[1], keys[1], k=10)
    for a, b in zip(sub, full):
        assert np.array_equal(a, b[sel])


def test_tau_invariant_when_k_candidates_survive(orc):
    """Ranking section: dropping candidates with Hamming distance > tau cannot
    change a query whose k nearest (Hamming, index) candidates all have
    distance <= tau; checked per query against a Python count of the union."""
    rc, rb = synth.projection_matrices()
    w = synth.single_pair(n=1200, n_shared=700)
    codes, keys = orc.build_codes(w.images, rc, rb)
    A, B = w.images
    full = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=10)
    k = 10
    total_checked = 0
    for tau in (56, 60, 64):
        cut = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=k, tau=tau)
        cb = [int(c0) | (int(c1) << 64) for c0, c1 in codes[1]]
        n_same = n_checked = 0
        for q in range(0, len(A), 7):
            cq = int(codes[0][q, 0]) | (int(codes[0][q, 1]) << 64)
            union = {j for t in range(6) for j in np.flatnonzero(keys[1][:, t] == keys[0][q, t])}
            hs = sorted((cq ^ cb[j]).bit_count() for j in union)
            if len(hs) >= k and hs[k - 1] <= tau:
                n_checked += 1
                assert (full[0][q], full[1][q], full[2][q]) == (cut[0][q], cut[1][q], cut[2][q])
            n_same += int(full[0][q] == cut[0][q])
        total_checked += n_checked
    assert total_checked > 50
    # a tau below every Hamming distance of a true match loses matches
    low = orc.match_pair(A, codes[0], keys[0], B, codes[1], keys[1], k=k, tau=2)
    assert (low[0] >= 0).sum() < (full[0] >= 0).sum()
