"""GPU path (C ABI, HIP kernels on gfx950) against the CPU oracle, bit for bit:
codes, keys, match indices and squared distances are integers, so the bar is
exact equality.  Inputs are seeded synthetic workloads (see synth)."""
import numpy as np
import pytest

import oracle
from paper_1805_08995_amd import binding, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


def _np(ts):
    return [t.cpu().numpy() for t in ts]


def _codes_np(codes):
    return [c.cpu().numpy().view(np.uint64) for c in codes]


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def mats():
    return synth.projection_matrices()


def _gpu_codes(m, images):
    dimgs = _dev(images)
    codes, keys, st = m.build_codes(dimgs)
    return dimgs, codes, keys, st


def _assert_codes(codes, keys, oc, ok, tag):
    for i, (c, k) in enumerate(zip(_codes_np(codes), _np(keys))):
        bad = np.flatnonzero((c != oc[i]).any(1) | (k != ok[i]).any(1))
        assert len(bad) == 0, f"{tag}: image {i}: {len(bad)} descriptors differ, first {bad[:5]}"


def _assert_match(got, exp, tag):
    for g, e, name in zip(got, exp, ("match_idx", "d1sq", "d2sq")):
        g = g.cpu().numpy() if hasattr(g, "cpu") else g
        bad = np.flatnonzero(g != e)
        assert len(bad) == 0, f"{tag}: {name}: {len(bad)} of {len(e)} differ, first {bad[:5]}: {g[bad[:5]]} vs {e[bad[:5]]}"


# ------------------------------------------------------------------ codes

@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_codes_single_pair(mats, mode):
    _say(f"codes single pair 2000x2000 mode={mode}")
    w = synth.single_pair()
    oc, ok = oracle.build_codes(w.images, *mats)
    m = binding.Matcher(*mats, mode=mode)
    _, codes, keys, st = _gpu_codes(m, w.images)
    _assert_codes(codes, keys, oc, ok, mode)
    # the margin test flags a small fraction of the 176 projections per descriptor
    assert 0 < st["near_margin_recomputes"] < 0.02 * 4000 * 176


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_codes_exact_ties_and_zero_rows(mats, mode):
    """Identity rows on integer sets with exact ties (projection exactly 0),
    zero bucket rows, ragged image sizes: every near-zero value goes through
    the binary64 recompute and must give the oracle's bit."""
    rng = np.random.default_rng(9)
    ims = [rng.choice([0, 2, 4, 6], size=(n, 128)).astype(np.uint8) for n in (1, 15, 16, 17, 33, 0, 70)]
    rc = np.eye(128)
    rb = np.zeros((6, 8, 128))
    rb[2, 3, 7] = -1.0
    oc, ok = oracle.build_codes(ims, rc, rb)
    m = binding.Matcher(rc, rb, mode=mode)
    _, codes, keys, st = _gpu_codes(m, ims)
    _assert_codes(codes, keys, oc, ok, mode)
    assert st["near_margin_recomputes"] > 100


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_codes_adversarial_near_margin(mats, mode):
    """Descriptors constructed so that many projections sit at or just next to
    zero: pairs x, y differing in two components with rows of +-1 give
    r . (N x - S) in {-1, 0, 1} * small."""
    rng = np.random.default_rng(10)
    base = synth.desc(rng, 40)
    pert = base.copy()
    pert[:, 0] = np.clip(pert[:, 0].astype(int) + 1, 0, 255)
    pert[:, 1] = np.clip(pert[:, 1].astype(int) - 1, 0, 255)
    ims = [base, pert]
    rc = rng.choice([-1.0, 1.0], size=(128, 128))
    rc[:, 0] = rc[:, 1]  # r0 == r1: the +1/-1 perturbation cancels
    rb = rng.choice([-1.0, 0.0, 1.0], size=(6, 8, 128))
    oc, ok = oracle.build_codes(ims, rc, rb)
    m = binding.Matcher(rc, rb, mode=mode, margin_coef=2e-3)
    _, codes, keys, st = _gpu_codes(m, ims)
    _assert_codes(codes, keys, oc, ok, mode)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_codes_every_projection_recomputed(mats, mode):
    """A margin so wide that every projection is flagged: all 176 bits of
    every descriptor come from the binary64 recompute, and each row holds
    more recomputes than its region of the row-sorted job list, so the
    recompute takes its spread form (jobs of any row per wavefront)."""
    _say(f"codes, every projection recomputed, mode={mode}")
    rng = np.random.default_rng(21)
    ims = [synth.desc(rng, n) for n in (1000, 37, 1, 0, 129)]
    oc, ok = oracle.build_codes(ims, *mats)
    m = binding.Matcher(*mats, mode=mode, margin_coef=1e3)
    _, codes, keys, st = _gpu_codes(m, ims)
    _assert_codes(codes, keys, oc, ok, mode)
    assert st["near_margin_recomputes"] == 1167 * 176


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_codes_row_sorted_recompute_many_chunks(mats, mode):
    """60000 descriptors at the default margin: about 80 recomputes per row,
    so rows span two or more 64-job chunks of the row-sorted recompute, with
    room to spare in every row's region."""
    _say(f"codes, 6 x 10000, mode={mode}")
    rng = np.random.default_rng(22)
    ims = [synth.desc(rng, 10000) for _ in range(6)]
    oc, ok = oracle.build_codes(ims, *mats)
    m = binding.Matcher(*mats, mode=mode)
    _, codes, keys, st = _gpu_codes(m, ims)
    _assert_codes(codes, keys, oc, ok, mode)
    assert 64 * 176 < st["near_margin_recomputes"] < 60000


def test_codes_random_matrices_many_sizes(mats):
    """Other seeds, scaled rows and uneven sizes."""
    for seed in (1, 2, 3):
        rng = np.random.default_rng(seed)
        rc = rng.standard_normal((128, 128)) * (0.5 + seed)
        rb = rng.standard_normal((6, 8, 128))
        ims = [synth.desc(rng, n) for n in (3, 500, 1023, 64)]
        oc, ok = oracle.build_codes(ims, rc, rb)
        norms = np.linalg.norm(np.concatenate([rc, rb.reshape(48, 128)]), axis=1)
        coef = max(1e-3, 6e-5 * norms.max())
        for mode in ("batched", "plain"):
            m = binding.Matcher(rc, rb, mode=mode, margin_coef=coef)
            _, codes, keys, _ = _gpu_codes(m, ims)
            _assert_codes(codes, keys, oc, ok, f"seed {seed} {mode}")


def test_codes_one_context_changing_sizes(mats):
    """One context building codes for sets of different image sizes in turn
    (the device keeps the row chunks of the last sizes; a change must
    rebuild them), including an empty image and a set seen before."""
    rng = np.random.default_rng(17)
    sets = [[synth.desc(rng, n) for n in sizes] for sizes in ((700, 16, 1), (33, 0, 2048, 5), (700, 16, 1))]
    m = binding.Matcher(*mats)
    for i, ims in enumerate(sets):
        oc, ok = oracle.build_codes(ims, *mats)
        _, codes, keys, _ = _gpu_codes(m, ims)
        _assert_codes(codes, keys, oc, ok, f"set {i}")


# ------------------------------------------------------------------ matching

def _oracle_all(images, oc, ok, pairs, **kw):
    return oracle.match_pairs(images, oc, ok, pairs, **kw)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_match_single_pair(mats, mode):
    _say(f"match single pair mode={mode}")
    w = synth.single_pair()
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=10)
    m = binding.Matcher(*mats, mode=mode)
    dimgs, codes, keys, _ = _gpu_codes(m, w.images)
    got, st = m.match_pairs(dimgs, codes, keys, w.pairs)
    _assert_match(got, exp, mode)
    assert st["queries"] == 2000 and st["bucket_entries"] >= st["union_size"] > 0
    ms, launches = m.last_kernel_ms()
    assert ms > 0 and launches == 1


@pytest.mark.parametrize("k,tau", [(1, 128), (2, 128), (10, 40), (10, 0), (37, 128), (64, 128), (64, 70)])
def test_match_k_and_tau(mats, k, tau):
    _say(f"match k={k} tau={tau}")
    w = synth.single_pair(n=900, n_shared=500)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=k, tau=tau)
    m = binding.Matcher(*mats, k=k, max_hamming=tau)
    dimgs, codes, keys, _ = _gpu_codes(m, w.images)
    got, _ = m.match_pairs(dimgs, codes, keys, w.pairs)
    _assert_match(got, exp, f"k={k} tau={tau}")


@pytest.mark.parametrize("k", [1, 10, 64])
def test_match_unbounded_candidates(mats, k):
    """Zero bucket rows: all keys 0, so every query's candidate set is the
    whole train image (2500 > the in-LDS list) and the ranking takes the
    re-gather path; many Hamming ties exercise the index digits."""
    rc, _ = mats
    rb = np.zeros((6, 8, 128))
    rng = np.random.default_rng(4)
    A = synth.desc(rng, 300)
    B = np.concatenate([synth.noisy(rng, A[:100]), synth.desc(rng, 2400)])
    oc, ok = oracle.build_codes([A, B], rc, rb)
    pairs = np.array([[0, 1], [1, 0]], np.int32)
    exp = _oracle_all([A, B], oc, ok, pairs, k=k)
    m = binding.Matcher(rc, rb, k=k)
    dimgs, codes, keys, _ = _gpu_codes(m, [A, B])
    got, st = m.match_pairs(dimgs, codes, keys, pairs)
    _assert_match(got, exp, f"unbounded k={k}")
    assert st["union_size"] == 300 * 2500 + 2500 * 300


def test_match_hamming_ties_coarse_codes(mats):
    """Code rows with only 4 distinct rows: Hamming distance takes few values,
    so the k-th candidate's bin holds many ties resolved by index."""
    rng = np.random.default_rng(12)
    rc = np.repeat(rng.standard_normal((4, 128)), 32, axis=0)
    rb = rng.standard_normal((6, 8, 128))
    rb[:, 3:, :] = 0.0
    A = synth.desc(rng, 400)
    B = np.concatenate([synth.noisy(rng, A[:150]), synth.desc(rng, 700)])
    oc, ok = oracle.build_codes([A, B], rc, rb)
    pairs = np.array([[0, 1]], np.int32)
    for k in (3, 10, 50):
        exp = _oracle_all([A, B], oc, ok, pairs, k=k)
        m = binding.Matcher(rc, rb, k=k)
        dimgs, codes, keys, _ = _gpu_codes(m, [A, B])
        got, _ = m.match_pairs(dimgs, codes, keys, pairs)
        _assert_match(got, exp, f"coarse k={k}")


def test_match_degenerate_images(mats):
    """Empty images, a one-feature train image, self pairs, duplicate rows,
    ragged sizes around the 32-query tile and 64-lane wave."""
    rng = np.random.default_rng(5)
    A = synth.desc(rng, 95)
    A[7] = A[3]  # duplicate rows: d1 == d2 == 0 in self-matching
    ims = [A, np.zeros((0, 128), np.uint8), synth.desc(rng, 1), synth.noisy(rng, A[:65]), synth.desc(rng, 33)]
    oc, ok = oracle.build_codes(ims, *mats)
    pairs = np.array([[0, 0], [0, 1], [1, 0], [0, 2], [2, 0], [3, 0], [0, 3], [4, 3], [1, 1], [3, 3], [2, 2]],
                     np.int32)
    exp = _oracle_all(ims, oc, ok, pairs, k=10)
    for mode in ("batched", "plain"):
        m = binding.Matcher(*mats, mode=mode)
        dimgs, codes, keys, _ = _gpu_codes(m, ims)
        got, _ = m.match_pairs(dimgs, codes, keys, pairs)
        _assert_match(got, exp, f"degenerate {mode}")


def test_match_scene_set_all_pairs_both_forms(mats):
    _say("scene set 8x3000, all pairs, both forms")
    w = synth.scene_set(seed=7, n_images=8, n_feat=3000, n_scenes=3)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=10)
    outs = {}
    for mode in ("batched", "plain"):
        m = binding.Matcher(*mats, mode=mode)
        dimgs, codes, keys, _ = _gpu_codes(m, w.images)
        _assert_codes(codes, keys, oc, ok, mode)
        got, st = m.match_pairs(dimgs, codes, keys, w.pairs)
        _assert_match(got, exp, mode)
        outs[mode] = [g.cpu().numpy() for g in got]
        _, launches = m.last_kernel_ms()
        assert launches == (1 if mode == "batched" else len(w.pairs))
    # reversed and shuffled pair lists give the same per-pair results
    m = binding.Matcher(*mats)
    dimgs, codes, keys, _ = _gpu_codes(m, w.images)
    perm = np.random.default_rng(0).permutation(len(w.pairs))
    got, _ = m.match_pairs(dimgs, codes, keys, w.pairs[perm])
    n = 3000
    g0 = got[0].cpu().numpy().reshape(len(perm), n)
    assert np.array_equal(g0, outs["batched"][0].reshape(len(perm), n)[perm])


def test_match_deterministic_repeat(mats):
    w = synth.scene_set(seed=8, n_images=5, n_feat=2500, n_scenes=2)
    m = binding.Matcher(*mats)
    dimgs, codes, keys, _ = _gpu_codes(m, w.images)
    a, _ = m.match_pairs(dimgs, codes, keys, w.pairs)
    a = [x.cpu().numpy() for x in a]
    for _ in range(3):
        b, _ = m.match_pairs(dimgs, codes, keys, w.pairs)
        for x, y in zip(a, b):
            assert np.array_equal(x, y.cpu().numpy())


def test_bound_buffer_lists(mats):
    """Buffer lists marshalled once (Matcher.bind) give the same codes and
    matches as plain lists, in device and host mode, over repeated calls."""
    w = synth.scene_set(seed=12, n_images=6, n_feat=1800, n_scenes=2)
    imgs = list(w.images)
    imgs[2] = imgs[2][:0]  # an empty image
    oc, ok = oracle.build_codes(imgs, *mats)
    exp = _oracle_all(imgs, oc, ok, w.pairs, k=10)
    m = binding.Matcher(*mats)
    dimgs = _dev(imgs)
    codes = [torch.empty((len(a), 2), dtype=torch.int64, device="cuda") for a in imgs]
    keys = [torch.empty((len(a), 6), dtype=torch.uint8, device="cuda") for a in imgs]
    bi, bc, bk = m.bind(dimgs), m.bind(codes), m.bind(keys)
    n = sum(len(imgs[q]) for q in w.pairs[:, 0])
    outs = tuple(torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3))
    for rep in range(2):
        c, k, _ = m.build_codes(bi, out=(bc, bk))
        _assert_codes(codes, keys, oc, ok, f"bound codes {rep}")
        got, _ = m.match_pairs(bi, c, k, w.pairs, out=outs)
        _assert_match(got, exp, f"bound device {rep}")
    mh = binding.Matcher(*mats, mem="host", device_budget_bytes=4_000_000)
    hb = mh.bind(imgs, np.uint8)
    hc, hk, _ = mh.build_codes(hb)
    got, _ = mh.match_pairs(hb, mh.bind(hc), mh.bind(hk), w.pairs)
    _assert_match(got, exp, "bound host")


# ------------------------------------------------------------------ epipolar

@pytest.mark.parametrize("k", [10, 33, 64])
def test_epipolar_small_set(mats, k):
    """The band kernel's tiles hold at most 320 kept candidates (32 queries
    at k = 10, 9 at k = 33, 5 at k = 64)."""
    _say(f"epipolar 10 images x 3000 k={k}")
    w = synth.epipolar_set(seed=6, n_images=10, n_feat=3000, n_points=20000, n_neighbours=4)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = oracle.match_pairs(w.images, oc, ok, w.pairs, k=k, kp=w.kp, F=w.F, max_px=4.0)
    for mode in ("batched", "plain"):
        m = binding.Matcher(*mats, mode=mode, k=k)
        dimgs, codes, keys, _ = _gpu_codes(m, w.images)
        dkp = _dev(w.kp)
        got, st = m.match_pairs_epipolar(dimgs, codes, keys, dkp, w.pairs, w.F, 4.0)
        _assert_match(got, exp, f"epipolar {mode} k={k}")
        assert st["union_size"] < st["bucket_entries"]
    # a band wider than any image equals plain matching
    plain = oracle.match_pairs(w.images, oc, ok, w.pairs, k=k)
    got, _ = m.match_pairs_epipolar(dimgs, codes, keys, dkp, w.pairs, w.F, 1e7)
    _assert_match(got, plain, f"epipolar huge band k={k}")


@pytest.mark.parametrize("k", [1, 10])
def test_epipolar_unbounded_candidates_huge_band(mats, k):
    """Zero bucket rows and a band wider than the images: every bucket entry
    (6 x 1080 per query) survives the band pass, more than the register
    slots and the LDS list hold, so the band kernel takes its fallback path
    (band test per entry during the gather); results equal plain matching."""
    _say(f"epipolar unbounded candidates k={k}")
    rc, _ = mats
    rb = np.zeros((6, 8, 128))
    rng = np.random.default_rng(14)
    A = synth.desc(rng, 200)
    B = np.concatenate([synth.noisy(rng, A[:80]), synth.desc(rng, 1000)])
    oc, ok = oracle.build_codes([A, B], rc, rb)
    pairs = np.array([[0, 1], [1, 0]], np.int32)
    exp = _oracle_all([A, B], oc, ok, pairs, k=k)
    m = binding.Matcher(rc, rb, k=k)
    dimgs, codes, keys, _ = _gpu_codes(m, [A, B])
    kp = [rng.uniform(0, 1000, (len(A), 2)).astype(np.float32), rng.uniform(0, 1000, (len(B), 2)).astype(np.float32)]
    F = np.tile(np.array([[0, 0, 0, 0, 0, -1, 0, 1, 0]], np.float64), (2, 1))
    got, st = m.match_pairs_epipolar(dimgs, codes, keys, _dev(kp), pairs, F, 1e7)
    _assert_match(got, exp, f"epipolar unbounded k={k}")
    assert st["union_size"] == 200 * 1080 + 1080 * 200


def test_epipolar_rectified_boundary(mats):
    """Rectified F: keep iff (y - y')^2 <= d^2; y' = 4 kept, 4 + 2^-21 dropped."""
    F = np.array([[0, 0, 0, 0, 0, -1, 0, 1, 0]], np.float64)
    A = np.zeros((1, 128), np.uint8)
    B = np.zeros((3, 128), np.uint8)
    B[:, 0] = [4, 5, 6]
    oc, ok = oracle.build_codes([A, B], np.eye(128), np.zeros((6, 8, 128)))
    pairs = np.array([[0, 1]], np.int32)
    m = binding.Matcher(np.eye(128), np.zeros((6, 8, 128)), k=64)
    dimgs, codes, keys, _ = _gpu_codes(m, [A, B])
    off = float(np.nextafter(np.float32(4.0), np.float32(5.0)))
    for ys in ([4.0, 0.0, 1.0], [off, 0.0, 1.0], [-4.0, 9.0, -9.0]):
        kp = [np.array([[100.0, 0.0]], np.float32), np.array([[7.0, ys[0]], [500.0, ys[1]], [-3.0, ys[2]]], np.float32)]
        exp = oracle.match_pairs([A, B], oc, ok, pairs, k=64, kp=kp, F=F, max_px=4.0)
        got, _ = m.match_pairs_epipolar(dimgs, codes, keys, _dev(kp), pairs, F, 4.0)
        _assert_match(got, exp, f"rectified {ys}")


# ------------------------------------------------------------------ host-memory mode

@pytest.mark.parametrize("budget", [0, 6_000_000, 2_500_000])
def test_host_memory_mode_streams_blocks(mats, budget):
    """Numpy inputs streamed by the library in scheduled blocks (budgets that
    force 1, several and many blocks) equal the oracle and the device mode."""
    _say(f"host mode budget={budget}")
    w = synth.scene_set(seed=9, n_images=9, n_feat=1500, n_scenes=3)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=10)
    m = binding.Matcher(*mats, mem="host", device_budget_bytes=budget)
    codes, keys, st = m.build_codes(w.images)
    for i in range(len(w.images)):
        assert np.array_equal(codes[i], oc[i]) and np.array_equal(keys[i], ok[i])
    got, st = m.match_pairs(w.images, codes, keys, w.pairs)
    _assert_match(got, exp, f"host budget {budget}")
    assert st["h2d_bytes"] > 0 and st["d2h_bytes"] == 12 * st["queries"]
    if budget == 2_500_000:
        assert st["image_loads"] > len(w.images)


@pytest.mark.parametrize("budget", [0, 6_000_000])
def test_host_memory_many_parts(mats, monkeypatch, budget):
    """Host mode with each scheduler step split into many small parts (the
    part size lowered from 2^24 queries to 2500): every part's download runs
    on its own stream while the next part computes, on two alternating output
    buffers; ragged image sizes give parts of uneven length.  The outputs
    equal the oracle's, over two calls in a row."""
    _say(f"host mode, small parts, budget={budget}")
    w = synth.uneven_set(seed=12, n_images=24, lo=300, hi=3000, n_scenes=4, n_partners=5)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=10)
    monkeypatch.setenv("CASHASH_PART_QUERIES", "2500")
    m = binding.Matcher(*mats, mem="host", device_budget_bytes=budget)
    for call in range(2):
        got, st = m.match_pairs(w.images, oc, ok, w.pairs)
        _assert_match(got, exp, f"host small parts budget {budget} call {call}")
        assert st["d2h_bytes"] == 12 * st["queries"]
        if budget:
            assert st["image_loads"] > len(w.images)  # blocks streamed and reloaded


def test_host_memory_epipolar(mats):
    w = synth.epipolar_set(seed=11, n_images=6, n_feat=1200, n_points=8000, n_neighbours=2)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = oracle.match_pairs(w.images, oc, ok, w.pairs, k=10, kp=w.kp, F=w.F, max_px=4.0)
    m = binding.Matcher(*mats, mem="host", device_budget_bytes=3_000_000)
    got, st = m.match_pairs_epipolar(w.images, oc, ok, w.kp, w.pairs, w.F, 4.0)
    _assert_match(got, exp, "host epipolar")


# ------------------------------------------------------------------ error paths

def test_errors_raise(mats):
    m = binding.Matcher(*mats)
    w = synth.single_pair(n=64, n_shared=10)
    dimgs, codes, keys, _ = _gpu_codes(m, w.images)
    with pytest.raises(binding.CashashError) as e:
        m.match_pairs(dimgs, codes, keys, np.array([[0, 5]], np.int32))
    assert e.value.code == binding.E_INVAL
    big = torch.zeros((70000, 128), dtype=torch.uint8, device="cuda")
    with pytest.raises(binding.CashashError) as e:
        m.build_codes([big])
    assert e.value.code == binding.E_LIMIT
    with pytest.raises(binding.CashashError) as e:
        kp = _dev([np.zeros((64, 2), np.float32)] * 2)
        m.match_pairs_epipolar(dimgs, codes, keys, kp, w.pairs, np.full(9, np.nan), 4.0)
    assert e.value.code == binding.E_INVAL
    # the context still works after errors
    got, _ = m.match_pairs(dimgs, codes, keys, w.pairs)
    assert got[0].shape[0] == 64


# ------------------------------------------------------------------ graph replays

def test_graph_replays_match_eager(mats, monkeypatch):
    """The batched matcher launch is captured once and replayed; every replay,
    with unrelated eager work and synchronisations in between, equals the
    result of a context that never uses graphs."""
    w = synth.scene_set(seed=13, n_images=6, n_feat=2000, n_scenes=2)
    monkeypatch.setenv("CASHASH_GRAPHS", "0")
    eager = binding.Matcher(*mats)
    monkeypatch.delenv("CASHASH_GRAPHS")
    graphed = binding.Matcher(*mats)
    dimgs, codes, keys, _ = _gpu_codes(eager, w.images)
    ref, st = eager.match_pairs(dimgs, codes, keys, w.pairs)
    ref = [r.cpu().numpy() for r in ref]
    assert st["graph_replayed"] == 0
    out = tuple(torch.full((len(ref[0]),), -7, dtype=torch.int32, device="cuda") for _ in range(3))
    other = w.pairs[::-1].copy()
    replays = 0
    for it in range(5):
        for o in out:
            o.fill_(-7)
        got, st = graphed.match_pairs(dimgs, codes, keys, w.pairs, out=out)
        replays += st["graph_replayed"]
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert np.array_equal(g.cpu().numpy(), r), f"replay {it}"
        # eager work between replays: other calls on both contexts
        eager.match_pairs(dimgs, codes, keys, other)
        graphed.build_codes(dimgs)
        torch.cuda.synchronize()
    assert replays >= 3


def test_autotune_cache_file_and_fixed_shape(mats, monkeypatch, tmp_path):
    """The autotuner writes its choice as a JSON line to CASHASH_AUTOTUNE_CACHE
    and a new context reuses it; CASHASH_AUTOTUNE=0 uses the fixed default.
    Every launch shape gives the same outputs."""
    import json
    w = synth.scene_set(seed=14, n_images=4, n_feat=1500, n_scenes=2)
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("CASHASH_AUTOTUNE_CACHE", str(cache))
    m1 = binding.Matcher(*mats)
    dimgs, codes, keys, _ = _gpu_codes(m1, w.images)
    ref, st1 = m1.match_pairs(dimgs, codes, keys, w.pairs)
    ref = [r.cpu().numpy() for r in ref]
    lines = [json.loads(x) for x in cache.read_text().splitlines()]
    assert len(lines) == 1 and lines[0]["qt"] == st1["tile_queries"] and lines[0]["key"].startswith("gfx950/batched")
    m2 = binding.Matcher(*mats)
    got, st2 = m2.match_pairs(dimgs, codes, keys, w.pairs)
    assert (st2["tile_queries"], st2["blocks_per_cu"]) == (st1["tile_queries"], st1["blocks_per_cu"])
    assert len(cache.read_text().splitlines()) == 1  # reused, not tuned again
    monkeypatch.delenv("CASHASH_AUTOTUNE_CACHE")
    monkeypatch.setenv("CASHASH_AUTOTUNE", "0")
    m3 = binding.Matcher(*mats)
    got3, st3 = m3.match_pairs(dimgs, codes, keys, w.pairs)
    for a, b, c in zip(ref, got, got3):
        assert np.array_equal(a, b.cpu().numpy()) and np.array_equal(a, c.cpu().numpy())


# ------------------------------------------------------------------ stream order

def test_inputs_written_by_queued_torch_work(mats):
    """A context made without a stream runs on its own stream, yet follows
    the caller's default stream: inputs whose writes are still queued there
    behind slow work are read only after those writes (codes, then matches,
    equal the oracle)."""
    w = synth.single_pair(n=900, n_shared=500)
    oc, ok = oracle.build_codes(w.images, *mats)
    exp = _oracle_all(w.images, oc, ok, w.pairs, k=10)
    m = binding.Matcher(*mats)
    src = _dev(w.images)
    dst = [torch.zeros_like(s) for s in src]
    torch.cuda.synchronize()

    def slow():
        a = torch.randn(4096, 4096, device="cuda")
        for _ in range(12):
            a = a @ a
            a = a / a.abs().max()
        return a

    slow()
    for s, d in zip(src, dst):
        d.copy_(s)  # queued behind the products on the default stream
    codes, keys, _ = m.build_codes(dst)
    _assert_codes(codes, keys, oc, ok, "codes after queued writes")
    c2 = [torch.zeros_like(c) for c in codes]
    k2 = [torch.zeros_like(k) for k in keys]
    torch.cuda.synchronize()
    slow()
    for a, b in zip(c2 + k2, list(codes) + list(keys)):
        a.copy_(b)
    got, _ = m.match_pairs(dst, c2, k2, w.pairs)
    _assert_match(got, exp, "matches after queued writes")
