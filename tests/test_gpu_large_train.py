"""Train images above 9000 points against the oracle, bit for bit.

Pairs whose train image has 9001-14000 points run the 6-register-slot
matcher, above 14000 the 8-slot one (in both the batched and the plain
per-pair form), each in two instantiations: without a Hamming filter
(tau = 128) and with one (tau < 128, the ranking section's threshold).  At
these sizes some queries collect more bucket entries than the register slots
hold, so the LDS-list path runs too.  Query images are small so that the
oracle matches every query of every pair in test time.
"""
import numpy as np
import pytest

import oracle
from paper_1805_08995_amd import binding, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TRAIN_SIZES = (9001, 9600, 13999, 14000, 14001, 16500, 20000)


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def large_set():
    """Two query images (500 and 97 points) and train images of TRAIN_SIZES
    points, each train image holding noisy copies of a share of the first
    query image (so that matches exist) among fresh descriptors."""
    rng = np.random.default_rng(31)
    qa = synth.desc(rng, 500)
    qb = synth.desc(rng, 97)
    trains = []
    for i, n in enumerate(TRAIN_SIZES):
        shared = 150 + 40 * i
        t = np.concatenate([synth.noisy(rng, qa[:shared]), synth.desc(rng, n - shared)])
        trains.append(t[rng.permutation(n)])
    images = [qa, qb] + trains
    pairs = np.array([(q, 2 + i) for i in range(len(TRAIN_SIZES)) for q in (0, 1)], np.int32)
    mats = synth.projection_matrices()
    oc, ok = oracle.build_codes(images, *mats)
    return dict(images=images, pairs=pairs, mats=mats, oc=oc, ok=ok)


def _assert_match(got, exp, tag):
    for g, e, name in zip(got, exp, ("match_idx", "d1sq", "d2sq")):
        g = g.cpu().numpy()
        bad = np.flatnonzero(g != e)
        assert len(bad) == 0, f"{tag}: {name}: {len(bad)} of {len(e)} differ, first {bad[:5]}: {g[bad[:5]]} vs {e[bad[:5]]}"


@pytest.mark.parametrize("mode", ["batched", "plain"])
@pytest.mark.parametrize("k,tau", [(10, 128), (10, 40), (10, 56), (37, 128), (37, 48)])
def test_large_train_images(large_set, mode, k, tau):
    w = large_set
    _say(f"large train images {TRAIN_SIZES}: mode={mode} k={k} tau={tau}")
    exp = oracle.match_pairs(w["images"], w["oc"], w["ok"], w["pairs"], k=k, tau=tau)
    m = binding.Matcher(*w["mats"], mode=mode, k=k, max_hamming=tau)
    d = [torch.from_numpy(im).cuda() for im in w["images"]]
    codes, keys, _ = m.build_codes(d)
    for i, (c, kk) in enumerate(zip(codes, keys)):
        assert np.array_equal(c.cpu().numpy().view(np.uint64), w["oc"][i]), f"codes of image {i}"
        assert np.array_equal(kk.cpu().numpy(), w["ok"][i]), f"keys of image {i}"
    got, st = m.match_pairs(d, codes, keys, w["pairs"])
    _assert_match(got, exp, f"{mode} k={k} tau={tau}")
    # the workload reaches past the register slots of the 8-slot kernel for
    # some queries (the LDS-list path) and matches exist
    assert st["bucket_entries"] > 0 and int((exp[0] >= 0).sum()) > 100
    if tau < 128:
        assert st["union_size"] < st["bucket_entries"]
    m.close()


def test_large_train_bucket_entries_reach_every_path(large_set):
    """The fixture is large enough to matter: the 20000-point train image
    gives some queries more than 512 bucket entries (beyond 8 register slots)
    and the 9001-point one some queries with more than 256 (beyond 4)."""
    w = large_set
    kq, kt_small, kt_big = w["ok"][0], w["ok"][2], w["ok"][-1]

    def entries(kt):
        hist = np.stack([np.bincount(kt[:, t], minlength=256) for t in range(6)])
        return hist[np.arange(6)[None, :], kq.astype(np.int64)].sum(1)

    assert (entries(kt_big) > 512).any()
    assert (entries(kt_small) > 256).any()


@pytest.fixture(scope="module")
def max_set():
    """Images at the size limit (65535 points, the 16-bit index of a packed
    candidate key): a 65535-point train image with noisy copies of a 300-point
    query image, and a 65535-point query image whose first 400 points have
    copies in a 2000-point train image; keypoints in a 4000 x 3000 frame."""
    rng = np.random.default_rng(37)
    q_small = synth.desc(rng, 300)
    t_big = np.concatenate([synth.noisy(rng, q_small[:200]), synth.desc(rng, 65535 - 200)])
    t_big = t_big[rng.permutation(65535)]
    q_big = synth.desc(rng, 65535)
    t_small = np.concatenate([synth.noisy(rng, q_big[:400]), synth.desc(rng, 1600)])
    images = [q_small, t_big, q_big, t_small]
    pairs = np.array([(0, 1), (2, 3), (1, 0), (3, 3)], np.int32)
    kp = [rng.uniform((0, 0), (4000, 3000), size=(len(im), 2)).astype(np.float32) for im in images]
    F = rng.standard_normal((len(pairs), 9)) * 1e-3
    mats = synth.projection_matrices()
    oc, ok = oracle.build_codes(images, *mats)
    return dict(images=images, pairs=pairs, kp=kp, F=F, mats=mats, oc=oc, ok=ok)


@pytest.mark.parametrize("mode", ["batched", "plain"])
@pytest.mark.parametrize("k", [10, 64])
def test_maximum_image_size(max_set, mode, k):
    """Codes, matches and the band form at the 65535-point limit (the largest
    train index, 65534, must survive the key packing), k up to its maximum;
    one point more is refused."""
    w = max_set
    _say(f"maximum image size: mode={mode} k={k}")
    m = binding.Matcher(*w["mats"], mode=mode, k=k)
    d = [torch.from_numpy(im).cuda() for im in w["images"]]
    codes, keys, _ = m.build_codes(d)
    for i, (c, kk) in enumerate(zip(codes, keys)):
        assert np.array_equal(c.cpu().numpy().view(np.uint64), w["oc"][i]), f"codes of image {i}"
        assert np.array_equal(kk.cpu().numpy(), w["ok"][i]), f"keys of image {i}"
    exp = oracle.match_pairs(w["images"], w["oc"], w["ok"], w["pairs"], k=k)
    got, _ = m.match_pairs(d, codes, keys, w["pairs"])
    _assert_match(got, exp, f"{mode} k={k}")
    # the allocation-free entry point takes the same call within its scratch
    outs = tuple(torch.full((len(exp[0]),), -7, dtype=torch.int32, device="cuda") for _ in range(3))
    got_n, _ = m.match_pairs_noalloc(d, codes, keys, w["pairs"], outs)
    _assert_match(got_n, exp, f"{mode} k={k} noalloc")
    # the largest indices occur among the matches of the 65535-point train image
    n0 = len(w["images"][0])
    assert int(exp[0][:n0].max()) > 60000
    kp = [torch.from_numpy(a).cuda() for a in w["kp"]]
    exp_e = oracle.match_pairs(w["images"], w["oc"], w["ok"], w["pairs"], k=k, kp=w["kp"], F=w["F"], max_px=300.0)
    got_e, _ = m.match_pairs_epipolar(d, codes, keys, kp, w["pairs"], w["F"], 300.0)
    _assert_match(got_e, exp_e, f"{mode} k={k} band")
    with pytest.raises(binding.CashashError) as e:
        m.build_codes([torch.zeros((65536, 128), dtype=torch.uint8, device="cuda")])
    assert e.value.code == binding.E_LIMIT
    m.close()
