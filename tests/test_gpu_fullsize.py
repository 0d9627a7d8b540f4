"""Full-size workloads on the GPU, every pair checked against the oracle.

The oracle's outputs of these workloads are stored as digests (per image:
codes and keys; per pair: match_idx, d1sq and d2sq over all its queries) in
tests/golden/fullsize_<name>.npz, written by tests/golden/make_fullsize_digests.py
from the CPU oracle alone.  The GPU's outputs are digested the same way and
every image and every pair must agree.

  scenes   : 100 images x 8000 features, 4950 exhaustive pairs, in the launch
             configuration bench.py times (device memory, batched, autotuned),
             and in the plain per-pair form.
  uneven   : 2000 images of 1000-20000 features (log-uniform), 30 partners
             each (60000 pairs; the 4-, 6- and 8-slot matchers); device mode,
             and host mode streamed in scheduled blocks under a 3 GB device
             budget.
  epipolar : 500 images x 12000 features, 15000 neighbour pairs, 4 px band.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1805_08995_amd import binding, synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from digests import code_digests, pair_digests, pair_offsets  # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, flush=True)


def _golden(name):
    return np.load(os.path.join(GOLDEN, f"fullsize_{name}.npz"))


def _dev_flat(images):
    flat = torch.from_numpy(np.concatenate(images)).cuda()
    offs = np.concatenate([[0], np.cumsum([im.shape[0] for im in images])])
    return [flat[offs[i]:offs[i + 1]] for i in range(len(images))]


def _check_codes(g, codes, keys, tag):
    c = [x.cpu().numpy().view(np.uint64) if hasattr(x, "cpu") else x for x in codes]
    k = [x.cpu().numpy() if hasattr(x, "cpu") else x for x in keys]
    bad = np.flatnonzero(code_digests(c, k) != g["code_digest"])
    assert len(bad) == 0, f"{tag}: codes or keys of {len(bad)} images differ from the oracle, first {bad[:8]}"


def _check_pairs(g, w, got, tag):
    got = [x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x) for x in got]
    assert len(got[0]) == int(g["n_queries"])
    d = pair_digests(*got, pair_offsets(w.n_feat, w.pairs))
    bad = np.flatnonzero(d != g["pair_digest"])
    assert len(bad) == 0, (f"{tag}: {len(bad)} of {len(d)} pairs differ from the oracle, first "
                           f"{[(int(p), tuple(int(x) for x in w.pairs[p])) for p in bad[:6]]}")
    assert int((got[0] >= 0).sum()) == int(g["n_matches"])
    _say(f"{tag}: all {len(d)} pairs equal the oracle ({int(g['n_matches'])} matches)")
    return got


def test_scenes_full_size_bench_configuration():
    _say("full size: scenes 100 x 8000, 4950 pairs (bench configuration)")
    g = _golden("scenes")
    w = synth.scene_set()
    mats = synth.projection_matrices()
    d = _dev_flat(w.images)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, st = m.build_codes(d)
    _check_codes(g, codes, keys, "batched codes")
    _say(f"codes equal; near-margin recomputes {st['near_margin_recomputes']}")
    got, stm = m.match_pairs(d, codes, keys, w.pairs)
    _check_pairs(g, w, got, "batched")
    # the plain per-pair form (fp32 projection, one launch per pair)
    mp = binding.Matcher(*mats, mode="plain", mem="device")
    cp, kp, _ = mp.build_codes(d)
    _check_codes(g, cp, kp, "plain codes")
    gp, _ = mp.match_pairs(d, cp, kp, w.pairs)
    _check_pairs(g, w, gp, "plain")


@pytest.fixture(scope="module")
def uneven():
    _say("generating uneven set: 2000 images, 1k-20k features, 60000 pairs")
    return synth.uneven_set()


def test_uneven_full_size_device_and_streamed(uneven):
    w = uneven
    g = _golden("uneven")
    mats = synth.projection_matrices()
    nf = w.n_feat
    assert nf.min() >= 1000 and nf.max() <= 20000 and len(w.pairs) == 60000
    d = _dev_flat(w.images)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, st = m.build_codes(d)
    _check_codes(g, codes, keys, "uneven device codes")
    got, stm = m.match_pairs(d, codes, keys, w.pairs)
    _say(f"device mode done: {stm['queries']} queries, {stm['ms_match']:.1f} ms")
    _check_pairs(g, w, got, "uneven device")
    # host-memory mode: numpy inputs streamed in scheduled blocks
    del d, codes, keys, got
    torch.cuda.empty_cache()
    mh = binding.Matcher(*mats, mode="batched", mem="host", device_budget_bytes=3 << 30)
    hcodes, hkeys, sth = mh.build_codes(w.images)
    _check_codes(g, hcodes, hkeys, "uneven host codes")
    goth, sth2 = mh.match_pairs(w.images, hcodes, hkeys, w.pairs)
    _say(f"host mode: {sth2['image_loads']} image loads, {sth2['h2d_bytes'] / 1e9:.2f} GB up, "
         f"{sth2['ms_match']:.0f} ms")
    assert sth2["image_loads"] > len(w.images)
    _check_pairs(g, w, goth, "uneven host")
    del goth
    # the whole set resident: one scheduler step matched in many parts
    mr = binding.Matcher(*mats, mode="batched", mem="host")
    gotr, str_ = mr.match_pairs(w.images, hcodes, hkeys, w.pairs)
    _say(f"host mode, resident: {str_['image_loads']} image loads, {str_['ms_match']:.0f} ms")
    assert str_["image_loads"] == len(w.images)
    _check_pairs(g, w, gotr, "uneven host resident")


def test_epipolar_full_size():
    _say("generating epipolar set: 500 images x 12000, 15000 pairs")
    g = _golden("epipolar")
    w = synth.epipolar_set()
    assert float(g["max_px"]) == w.max_px
    mats = synth.projection_matrices()
    d = _dev_flat(w.images)
    kp = _dev_flat(w.kp)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, _ = m.build_codes(d)
    _check_codes(g, codes, keys, "epipolar codes")
    got, st = m.match_pairs_epipolar(d, codes, keys, kp, w.pairs, w.F, w.max_px)
    _say(f"epipolar: {st['queries']} queries, union/bucket = {st['union_size'] / st['bucket_entries']:.3f}, "
         f"{st['ms_match']:.1f} ms")
    assert st["union_size"] < 0.2 * st["bucket_entries"]
    _check_pairs(g, w, got, "epipolar")


def test_geometric_full_size():
    """Two-stage matching on 2 scenes x 250 cameras x 12000 features, 15000
    pairs (a third of them across scenes): per-pair status, match and inlier
    counts and F for every pair; stage-2 outputs on sampled queries."""
    from oracle import geometry as G
    _say("generating geometric set: 2 scenes x 250 cameras x 12000, 15000 pairs")
    w = synth.geometric_set()
    mats = synth.projection_matrices()
    d, kp, sc = _dev_flat(w.images), _dev_flat(w.kp), _dev_flat(w.scales)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, _ = m.build_codes(d)
    rand = np.random.default_rng(7).integers(0, 2**32, (256, 8), dtype=np.uint64).astype(np.uint32)
    out, res, st = m.match_pairs_geometric(d, codes, keys, kp, sc, w.pairs, rand)
    got = [o.cpu().numpy() for o in out]
    ms = m.last_geometric_ms()
    _say(f"GPU: accepted {int((res['status'] == 0).sum())} of {len(w.pairs)}; ms subset {ms[0]:.2f}, "
         f"stage 1 {ms[1]:.2f}, F {ms[2]:.2f}, stage 2 {ms[3]:.2f}")
    # oracle: subsets and their codes, stage 1 over every pair, F for every pair
    S, N = oracle.column_sums(w.images)
    rows = [G.top_scale(s) for s in w.scales]
    sub = [w.images[i][r] for i, r in enumerate(rows)]
    sc_k = [oracle.project(x, S, N, *mats) for x in sub]
    m1 = oracle.match_pairs(sub, [c for c, _ in sc_k], [k for _, k in sc_k], w.pairs)
    nq1 = np.array([len(rows[q]) for q in w.pairs[:, 0]])
    off1 = np.concatenate([[0], np.cumsum(nq1)])
    ql, tl = [], []
    for p, (qi, ti) in enumerate(w.pairs):
        a, b = G.stage1_points(w.kp[qi][rows[qi]], w.kp[ti][rows[ti]], m1[0][off1[p]:off1[p + 1]])
        ql.append(a)
        tl.append(b)
    est, F, ni, _ = G.fundamental_batch(ql, tl, rand)
    assert np.array_equal(res["n_matches"], [len(a) for a in ql])
    assert np.array_equal(res["status"], est)
    assert np.array_equal(res["n_inliers"], ni)
    assert np.array_equal(res["F"], F)
    same = np.array([np.any(f != 0) for f in w.F])
    _say(f"per-pair results equal the oracle; same-scene accepted {np.mean(est[same] == 0):.3f}, "
         f"cross-scene accepted {np.mean(est[~same] == 0):.3f}")
    assert np.mean(est[same] == 0) > 0.95 and np.all(est[~same] != 0)
    # stage 2 on sampled queries of accepted pairs; rejected pairs are all -1
    nq = np.array([w.images[q].shape[0] for q in w.pairs[:, 0]])
    off = np.concatenate([[0], np.cumsum(nq)])
    rng = np.random.default_rng(3)
    acc = np.flatnonzero(est == 0)
    cache = {}

    def full_codes(i):
        if i not in cache:
            cache[i] = oracle.project(w.images[i], S, N, *mats)
        return cache[i]

    for p in rng.choice(acc, size=25, replace=False):
        qi, ti = (int(x) for x in w.pairs[p])
        sel = np.sort(rng.choice(nq[p], size=300, replace=False)).astype(np.int32)
        cq, kq = full_codes(qi)
        ct, kt = full_codes(ti)
        exp = oracle.match_pair(w.images[qi], cq, kq, w.images[ti], ct, kt, k=10, q_idx=sel, kp_q=w.kp[qi],
                                kp_t=w.kp[ti], F=F[p], max_px=w.max_px)
        for g, e in zip(got, exp):
            assert np.array_equal(g[off[p] + sel], e), p
    for p in rng.choice(np.flatnonzero(est != 0), size=20, replace=False):
        assert all(np.all(g[off[p]:off[p + 1]] == -1) for g in got)
    _say("sampled stage-2 queries equal the oracle")
