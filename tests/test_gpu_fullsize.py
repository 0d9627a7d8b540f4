"""Full-size workloads on the GPU, checked against the oracle on sampled
outputs (the oracle cannot match every pair in test time) and, where two GPU
forms exist, against each other in full.

  scenes   : 100 images x 8000 features, 4950 exhaustive pairs, in the launch
             configuration bench.py times (device memory, batched, autotuned);
             codes and keys compared in full.
  uneven   : 2000 images of 1000-20000 features (log-uniform), 30 partners
             each (60000 pairs); device mode, and host mode streamed in
             scheduled blocks under a 3 GB device budget.
  epipolar : 500 images x 12000 features, 15000 neighbour pairs, 4 px band.
"""
import numpy as np
import pytest

import oracle
from paper_1805_08995_amd import binding, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


def _dev_flat(images):
    flat = torch.from_numpy(np.concatenate(images)).cuda()
    offs = np.concatenate([[0], np.cumsum([im.shape[0] for im in images])])
    return [flat[offs[i]:offs[i + 1]] for i in range(len(images))]


def _pair_offsets(images, pairs):
    nq = np.array([images[q].shape[0] for q in pairs[:, 0]], np.int64)
    return np.concatenate([[0], np.cumsum(nq)])


def _check_sampled(w, S, N, mats, got, sample_pairs, n_q_per_pair, rng, **kw):
    """Oracle on sampled (pair, query) outputs.  Codes of the sampled images
    come from the oracle itself (column sums over the whole set)."""
    off = _pair_offsets(w.images, w.pairs)
    cache = {}

    def codes(m):
        if m not in cache:
            cache[m] = oracle.project(w.images[m], S, N, *mats)
        return cache[m]

    checked = 0
    for p in sample_pairs:
        qi, ti = (int(x) for x in w.pairs[p])
        nq = w.images[qi].shape[0]
        if nq == 0:
            continue
        sel = np.sort(rng.choice(nq, size=min(nq, n_q_per_pair), replace=False)).astype(np.int32)
        cq, kq = codes(qi)
        ct, kt = codes(ti)
        extra = {}
        if "F" in kw:
            extra = dict(kp_q=w.kp[qi], kp_t=w.kp[ti], F=w.F[p], max_px=kw["max_px"])
        exp = oracle.match_pair(w.images[qi], cq, kq, w.images[ti], ct, kt, k=10, q_idx=sel, **extra)
        for g, e, name in zip(got, exp, ("match_idx", "d1sq", "d2sq")):
            gv = g[off[p] + sel]
            bad = np.flatnonzero(gv != e)
            assert len(bad) == 0, f"pair {p} ({qi},{ti}) {name}: {len(bad)} differ, e.g. q={sel[bad[:3]]} {gv[bad[:3]]} vs {e[bad[:3]]}"
        checked += len(sel)
    return checked


def test_scenes_full_size_bench_configuration():
    _say("full size: scenes 100 x 8000, 4950 pairs (bench configuration)")
    w = synth.scene_set()
    mats = synth.projection_matrices()
    d = _dev_flat(w.images)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, st = m.build_codes(d)
    oc, ok = oracle.build_codes(w.images, *mats)
    for i in range(len(w.images)):
        assert np.array_equal(codes[i].cpu().numpy().view(np.uint64), oc[i]), f"codes of image {i}"
        assert np.array_equal(keys[i].cpu().numpy(), ok[i]), f"keys of image {i}"
    _say(f"codes equal; near-margin recomputes {st['near_margin_recomputes']}")
    got, stm = m.match_pairs(d, codes, keys, w.pairs)
    got = [g.cpu().numpy() for g in got]
    S, N = oracle.column_sums(w.images)
    rng = np.random.default_rng(0)
    sample = rng.choice(len(w.pairs), size=40, replace=False)
    n = _check_sampled(w, S, N, mats, got, sample, 400, rng)
    # two pairs in full
    for p in sample[:2]:
        qi, ti = w.pairs[p]
        exp = oracle.match_pair(w.images[qi], oc[qi], ok[qi], w.images[ti], oc[ti], ok[ti], k=10)
        off = _pair_offsets(w.images, w.pairs)
        for g, e in zip(got, exp):
            assert np.array_equal(g[off[p]:off[p + 1]], e)
    _say(f"sampled {n} queries equal the oracle")
    # the plain per-pair form gives identical outputs
    mp = binding.Matcher(*mats, mode="plain", mem="device")
    cp, kp, _ = mp.build_codes(d)
    for i in range(len(w.images)):
        assert torch.equal(cp[i], codes[i]) and torch.equal(kp[i], keys[i])
    gp, _ = mp.match_pairs(d, cp, kp, w.pairs)
    for a, b in zip(got, gp):
        assert np.array_equal(a, b.cpu().numpy())


@pytest.fixture(scope="module")
def uneven():
    _say("generating uneven set: 2000 images, 1k-20k features, 60000 pairs")
    return synth.uneven_set()


def test_uneven_full_size_device_and_streamed(uneven):
    w = uneven
    mats = synth.projection_matrices()
    nf = w.n_feat
    assert nf.min() >= 1000 and nf.max() <= 20000 and len(w.pairs) == 60000
    d = _dev_flat(w.images)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, st = m.build_codes(d)
    got, stm = m.match_pairs(d, codes, keys, w.pairs)
    got = [g.cpu().numpy() for g in got]
    _say(f"device mode done: {stm['queries']} queries, {stm['ms_match']:.1f} ms")
    S, N = oracle.column_sums(w.images)
    rng = np.random.default_rng(1)
    # codes of sampled images in full
    for i in rng.choice(len(w.images), size=12, replace=False):
        c, k = oracle.project(w.images[i], S, N, *mats)
        assert np.array_equal(codes[i].cpu().numpy().view(np.uint64), c) and np.array_equal(keys[i].cpu().numpy(), k)
    # the largest and smallest pairs are in the sample
    cost = nf[w.pairs[:, 0]].astype(np.int64) * nf[w.pairs[:, 1]]
    sample = np.concatenate([[np.argmax(cost), np.argmin(cost)], rng.choice(len(w.pairs), size=30, replace=False)])
    n = _check_sampled(w, S, N, mats, got, sample, 300, rng)
    _say(f"sampled {n} queries equal the oracle")
    # host-memory mode: numpy inputs streamed in scheduled blocks
    del d, codes, keys
    torch.cuda.empty_cache()
    mh = binding.Matcher(*mats, mode="batched", mem="host", device_budget_bytes=3 << 30)
    hcodes, hkeys, sth = mh.build_codes(w.images)
    goth, sth2 = mh.match_pairs(w.images, hcodes, hkeys, w.pairs)
    _say(f"host mode: {sth2['image_loads']} image loads, {sth2['h2d_bytes'] / 1e9:.2f} GB up, "
         f"{sth2['ms_match']:.0f} ms")
    assert sth2["image_loads"] > len(w.images)
    for a, b in zip(got, goth):
        assert np.array_equal(a, b)


def test_epipolar_full_size():
    _say("generating epipolar set: 500 images x 12000, 15000 pairs")
    w = synth.epipolar_set()
    mats = synth.projection_matrices()
    d = _dev_flat(w.images)
    kp = _dev_flat(w.kp)
    m = binding.Matcher(*mats, mode="batched", mem="device")
    codes, keys, _ = m.build_codes(d)
    got, st = m.match_pairs_epipolar(d, codes, keys, kp, w.pairs, w.F, w.max_px)
    got = [g.cpu().numpy() for g in got]
    _say(f"epipolar: {st['queries']} queries, union/bucket = {st['union_size'] / st['bucket_entries']:.3f}, "
         f"{st['ms_match']:.1f} ms")
    assert st["union_size"] < 0.2 * st["bucket_entries"]
    S, N = oracle.column_sums(w.images)
    rng = np.random.default_rng(2)
    sample = rng.choice(len(w.pairs), size=30, replace=False)
    n = _check_sampled(w, S, N, mats, got, sample, 400, rng, F=True, max_px=w.max_px)
    _say(f"sampled {n} queries equal the oracle")


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
