"""Geometry-aware two-stage matching on the GPU against the oracle, bit for
bit: top-scale subsets, row gathers, RANSAC fundamental matrices (F, inlier
counts, best hypothesis, status) and the whole two-stage call."""
import numpy as np
import pytest

import oracle
from oracle import geometry as G
from paper_1805_08995_amd import binding, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


def _rand(h, seed=7):
    return np.random.default_rng(seed).integers(0, 2**32, (h, 8), dtype=np.uint64).astype(np.uint32)


@pytest.fixture(scope="module")
def m():
    return binding.Matcher(*synth.projection_matrices(), mode="batched", mem="device")


def _cuda(arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


# ---- subset -----------------------------------------------------------------

@pytest.mark.parametrize("frac", [(1, 5), (1, 1), (2, 3)])
def test_top_scale_parity(m, frac):
    rng = np.random.default_rng(11)
    sizes = [0, 1, 5, 7, 255, 256, 257, 3001, 12000, 65535]
    scales = []
    for i, n in enumerate(sizes):
        if i % 3 == 0:
            s = rng.integers(1, 30, n).astype(np.float32) * np.float32(0.5)     # heavy ties
        elif i % 3 == 1:
            s = rng.lognormal(0.0, 1.0, n).astype(np.float32)
        else:
            s = rng.choice(np.array([-0.0, 0.0, -1.5, 2.0, np.inf, -np.inf, 1e-38, 3.0], np.float32), n)
        scales.append(s)
    _say(f"top scale, fraction {frac}, sizes {sizes}")
    rows = m.select_top_scale(_cuda(scales), frac)
    for s, r in zip(scales, rows):
        assert np.array_equal(r.cpu().numpy(), G.top_scale(s, frac)), len(s)


# ---- gather -------------------------------------------------------------------

def test_gather_rows_parity_and_range_check(m):
    rng = np.random.default_rng(12)
    nf = [0, 3, 1000, 4097]
    desc = [rng.integers(0, 256, (n, 128), dtype=np.uint8) for n in nf]
    codes = [rng.integers(0, 2**63, (n, 2), dtype=np.int64) for n in nf]
    keys = [rng.integers(0, 256, (n, 6), dtype=np.uint8) for n in nf]
    kp = [rng.uniform(0, 1000, (n, 2)).astype(np.float32) for n in nf]
    rows = [np.sort(rng.choice(n, size=n // 2, replace=False)).astype(np.int32) if n else np.zeros(0, np.int32)
            for n in nf]
    rows[1] = np.array([2, 0, 2], np.int32)           # repeats and any order are allowed
    od, oc, ok, okp = m.gather_rows(_cuda(rows), nf, _cuda(desc), _cuda(codes), _cuda(keys), _cuda(kp))
    for i in range(len(nf)):
        assert np.array_equal(od[i].cpu().numpy(), desc[i][rows[i]])
        assert np.array_equal(oc[i].cpu().numpy(), codes[i][rows[i]])
        assert np.array_equal(ok[i].cpu().numpy(), keys[i][rows[i]])
        assert np.array_equal(okp[i].cpu().numpy(), kp[i][rows[i]])
    # one field only
    od2, oc2, ok2, okp2 = m.gather_rows(_cuda(rows), nf, kp=_cuda(kp))
    assert od2 is None and oc2 is None and ok2 is None
    assert all(np.array_equal(a.cpu().numpy(), b[r]) for a, b, r in zip(okp2, kp, rows))
    bad = [r.copy() for r in rows]
    bad[2][5] = 1000
    with pytest.raises(binding.CashashError):
        m.gather_rows(_cuda(bad), nf, kp=_cuda(kp))


# ---- fundamental matrices ---------------------------------------------------------

def _cameras(rng, angle):
    K = np.array([[1500.0, 0, 960], [0, 1500.0, 540], [0, 0, 1]])

    def cam(th):
        c = np.array([40 * np.cos(th), 40 * np.sin(th), 2.0])
        f = -c / np.linalg.norm(c)
        r = np.cross(f, [0, 0, 1.0])
        r /= np.linalg.norm(r)
        R = np.stack([r, np.cross(f, r), f])
        return R, -R @ c

    Ri, ti = cam(0.3)
    Rj, tj = cam(0.3 + angle)

    def project(X, R, t):
        x = (X @ R.T + t) @ K.T
        return x[:, :2] / x[:, 2:3]

    return (lambda X: project(X, Ri, ti)), (lambda X: project(X, Rj, tj))


def _pair_images(rng, n_true, n_out, extra_q, extra_t, noise, angle=np.pi / 6):
    """Query / train keypoints and the query -> train match list of one pair:
    n_true projections of common 3-D points (with pixel noise), n_out random
    correspondences, extra unmatched points on both sides, all shuffled."""
    Pi, Pj = _cameras(rng, angle)
    X = rng.uniform(-10, 10, (n_true, 3))
    q = np.r_[Pi(X) + rng.standard_normal((n_true, 2)) * noise, rng.uniform([0, 0], [1920, 1080], (n_out, 2))]
    t = np.r_[Pj(X) + rng.standard_normal((n_true, 2)) * noise, rng.uniform([0, 0], [1920, 1080], (n_out, 2))]
    nm = n_true + n_out
    kq = np.r_[q, rng.uniform([0, 0], [1920, 1080], (extra_q, 2))].astype(np.float32)
    kt = np.r_[t, rng.uniform([0, 0], [1920, 1080], (extra_t, 2))].astype(np.float32)
    pq, pt = rng.permutation(len(kq)), rng.permutation(len(kt))
    inv_t = np.argsort(pt)
    match = -np.ones(len(kq), np.int32)
    match[np.argsort(pq)[:nm]] = inv_t[:nm]
    return kq[pq], kt[pt], match


def _fundamental_case(rng, specs):
    kps, pairs, flat = [], [], []
    for spec in specs:
        kq, kt, match = _pair_images(rng, *spec)
        pairs.append((len(kps), len(kps) + 1))
        kps += [kq, kt]
        flat.append(match)
    return kps, np.array(pairs, np.int32), np.concatenate(flat)


def _oracle_fundamental(kps, pairs, flat, rand, thr, min_matches):
    off = 0
    exp = []
    for qi, ti in pairs:
        mt = flat[off:off + len(kps[qi])]
        off += len(kps[qi])
        a, b = G.stage1_points(kps[qi], kps[ti], mt)
        exp.append(G.fundamental(a, b, rand, thr, min_matches) + (len(a),))
    return exp


@pytest.mark.parametrize("n_hyp", [1, 256, 700])
def test_fundamental_parity(m, n_hyp):
    rng = np.random.default_rng(13)
    specs = [(100, 0, 30, 50, 0.0), (150, 50, 400, 100, 0.3), (0, 200, 50, 50, 0.0), (10, 5, 20, 20, 0.0),
             (8, 0, 0, 0, 0.0), (40, 20, 0, 0, 0.5, 0.05), (600, 150, 200, 300, 0.3), (16, 0, 3, 3, 0.2)]
    kps, pairs, flat = _fundamental_case(rng, specs)
    # a pair with coincident query points
    kps.append(np.full((40, 2), 100.0, np.float32))
    kps.append(rng.uniform(0, 1000, (40, 2)).astype(np.float32))
    pairs = np.r_[pairs, [[len(kps) - 2, len(kps) - 1]]].astype(np.int32)
    flat = np.r_[flat, np.arange(40, dtype=np.int32)]
    rand = _rand(n_hyp, seed=n_hyp)
    nf = [len(k) for k in kps]
    _say(f"fundamental: {len(pairs)} pairs, {n_hyp} hypotheses")
    got = m.estimate_fundamental(nf, _cuda(kps), pairs, torch.from_numpy(flat).cuda(), rand, thr=2.0)
    exp = _oracle_fundamental(kps, pairs, flat, rand, 2.0, 16)
    for p, (st, F, ni, bh, nm) in enumerate(exp):
        assert got["n_matches"][p] == nm, p
        assert got["status"][p] == st, (p, got["status"][p], st)
        assert got["best_h"][p] == bh, (p, got["best_h"][p], bh)
        assert got["n_inliers"][p] == ni, (p, got["n_inliers"][p], ni)
        assert np.array_equal(got["F"][p], F), (p, got["F"][p] - F)
    statuses = set(int(s) for s in got["status"])
    if n_hyp >= 256:
        assert {G.ACCEPT, G.FEW_MATCHES, G.DEGENERATE, G.FEW_INLIERS} <= statuses


def test_fundamental_many_matches_uses_large_lds(m):
    # 5000 matches per pair needs an 85 KB LDS list
    rng = np.random.default_rng(14)
    kps, pairs, flat = _fundamental_case(rng, [(4000, 1000, 100, 100, 0.3), (3000, 100, 0, 0, 0.3)])
    rand = _rand(256)
    got = m.estimate_fundamental([len(k) for k in kps], _cuda(kps), pairs, torch.from_numpy(flat).cuda(), rand)
    exp = _oracle_fundamental(kps, pairs, flat, rand, 2.0, 16)
    for p, (st, F, ni, bh, nm) in enumerate(exp):
        assert (got["status"][p], got["n_inliers"][p], got["best_h"][p], got["n_matches"][p]) == (st, ni, bh, nm)
        assert np.array_equal(got["F"][p], F)


def test_fundamental_limits_and_errors(m):
    rng = np.random.default_rng(15)
    kps = [rng.uniform(0, 100, (binding.GEO_MAX_MATCHES + 1, 2)).astype(np.float32),
           rng.uniform(0, 100, (10, 2)).astype(np.float32)]
    flat = -np.ones(len(kps[0]), np.int32)
    with pytest.raises(binding.CashashError) as e:
        m.estimate_fundamental([len(k) for k in kps], _cuda(kps), [[0, 1]], torch.from_numpy(flat).cuda(), _rand(4))
    assert e.value.code == binding.E_LIMIT
    flat = np.zeros(10, np.int32)
    flat[3] = 10                                        # outside the train image
    with pytest.raises(binding.CashashError) as e:
        m.estimate_fundamental([10, 10], _cuda([kps[1], kps[1]]), [[0, 1]], torch.from_numpy(flat).cuda(), _rand(4))
    assert e.value.code == binding.E_INVAL


# ---- the two stages -------------------------------------------------------------

def _run_pipeline(m, w, rand, **kw):
    d = _cuda(w.images)
    codes, keys, _ = m.build_codes(d)
    out, res, st = m.match_pairs_geometric(d, codes, keys, _cuda(w.kp), _cuda(w.scales), w.pairs, rand, **kw)
    return codes, keys, [o.cpu().numpy() for o in out], res, st


def test_geometric_pipeline_small_set(m):
    w = synth.geometric_set(cams_per_scene=12, n_feat=3000, n_points=30000, n_near=4, n_far=2)
    rand = _rand(256)
    _say(f"two-stage matching: {len(w.images)} images x 3000, {len(w.pairs)} pairs")
    codes, keys, got, res, st = _run_pipeline(m, w, rand)
    oc, ok = oracle.build_codes(w.images, *synth.projection_matrices())
    exp = G.geometric_match(w.images, oc, ok, w.kp, w.scales, w.pairs, rand)
    assert np.array_equal(res["status"], exp["status"])
    assert np.array_equal(res["n_matches"], exp["n_matches"])
    assert np.array_equal(res["n_inliers"], exp["n_inliers"])
    assert np.array_equal(res["F"], exp["F"])
    assert set(res["status"]) >= {G.ACCEPT, G.FEW_MATCHES}
    nq = np.array([w.images[q].shape[0] for q in w.pairs[:, 0]])
    off = np.concatenate([[0], np.cumsum(nq)])
    acc = exp["accepted"]
    aoff = np.concatenate([[0], np.cumsum(nq[acc])])
    for j, p in enumerate(acc):
        for g, e in zip(got, exp["stage2"]):
            assert np.array_equal(g[off[p]:off[p + 1]], e[aoff[j]:aoff[j + 1]]), p
    for p in np.flatnonzero(exp["status"] != G.ACCEPT):
        for g in got:
            assert np.all(g[off[p]:off[p + 1]] == -1)
    ms = m.last_geometric_ms()
    _say(f"stage times ms: subset {ms[0]:.3f}, stage 1 {ms[1]:.3f}, F {ms[2]:.3f}, stage 2 {ms[3]:.3f}")
    assert all(x > 0 for x in ms)
    # a second call on the same context gives the same outputs
    _, _, got2, res2, _ = _run_pipeline(m, w, rand)
    assert all(np.array_equal(a, b) for a, b in zip(got, got2))
    assert np.array_equal(res["F"], res2["F"])


def test_geometric_host_mode_is_refused():
    import ctypes as C
    mh = binding.Matcher(*synth.projection_matrices(), mem="host")
    s = np.zeros(10, np.float32)
    rows = np.zeros(2, np.int32)
    nf = np.array([10], np.int32)
    rc = binding.lib().cashash_select_top_scale(mh.h, 1, (C.c_void_p * 1)(s.ctypes.data), nf.ctypes.data, 1, 5,
                                                (C.c_void_p * 1)(rows.ctypes.data))
    assert rc == binding.E_INVAL
    assert "device" in binding.lib().cashash_last_error().decode()
