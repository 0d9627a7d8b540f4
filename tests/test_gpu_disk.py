"""Disk level of the data scheduling on the GPU: codes and matches streamed
from a set file in groups equal the oracle's bit for bit, an interrupted
matching run resumes from its progress file, and a change of matching
configuration or of the codes file invalidates that progress."""
import numpy as np
import pytest

import oracle
from paper_1805_08995_amd import binding, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def workload(tmp_path_factory):
    rng = np.random.default_rng(21)
    w = synth.scene_set(n_images=24, n_feat=1500)
    imgs = list(w.images)
    imgs[3] = imgs[3][:0]            # an empty image
    imgs[7] = imgs[7][:37]           # a short one
    pairs = np.array([(i, j) for i in range(24) for j in range(24) if i != j and rng.random() < 0.35]
                     + [(5, 5), (7, 3), (3, 7), (2, 9), (2, 9)], np.int32)
    d = tmp_path_factory.mktemp("disk")
    set_path = d / "set.chs"
    binding.set_write(set_path, imgs)
    mats = synth.projection_matrices()
    # expected values: the CPU oracle
    oc, ok = oracle.build_codes(imgs, *mats)
    ref_codes = np.concatenate(oc)
    ref_keys = np.concatenate(ok)
    ref = list(oracle.match_pairs(imgs, oc, ok, pairs, k=10))
    ref_tau = list(oracle.match_pairs(imgs, oc, ok, pairs, k=10, tau=44))
    return dict(imgs=imgs, pairs=pairs, dir=d, set=set_path, mats=mats, ref_codes=ref_codes, ref_keys=ref_keys,
                ref=ref, ref_tau=ref_tau)


def _host_matcher(w, device_budget=6 << 20):
    return binding.Matcher(*w["mats"], mem="host", device_budget_bytes=device_budget)


def test_codes_from_disk_equal_in_memory(workload):
    w = workload
    m = _host_matcher(w)
    path = w["dir"] / "codes.chc"
    nbytes = sum(im.size for im in w["imgs"])
    st = m.build_codes_disk(w["set"], path, host_budget_bytes=2 * 600_000)
    _say(f"codes from disk: {st['group_loads']} group loads, {st['disk_bytes']} bytes read")
    codes, keys = binding.read_codes_file(path)
    assert np.array_equal(codes, w["ref_codes"]) and np.array_equal(keys, w["ref_keys"])
    assert st["group_loads"] >= 2 * 5 and st["disk_bytes"] == 2 * nbytes


def test_matches_from_disk_equal_in_memory_and_resume(workload):
    w = workload
    m = _host_matcher(w)
    codes_path = w["dir"] / "codes2.chc"
    m.build_codes_disk(w["set"], codes_path, host_budget_bytes=1 << 30)
    out_path, prog = w["dir"] / "out.cho", w["dir"] / "out.prog"
    budget = 3 * 700_000
    # interrupted after two group pairs, then resumed
    left, st1 = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog, max_steps=2)
    _say(f"first call: {st1['pairs']} pairs, {left} group pairs left")
    assert left > 0 and st1["pairs"] > 0
    left2, st2 = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    _say(f"resumed: {st2['pairs']} pairs, {st2['group_loads']} group loads, {st2['disk_bytes']} bytes read")
    assert left2 == 0
    assert st1["pairs"] + st2["pairs"] == len(w["pairs"])
    got = binding.read_output_file(out_path)
    for g, r in zip(got, w["ref"]):
        assert np.array_equal(g, r)
    # nothing left: no group is read again
    left3, st3 = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left3 == 0 and st3["pairs"] == 0 and st3["disk_bytes"] == 0


def test_stale_progress_is_reset(workload):
    w = workload
    m = _host_matcher(w)
    codes_path = w["dir"] / "codes3.chc"
    m.build_codes_disk(w["set"], codes_path, host_budget_bytes=1 << 30)
    out_path, prog = w["dir"] / "out3.cho", w["dir"] / "out3.prog"
    budget = 3 * 700_000
    m.match_pairs_disk(w["set"], codes_path, w["pairs"][:40], out_path, budget, prog)
    # a different pair list: the old progress must not be trusted
    left, st = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left == 0 and st["pairs"] == len(w["pairs"])
    for g, r in zip(binding.read_output_file(out_path), w["ref"]):
        assert np.array_equal(g, r)
    # without a progress file, in one call
    out4 = w["dir"] / "out4.cho"
    left, st = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out4, budget)
    assert left == 0
    for g, r in zip(binding.read_output_file(out4), w["ref"]):
        assert np.array_equal(g, r)


def test_disk_errors(workload, tmp_path):
    w = workload
    m = _host_matcher(w)
    with pytest.raises(binding.CashashError) as e:
        m.build_codes_disk(tmp_path / "missing.chs", tmp_path / "c.chc", 1 << 20)
    assert e.value.code == binding.E_IO
    with pytest.raises(binding.CashashError) as e:
        m.match_pairs_disk(w["set"], w["set"], w["pairs"], tmp_path / "o.cho", 1 << 20)
    assert e.value.code == binding.E_IO       # not a codes file
    md = binding.Matcher(*w["mats"], mem="device")
    with pytest.raises(binding.CashashError) as e:
        md.build_codes_disk(w["set"], tmp_path / "c.chc", 1 << 20)
    assert e.value.code == binding.E_INVAL
    with pytest.raises(binding.CashashError) as e:
        m.build_codes_disk(w["set"], tmp_path / "c2.chc", 1000)   # an image alone exceeds a group
    assert e.value.code == binding.E_NOMEM


def test_resume_progress_tied_to_config_and_codes(workload):
    """Progress of a finished run is not reused by a run with another Hamming
    threshold (every pair is matched again, and the outputs are the oracle's
    for that threshold), nor after the codes file is written again."""
    w = workload
    m = _host_matcher(w)
    codes_path = w["dir"] / "codes5.chc"
    m.build_codes_disk(w["set"], codes_path, host_budget_bytes=1 << 30)
    out_path, prog = w["dir"] / "out5.cho", w["dir"] / "out5.prog"
    budget = 3 * 700_000
    left, st = m.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left == 0 and st["pairs"] == len(w["pairs"])
    mt = binding.Matcher(*w["mats"], mem="host", device_budget_bytes=6 << 20, max_hamming=44)
    left, st = mt.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left == 0 and st["pairs"] == len(w["pairs"])
    for g, r in zip(binding.read_output_file(out_path), w["ref_tau"]):
        assert np.array_equal(g, r)
    # same config as the last run: nothing to do
    left, st = mt.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left == 0 and st["pairs"] == 0
    # the codes file written again: progress is stale
    mt.build_codes_disk(w["set"], codes_path, host_budget_bytes=1 << 30)
    left, st = mt.match_pairs_disk(w["set"], codes_path, w["pairs"], out_path, budget, prog)
    assert left == 0 and st["pairs"] == len(w["pairs"])
    for g, r in zip(binding.read_output_file(out_path), w["ref_tau"]):
        assert np.array_equal(g, r)
