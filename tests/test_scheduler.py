"""Host logic of host-memory matching: the block scheduler (paper, Three-Level
Data Scheduling Strategy, matching subsection).  No device is used."""
import numpy as np
import pytest

from paper_1805_08995_amd import binding, synth


def _check(img_bytes, pairs, slot):
    s = binding.plan_schedule(img_bytes, pairs, slot)
    order = s["order"]
    assert sorted(order.tolist()) == list(range(len(pairs)))  # every pair exactly once
    # block of each used image from the steps: blocks are consecutive used images under the slot size
    used = np.unique(pairs.reshape(-1)) if len(pairs) else np.array([], int)
    blocks, cur, fill = {}, 0, 0
    for m in used:
        if fill + img_bytes[m] > slot and fill > 0:
            cur, fill = cur + 1, 0
        blocks[int(m)] = cur
        fill += img_bytes[m]
    assert s["n_blocks"] == (cur + 1 if len(used) else 0)
    for m in used:  # each block fits a slot
        assert img_bytes[m] <= slot
    # steps: each step's pairs belong to its block pair; visiting order is (i,i+1..), then (i,i)
    seen_keys = []
    for bi, bk, b0, b1 in s["steps"]:
        assert bi <= bk and b1 > b0
        for p in order[b0:b1]:
            q, t = pairs[p]
            assert sorted((blocks[int(q)], blocks[int(t)])) == [bi, bk]
        seen_keys.append((bi, bk if bk != bi else 10**9))
    assert seen_keys == sorted(seen_keys)
    # residency: each step's blocks were loaded at least once; loads >= blocks touched
    assert s["block_loads"] >= s["n_blocks"]
    return s


def test_all_pairs_one_block():
    pairs = synth.exhaustive_pairs(20)
    s = _check(np.full(20, 100, np.int64), pairs, 10_000)
    assert s["n_blocks"] == 1 and s["n_steps"] == 1 and s["block_loads"] == 1 and s["image_loads"] == 20


@pytest.mark.parametrize("slot", [250, 400, 1000, 3000])
def test_exhaustive_many_blocks(slot):
    n = 30
    rng = np.random.default_rng(1)
    img_bytes = rng.integers(50, 250, n).astype(np.int64)
    pairs = synth.exhaustive_pairs(n)
    s = _check(img_bytes, pairs, slot)
    M = s["n_blocks"]
    # every block pair has pairs; a block's own step exists iff it holds >= 2 images
    sizes, fill, cur = [], 0, 0
    for b in img_bytes:
        if fill + b > slot and fill > 0:
            sizes.append(cur)
            fill, cur = 0, 0
        fill += b
        cur += 1
    sizes.append(cur)
    assert len(sizes) == M
    assert s["n_steps"] == M * (M - 1) // 2 + sum(1 for z in sizes if z >= 2)
    # paper order with three resident slots: block i is loaded once per row,
    # every later block once per row: loads = M + sum_i (M - 1 - i) at most
    assert s["block_loads"] <= M + M * (M - 1) // 2


def test_sparse_random_pairs_and_reverse_direction():
    rng = np.random.default_rng(2)
    n = 50
    img_bytes = rng.integers(10, 100, n).astype(np.int64)
    pairs = np.stack([rng.integers(0, n, 300), rng.integers(0, n, 300)], 1).astype(np.int32)
    _check(img_bytes, pairs, 400)
    _check(img_bytes, pairs[:, ::-1].copy(), 400)


def test_image_larger_than_slot():
    with pytest.raises(binding.CashashError) as e:
        binding.plan_schedule(np.array([10, 500], np.int64), np.array([[0, 1]], np.int32), 100)
    assert e.value.code == binding.E_NOMEM


def test_empty_and_bad_pairs():
    s = binding.plan_schedule(np.array([10, 20], np.int64), np.zeros((0, 2), np.int32), 100)
    assert s["n_steps"] == 0 and s["n_blocks"] == 0
    with pytest.raises(binding.CashashError) as e:
        binding.plan_schedule(np.array([10, 20], np.int64), np.array([[0, 2]], np.int32), 100)
    assert e.value.code == binding.E_INVAL
