"""The disk level's set file, written by the library (host code only, no
device): header, feature prefix sums, descriptors and keypoints where the
format puts them."""
import numpy as np

from paper_1805_08995_amd import binding


def test_set_file_layout(tmp_path):
    rng = np.random.default_rng(0)
    nf = [3, 0, 17, 1]
    imgs = [rng.integers(0, 256, (n, 128), dtype=np.uint8) for n in nf]
    kps = [rng.uniform(0, 100, (n, 2)).astype(np.float32) for n in nf]
    path = tmp_path / "s.chs"
    binding.set_write(path, imgs, kps)
    raw = path.read_bytes()
    assert raw[:8] == b"CASHSET1"
    hdr = np.frombuffer(raw, np.int64, count=2, offset=8)
    assert list(hdr) == [4, 1]
    offs = np.frombuffer(raw, np.int64, count=5, offset=24)
    assert list(offs) == [0, 3, 3, 20, 21]
    data = (24 + 8 * 5 + 63) // 64 * 64
    desc = np.frombuffer(raw, np.uint8, count=21 * 128, offset=data).reshape(21, 128)
    assert np.array_equal(desc, np.concatenate(imgs))
    kp = np.frombuffer(raw, np.float32, count=42, offset=data + 21 * 128).reshape(21, 2)
    assert np.array_equal(kp, np.concatenate(kps))
    assert len(raw) == data + 21 * 128 + 21 * 8


def test_set_file_without_keypoints_and_empty(tmp_path):
    path = tmp_path / "e.chs"
    binding.set_write(path, [np.zeros((0, 128), np.uint8)])
    raw = path.read_bytes()
    assert list(np.frombuffer(raw, np.int64, count=2, offset=8)) == [1, 0]
    assert len(raw) == 64


def test_set_write_refuses_bad_path(tmp_path):
    import pytest
    with pytest.raises(binding.CashashError) as e:
        binding.set_write(tmp_path / "no" / "such" / "dir.chs", [np.zeros((2, 128), np.uint8)])
    assert e.value.code == binding.E_IO
