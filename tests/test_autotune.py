"""Launch-geometry tuning on the CPU: the C ABI validates grouped kinds and
grids, and the tuning table keeps one entry per (device, precision, size
bucket) and applies the entry of the nearest bucket."""
import json

import pytest

from paper_2108_10209_amd import autotune, n2f


@pytest.fixture
def restore_grids():
    saved = [n2f.group_grid(k) for k in range(len(n2f.GROUP_KINDS))]
    yield saved
    for k, g in enumerate(saved):
        n2f.set_group_grid(k, g)


def test_group_grid_get_set_and_validation(restore_grids):
    assert len(n2f.GROUP_KINDS) == 15
    assert all(1 <= g <= n2f.MAX_GROUP_GRID for g in restore_grids)
    n2f.set_group_grid(5, 512)
    assert n2f.group_grid(5) == 512
    for kind, grid in [(-1, 256), (15, 256), (0, 0), (0, n2f.MAX_GROUP_GRID + 1)]:
        with pytest.raises(n2f.N2FError) as e:
            n2f.set_group_grid(kind, grid)
        assert e.value.code == n2f.EINVAL
    with pytest.raises(n2f.N2FError):
        n2f.group_grid(99)
    assert n2f.group_grid(5) == 512          # a refused call changes nothing


def test_size_bucket():
    assert autotune.size_bucket(640 * 640) == 19
    assert autotune.size_bucket(256 * 256) == 16
    assert autotune.size_bucket(1) == 0


def test_table_entries_and_nearest_bucket(tmp_path, restore_grids):
    path = str(tmp_path / "t.json")
    base = {"device": "dev A", "precision": "bf16", "images": 4, "mean_pixels": 0, "report": {}}
    autotune.save_entry(dict(base, bucket=16, group_grid={"conv3x3_wgrad": 128}), path)
    autotune.save_entry(dict(base, bucket=20, group_grid={"conv3x3_wgrad": 1024, "adam": 512}), path)
    autotune.save_entry(dict(base, bucket=20, group_grid={"conv3x3_wgrad": 768}), path)   # replaces
    autotune.save_entry(dict(base, device="dev B", bucket=20, group_grid={"conv3x3_wgrad": 384}), path)
    entries = json.load(open(path))["entries"]
    assert len(entries) == 3
    e = autotune.apply(2 ** 19.2, path, device="dev A")          # nearest bucket 20
    assert e["bucket"] == 20 and n2f.group_grid(5) == 768
    e = autotune.apply(2 ** 15, path, device="dev A")            # nearest bucket 16
    assert e["bucket"] == 16 and n2f.group_grid(5) == 128
    assert autotune.apply(2 ** 18, path, device="dev C") is None
    assert n2f.group_grid(5) == 128                              # no entry: grids unchanged
    assert autotune.apply(2 ** 18, str(tmp_path / "missing.json"), device="dev A") is None


def test_committed_table_is_well_formed():
    for e in autotune.load_table():
        assert {"device", "precision", "bucket", "group_grid"} <= set(e)
        for name, g in e["group_grid"].items():
            assert name in n2f.GROUP_KINDS and 1 <= int(g) <= n2f.MAX_GROUP_GRID
