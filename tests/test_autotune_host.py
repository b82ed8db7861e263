"""The autotuner's cache lookup (host only, no GPU): the shipped entries
are found under the key dtb_autotune writes, and anything missing or
unreadable falls back to the library defaults."""
import json

from paper_2308_01241_amd import autotune


def test_shipped_entries_are_found():
    assert autotune.lookup(20_000_000, 2_000_000_000, 1, "f32", 20, arch="gfx950") == (868100, 0, 1, 2)
    assert autotune.lookup(20_000_000, 2_000_000_000, 1, "bf16", 20, arch="gfx950") == (781300, 0, 1, 2)
    assert autotune.lookup(14_673_808, 1_467_380_800, 64, "f32", 20, arch="gfx950") == (818900, 0, 1, 2)


def test_missing_shapes_and_files_fall_back_to_defaults(tmp_path):
    assert autotune.lookup(20_000_000, 2_000_000_000, 1, "f32", 19, arch="gfx950") == (0, 0, 0, 0)
    assert autotune.lookup(20_000_000, 2_000_000_000, 1, "f32", 20, arch="gfx942") == (0, 0, 0, 0)
    assert autotune.lookup(10, 100, path=str(tmp_path / "absent.json"), arch="gfx950") == (0, 0, 0, 0)
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert autotune.lookup(10, 100, path=str(bad), arch="gfx950") == (0, 0, 0, 0)


def test_key_format_and_older_entries(tmp_path):
    key = autotune.shape_key("gfx950", 1000, 20000, 2, "f32", 7)
    assert key == "gfx950|n=1000,nnz=20000,members=2,w=f32,D=7"
    db = tmp_path / "tuned.json"
    # an entry written before the fuse / events knobs existed
    db.write_text(json.dumps({key: {"bundle_syn": 65536, "unroll": 2}}))
    assert autotune.lookup(1000, 20000, 2, "f32", 7, path=str(db), arch="gfx950") == (65536, 2, 0, 0)
